// Batched explicit steps: several independent simulations advanced by one
// launch per step of the streamed tile kernel (their tiles numbered one after
// the other), with the chunk of steps captured once in a hipGraph and
// replayed.  The per-simulation state at the start of a chunk (step count,
// record buffer, half-step flag, steps to take, dt) travels in a small
// descriptor array uploaded before the graph runs, so the graph itself never
// changes while the same simulations are batched.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pd_kernels.hpp"

using namespace pdk;

struct pd_batch_s {
    pd_ctx ctx = nullptr;
    StreamInst *dev = nullptr;      // descriptors, capacity cap
    StreamInst *host = nullptr;     // pinned staging of the descriptors
    int cap = 0;
    hipEvent_t uploaded = nullptr;  // the staging buffer may be rewritten after this
    bool pending = false;
    hipStream_t capture = nullptr;  // graphs are captured here, launched on ctx->stream
    hipGraphExec_t exec = nullptr;
    // what the captured graph was built for
    int g_ninst = 0, g_dim = 0, g_lanes = 0, g_block = 0;
    int g_prec = -1;
    bool g_np = false;
    uint32_t g_ntiles = 0, g_tile = 0, g_hcap = 0, g_bcap = 0, g_mmax = 0;
    unsigned g_grid = 0;
    size_t g_lds = 0;
    int64_t g_steps = 0;
};

static void batch_free_graph(pd_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

extern "C" int pd_batch_create(pd_ctx ctx, pd_batch *out) {
    if (!out) return pd_set_error(ctx, PD_EINVAL, "out must not be NULL");
    *out = nullptr;
    PD_TRY(pd_check_ctx(ctx));
    pd_batch b = new (std::nothrow) pd_batch_s();
    if (!b) return PD_ENOMEM;
    b->ctx = ctx;
    ctx->refs += 1;
    int st = PD_OK;
    if (hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess)
        st = pd_set_error(ctx, PD_EDEVICE, "hipEventCreate failed");
    if (st == PD_OK && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
        st = pd_set_error(ctx, PD_EDEVICE, "hipStreamCreate failed");
    if (st != PD_OK) {
        pd_batch_destroy(b);
        return st;
    }
    *out = b;
    return PD_OK;
}

extern "C" int pd_batch_destroy(pd_batch b) {
    if (!b) return PD_EINVAL;
    pd_ctx ctx = b->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    batch_free_graph(b);
    pd_free(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    pd_ctx_unref(ctx);
    return PD_OK;
}

// the launches of one chunk: nsteps step kernels, the k-th told it is step k
static int batch_enqueue(pd_batch b, hipStream_t st, int dim, StreamArgs sa, int lanes,
                         int prec, bool np, int block, unsigned grid, size_t lds,
                         int64_t nsteps) {
    for (int64_t k = 0; k < nsteps; ++k) {
        sa.step = k;
        PD_TRY(pd_launch_stream(b->ctx, st, dim, sa, lanes, prec, np ? SK_NP : SK_LINEAR, block,
                                grid, lds));
    }
    return PD_OK;
}

extern "C" int pd_batch_step(pd_batch b, pd_sim *sims, int nsims, const int64_t *steps,
                             const double *dt, int64_t nsteps, int use_graph) {
    if (!b) return PD_EINVAL;
    pd_ctx ctx = b->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (nsims < 1 || !sims || !steps || !dt)
        return pd_set_error(ctx, PD_EINVAL, "need nsims >= 1 and the sims, steps and dt arrays");
    if (nsteps < 0) return pd_set_error(ctx, PD_EINVAL, "nsteps must be >= 0");
    const pd_sim s0 = sims[0];
    if (!s0) return pd_set_error(ctx, PD_EINVAL, "sims[0] is NULL");
    const int dim = s0->nbr->dim, lanes = s0->lanes;
    const int prec = s0->mat.precision;
    const bool np = s0->mat.law == PD_LAW_NP;
    const uint32_t tile = s0->nbr->tile_T;
    uint64_t ntiles = 0;
    uint32_t hcap = 0, bcap = 0;
    for (int k = 0; k < nsims; ++k) {
        const pd_sim s = sims[k];
        if (!s || s->ctx != ctx) return pd_set_error(ctx, PD_EINVAL, "sims[%d]: NULL or another context", k);
        if (!s->stream)
            return pd_set_error(ctx, PD_EINVAL, "sims[%d] does not run the streamed kernel", k);
        if (s->s_form == SK_LPS_FORCE)
            return pd_set_error(ctx, PD_EINVAL, "sims[%d]: the solid steps alone", k);
        if (s->nbr->dim != dim || s->lanes != lanes || s->nbr->tile_T != tile ||
            s->mat.precision != prec || (s->mat.law == PD_LAW_NP) != np)
            return pd_set_error(ctx, PD_EINVAL,
                                "sims[%d]: dim, lanes, tile size, precision and law must match",
                                k);
        for (int j = 0; j < k; ++j)
            if (sims[j] == s) return pd_set_error(ctx, PD_EINVAL, "sims[%d] is listed twice", k);
        if (steps[k] < 0 || steps[k] > nsteps)
            return pd_set_error(ctx, PD_EINVAL, "steps[%d] must be in [0, nsteps]", k);
        if (!(dt[k] > 0.0) || !std::isfinite(dt[k]))
            return pd_set_error(ctx, PD_EINVAL, "dt[%d] must be > 0", k);
        if (s->v_half && steps[k] > 0 && dt[k] != s->last_dt)
            return pd_set_error(ctx, PD_EINVAL,
                                "sims[%d]: dt changed mid-trajectory (read the state first)", k);
        ntiles += s->nbr->ntiles;
        hcap = std::max(hcap, pd_tile_hcap(s->nbr));
        bcap = std::max(bcap, pd_tile_bcap(s->nbr));
    }
    if (ntiles >= (1ull << 31)) return pd_set_error(ctx, PD_ECAPACITY, "too many tiles");
    if (nsteps == 0) return PD_OK;
    int block = 0;
    unsigned grid = 0;
    uint32_t mmax = 0;
    size_t lds = 0;
    if (!pd_stream_geometry(ctx, dim, (uint32_t)ntiles, tile, hcap, bcap, lanes, prec, true,
                            np ? SK_NP : SK_LINEAR, &block, &grid, &mmax, &lds))
        return pd_set_error(ctx, PD_ECAPACITY, "the batch does not fit the streamed kernel");

    // descriptors: previous upload done, then stage and upload
    if (nsims > b->cap) {
        if (b->pending) (void)hipEventSynchronize(b->uploaded);
        b->pending = false;
        batch_free_graph(b);          // the graph points at the old array
        pd_free(b->dev);
        b->dev = nullptr;
        if (b->host) (void)hipHostFree(b->host);
        b->host = nullptr;
        b->cap = 0;
        int cap = 16;
        while (cap < nsims) cap *= 2;
        PD_TRY(pd_alloc(ctx, &b->dev, (size_t)cap));
        if (hipHostMalloc((void **)&b->host, sizeof(StreamInst) * cap) != hipSuccess) {
            (void)hipGetLastError();
            return pd_set_error(ctx, PD_ENOMEM, "pinned descriptor buffer");
        }
        b->cap = cap;
    }
    if (b->pending) PD_HIP(ctx, hipEventSynchronize(b->uploaded));
    uint32_t begin = 0;
    for (int k = 0; k < nsims; ++k) {
        const pd_sim s = sims[k];
        if (steps[k] > 0 && s->rec_stale) {
            PD_TRY(pd_rec_pack(ctx, dim, s->nbr->n, s->xv, s->u[s->cur], s->rec[s->cur]));
            s->rec_stale = false;
        }
        StreamInst d = pd_stream_inst(s);
        d.tile_begin = begin;
        d.dt = dt[k];
        d.cur0 = s->cur;
        d.vhalf0 = s->v_half ? 1 : 0;
        d.step0 = s->step;
        d.limit = steps[k];
        b->host[k] = d;
        begin += s->nbr->ntiles;
    }
    PD_HIP(ctx, hipMemcpyAsync(b->dev, b->host, sizeof(StreamInst) * nsims,
                               hipMemcpyHostToDevice, ctx->stream));
    PD_HIP(ctx, hipEventRecord(b->uploaded, ctx->stream));
    b->pending = true;

    StreamArgs sa = pd_stream_args(s0, b->dev, (uint32_t)nsims, (uint32_t)ntiles);
    sa.hcap = hcap;
    sa.bcap = bcap;
    sa.mmax = mmax;
    if (!use_graph) {
        PD_TRY(batch_enqueue(b, ctx->stream, dim, sa, lanes, prec, np, block, grid, lds,
                             nsteps));
    } else {
        const bool same = b->exec && b->g_ninst == nsims && b->g_dim == dim &&
                          b->g_lanes == lanes && b->g_block == block && b->g_prec == prec &&
                          b->g_np == np &&
                          b->g_ntiles == (uint32_t)ntiles && b->g_tile == tile &&
                          b->g_hcap == hcap && b->g_bcap == bcap && b->g_mmax == mmax &&
                          b->g_grid == grid && b->g_lds == lds && b->g_steps == nsteps;
        if (!same) {
            batch_free_graph(b);
            hipGraph_t graph = nullptr;
            PD_HIP(ctx, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
            const int st = batch_enqueue(b, b->capture, dim, sa, lanes, prec, np, block, grid,
                                         lds, nsteps);
            const hipError_t e = hipStreamEndCapture(b->capture, &graph);
            if (st != PD_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return pd_hip_error(ctx, e, "capture", __FILE__, __LINE__);
            const hipError_t e2 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) {
                b->exec = nullptr;
                return pd_hip_error(ctx, e2, "hipGraphInstantiate", __FILE__, __LINE__);
            }
            b->g_ninst = nsims;
            b->g_dim = dim;
            b->g_lanes = lanes;
            b->g_block = block;
            b->g_prec = prec;
            b->g_np = np;
            b->g_ntiles = (uint32_t)ntiles;
            b->g_tile = tile;
            b->g_hcap = hcap;
            b->g_bcap = bcap;
            b->g_mmax = mmax;
            b->g_grid = grid;
            b->g_lds = lds;
            b->g_steps = nsteps;
        }
        PD_HIP(ctx, hipGraphLaunch(b->exec, ctx->stream));
    }
    for (int k = 0; k < nsims; ++k) pd_sim_advanced(sims[k], steps[k], dt[k]);
    return PD_OK;
}
