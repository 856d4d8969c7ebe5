// Autotuner for the explicit step: times the tile sizes and lane counts the
// tiled kernels support on a given mesh and keeps the fastest per (dimension,
// neighbour-count bucket, precision) in the context.  pd_sim_create then uses
// the cached choice for every mesh of that bucket while the context's tuning
// is automatic.  The measurement is the step itself (pd_verlet_step on a
// simulation built from the mesh, timed with HIP events on the context's
// stream), so it includes whichever kernel the automatic choice runs for that
// shape (streamed tiles for equal volumes, LDS tiles otherwise).
#include <algorithm>
#include <cmath>

#include "pd_internal.hpp"

namespace {

// tile sizes x lanes per node with T * lanes in [256, 1024] threads: the
// shapes the tile kernels are built for (one lane group per tile node); the
// large 4-lane tiles (192, 240) cut the per-node work per bond of 3-d meshes
constexpr int CAND[][2] = {{32, 8},  {32, 16}, {64, 4},  {64, 8},  {64, 16}, {128, 2},
                           {128, 4}, {128, 8}, {192, 4}, {240, 4}, {256, 2}, {256, 4}};
constexpr int NCAND = (int)(sizeof(CAND) / sizeof(CAND[0]));

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// the context's tuning, restored when the search ends
struct SavedTuning {
    pd_ctx ctx;
    int lanes, kernel, tile, block;
    explicit SavedTuning(pd_ctx c)
        : ctx(c), lanes(c->lanes), kernel(c->kernel), tile(c->tile), block(c->block) {}
    ~SavedTuning() {
        ctx->lanes = lanes;
        ctx->kernel = kernel;
        ctx->tile = tile;
        ctx->block = block;
    }
};

int store(pd_ctx ctx, int dim, int bucket, int precision, int tile, int lanes, double us) {
    for (pd_tune_entry &e : ctx->tuned)
        if (e.dim == dim && e.bucket == bucket && e.precision == precision) {
            e.tile = tile;
            e.lanes = lanes;
            e.us = us;
            return PD_OK;
        }
    pd_tune_entry e;
    e.dim = dim;
    e.bucket = bucket;
    e.precision = precision;
    e.tile = tile;
    e.lanes = lanes;
    e.us = us;
    ctx->tuned.push_back(e);
    return PD_OK;
}

int hip_ok(pd_ctx ctx, hipError_t e, const char *what) {
    return e == hipSuccess ? PD_OK : pd_hip_error(ctx, e, what, __FILE__, __LINE__);
}

bool valid_choice(int tile, int lanes) {
    for (int k = 0; k < NCAND; ++k)
        if (CAND[k][0] == tile && CAND[k][1] == lanes) return true;
    return false;
}

}  // namespace

// buckets of the mean neighbour count with edges between the counts of the
// common lattice horizons, so that a horizon's meshes share a bucket whatever
// their size (edge nodes lower the mean by up to ~15 %): 2-d 2h/3h/4h/5h
// have 12/28/48/80 neighbours inside the mesh, 3-d 2h/3h/4h 32/122/256
int pd_tune_bucket(double k) {
    constexpr double EDGES[] = {8, 20, 36, 64, 96, 176, 384, 768};
    int b = 0;
    for (double e : EDGES) b += k >= e ? 1 : 0;
    return b;
}

const pd_tune_entry *pd_tune_find(pd_ctx ctx, int dim, double k, int precision) {
    const int b = pd_tune_bucket(k);
    for (const pd_tune_entry &e : ctx->tuned)
        if (e.dim == dim && e.bucket == b && e.precision == precision) return &e;
    return nullptr;
}

extern "C" int pd_autotune(pd_ctx ctx, int dim, int64_t n, const double *X, const double *V,
                           double delta, int precision, int steps, pd_tune_result *table,
                           int table_cap, int *ntable, pd_tune_result *best) {
    PD_TRY(pd_check_ctx(ctx));
    if (ntable) *ntable = 0;
    if (precision != PD_FP64 && precision != PD_MIXED && precision != PD_FP32)
        return pd_set_error(ctx, PD_EINVAL, "precision must be PD_FP64, PD_MIXED or PD_FP32");
    if (steps < 1 || steps > 100000) return pd_set_error(ctx, PD_EINVAL, "steps must be in [1, 1e5]");
    if (table_cap < 0 || (table_cap > 0 && !table))
        return pd_set_error(ctx, PD_EINVAL, "table must hold table_cap entries");
    if (!V) return pd_set_error(ctx, PD_EINVAL, "V must not be NULL");
    PD_TRY(pd_check_dev_ptr(ctx, V, "V"));
    pd_nbr nbr = nullptr;
    PD_TRY(pd_build_neighbors(ctx, dim, n, X, delta, &nbr));
    const double k = (double)nbr->nnz / (double)nbr->n;
    pd_material mat{};
    mat.dim = dim;
    mat.c = pd_micromodulus(dim, 1.0, delta);
    mat.rho = 1.0;
    mat.s_c = 1e-3;                   // damage test on, as in the fracture workloads
    mat.precision = precision;
    const double dt = 0.1 * delta / 3.0;
    Events ev;
    int st = PD_OK;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
        st = pd_set_error(ctx, PD_EDEVICE, "hipEventCreate failed");
    pd_tune_result top{};
    top.us_per_step = -1.0;
    int rows = 0;
    {
        SavedTuning saved(ctx);
        for (int c = 0; c < NCAND && st == PD_OK; ++c) {
            pd_tune_result r{};
            r.tile = CAND[c][0];
            r.lanes = CAND[c][1];
            r.us_per_step = -1.0;
            ctx->lanes = r.lanes;
            ctx->kernel = 0;
            ctx->tile = r.tile;
            ctx->block = 0;
            pd_sim sim = nullptr;
            const int cs = pd_sim_create(ctx, nbr, &mat, X, V, nullptr, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, 0, 0, &sim);
            if (cs == PD_OK && sim->tiled && (int)nbr->tile_T == r.tile) {
                r.kernel = sim->stream ? 3 : 2;
                st = pd_verlet_step(sim, 2, dt);                       // warm-up
                if (st == PD_OK) st = hip_ok(ctx, hipEventRecord(ev.a, ctx->stream), "event");
                if (st == PD_OK) st = pd_verlet_step(sim, steps, dt);
                if (st == PD_OK) st = hip_ok(ctx, hipEventRecord(ev.b, ctx->stream), "event");
                if (st == PD_OK) st = hip_ok(ctx, hipEventSynchronize(ev.b), "event sync");
                float ms = 0.f;
                if (st == PD_OK) st = hip_ok(ctx, hipEventElapsedTime(&ms, ev.a, ev.b), "event time");
                if (st == PD_OK) r.us_per_step = 1e3 * (double)ms / steps;
            } else if (cs == PD_EDEVICE) {
                st = cs;
            } else if (cs == PD_OK) {
                r.kernel = 1;                 // the tile size does not fit: not a candidate
            }
            if (sim) {
                const int ds = pd_sim_destroy(sim);
                if (st == PD_OK && ds != PD_OK) st = ds;
            }
            if (rows < table_cap) table[rows] = r;
            rows += 1;
            if (r.us_per_step > 0 && (top.us_per_step < 0 || r.us_per_step < top.us_per_step))
                top = r;
        }
    }
    pd_nbr_destroy(nbr);
    if (st != PD_OK) return st;
    if (ntable) *ntable = std::min(rows, table_cap);
    if (top.us_per_step < 0)
        return pd_set_error(ctx, PD_ECAPACITY, "no tile size fits this mesh");
    PD_TRY(store(ctx, dim, pd_tune_bucket(k), precision, top.tile, top.lanes, top.us_per_step));
    if (best) *best = top;
    return PD_OK;
}

extern "C" int pd_tune_lookup(pd_ctx ctx, int dim, double mean_neighbors, int precision,
                              pd_tune_result *out) {
    if (!ctx || !out) return PD_EINVAL;
    *out = pd_tune_result{};
    const pd_tune_entry *e = pd_tune_find(ctx, dim, mean_neighbors, precision);
    if (e) {
        out->tile = e->tile;
        out->lanes = e->lanes;
        out->us_per_step = e->us;
    }
    return PD_OK;
}

extern "C" int pd_tune_set(pd_ctx ctx, int dim, double mean_neighbors, int precision, int tile,
                           int lanes) {
    if (!ctx) return PD_EINVAL;
    if (dim != 2 && dim != 3) return pd_set_error(ctx, PD_EINVAL, "dim must be 2 or 3");
    if (precision != PD_FP64 && precision != PD_MIXED && precision != PD_FP32)
        return pd_set_error(ctx, PD_EINVAL, "precision must be PD_FP64, PD_MIXED or PD_FP32");
    if (!(mean_neighbors > 0) || !std::isfinite(mean_neighbors))
        return pd_set_error(ctx, PD_EINVAL, "mean_neighbors must be > 0");
    if (!valid_choice(tile, lanes))
        return pd_set_error(ctx, PD_EINVAL, "(tile %d, lanes %d) is not a tuner candidate", tile,
                            lanes);
    return store(ctx, dim, pd_tune_bucket(mean_neighbors), precision, tile, lanes, 0.0);
}

extern "C" int pd_tune_clear(pd_ctx ctx) {
    if (!ctx) return PD_EINVAL;
    ctx->tuned.clear();
    return PD_OK;
}
