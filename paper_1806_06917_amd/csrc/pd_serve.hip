// Serving: independent explicit simulations submitted as requests, admitted
// in arrival order while their device memory fits a budget, advanced
// together (continuous batching: one batched launch per step covers every
// running simulation of a launch group -- same dimension, lane count, tile
// size, precision and law -- and simulations that arrive while others run join at
// the next chunk), retired as soon as they reach their step count.
//
// Host code only; the GPU work is pd_build_neighbors, pd_sim_create and
// pd_batch_step.  Timestamps come from a monotonic clock
// (pd_server_clock), so callers can replay arrival schedules against it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <vector>

#include "pd_kernels.hpp"

namespace {

struct Req {
    int64_t id = 0;
    pd_request_info info{};
    // host copies of the request's arrays
    int dim = 2;
    int64_t n = 0;
    std::vector<double> X, V, u0, v0, bc_vel, notch;
    std::vector<uint8_t> bc_kind;
    int nseg = 0;
    double delta = 0, dt = 0;
    pd_material mat{};
    int64_t nsteps = 0, ramp = 0, done = 0;
    int keep = 0;
    int64_t estimate = 0;
    // device state while running
    pd_nbr nbr = nullptr;
    pd_sim sim = nullptr;
    std::vector<double> u_out, v_out;
};

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// device bytes of a simulation and its neighbour list, from the sizes the
// library allocates (tiles and records included)
int64_t footprint(int dim, int64_t n, int64_t nnz, int64_t halo_total, int64_t ntiles,
                  bool bc_vel, bool lps) {
    const int64_t us = dim == 3 ? 4 : 2, rd = dim == 3 ? 6 : 4;
    const int64_t nbr = 16 * n + 8 + 10 * nnz + 4 * halo_total + 8 * ntiles + 8;
    const int64_t sim = 32 * n + 3 * 8 * us * n + (n + 16) + nnz + 16 * n +
                        (bc_vel ? 8 * us * n : 0) + 2 * nnz + 4 + 2 * 8 * rd * n +
                        (lps ? 48 * n : 0);   // the solid's {m, theta} and coefficients
    return nbr + sim;
}

// the same before the neighbour list exists: bonds from the horizon volume
// over the mean nodal volume, halo ids from a typical halo-to-tile ratio
int64_t estimate(const Req &r) {
    double vmean = 0;
    for (double x : r.V) vmean += x;
    vmean = r.n ? vmean / (double)r.n : 1.0;
    const double pi = 3.14159265358979323846;
    const double ball = r.dim == 3 ? 4.0 / 3.0 * pi * r.delta * r.delta * r.delta
                                   : pi * r.delta * r.delta;
    const double k = vmean > 0 ? ball / vmean : 0.0;
    const int64_t nnz = (int64_t)(k * (double)r.n) + r.n;
    const int64_t tile = 128, ratio = r.dim == 3 ? 12 : 5;
    return footprint(r.dim, r.n, nnz, ratio * r.n, r.n / tile + 1, !r.bc_vel.empty(),
                     r.mat.law == PD_LAW_LPS);
}

}  // namespace

// simulations that can share one streamed launch: dim, lanes, tile size,
// precision, law
using GroupKey = std::tuple<int, int, uint32_t, int, int>;

struct Group {
    pd_batch batch = nullptr;
    // shape of the previous chunk (graph reuse when unchanged)
    std::vector<pd_sim> last_sims;
    int64_t last_nsteps = -1;
};

struct pd_server_s {
    pd_ctx ctx = nullptr;
    // requests admitted while a chunk runs are built on a context of their
    // own (its own stream, reduction and status buffers), then moved to ctx
    pd_ctx actx = nullptr;
    hipStream_t astream = nullptr;
    int64_t budget = 0, used = 0, peak = 0;
    int64_t chunk = 100;
    int lanes = 0;
    int64_t next_id = 1;
    std::deque<Req *> queue;          // arrival order
    std::vector<Req *> running;
    std::map<int64_t, Req *> all;
    std::map<GroupKey, Group> groups;
    pd_server_stats stats{};
};

extern "C" double pd_server_clock(void) { return now_s(); }

extern "C" int pd_server_create(pd_ctx ctx, int64_t hbm_budget, int64_t chunk_steps, int lanes,
                                pd_server *out) {
    if (!out) return pd_set_error(ctx, PD_EINVAL, "out must not be NULL");
    *out = nullptr;
    PD_TRY(pd_check_ctx(ctx));
    if (hbm_budget <= 0) return pd_set_error(ctx, PD_EINVAL, "hbm_budget must be positive");
    if (chunk_steps < 1) return pd_set_error(ctx, PD_EINVAL, "chunk_steps must be >= 1");
    if (lanes != 0 && (lanes < 2 || lanes > 32 || (lanes & (lanes - 1))))
        return pd_set_error(ctx, PD_EINVAL, "lanes must be 0 or a power of two in [2, 32]");
    pd_server s = new (std::nothrow) pd_server_s();
    if (!s) return PD_ENOMEM;
    s->ctx = ctx;
    ctx->refs += 1;
    s->budget = hbm_budget;
    s->chunk = chunk_steps;
    s->lanes = lanes;
    // without a second stream admission simply runs between chunks
    if (hipStreamCreateWithFlags(&s->astream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        s->astream = nullptr;
    } else if (pd_ctx_create(ctx->device, (void *)s->astream, &s->actx) != PD_OK) {
        s->actx = nullptr;
        (void)hipStreamDestroy(s->astream);
        s->astream = nullptr;
    }
    *out = s;
    return PD_OK;
}

static void release_device(pd_server s, Req *r) {
    if (r->sim) pd_sim_destroy(r->sim);
    if (r->nbr) pd_nbr_destroy(r->nbr);
    r->sim = nullptr;
    r->nbr = nullptr;
    s->used -= r->info.bytes;
}

extern "C" int pd_server_destroy(pd_server s) {
    if (!s) return PD_EINVAL;
    pd_ctx ctx = s->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (Req *r : s->running) release_device(s, r);
    for (auto &kv : s->all) delete kv.second;
    for (auto &kv : s->groups) pd_batch_destroy(kv.second.batch);
    if (s->actx) pd_ctx_destroy(s->actx);
    if (s->astream) (void)hipStreamDestroy(s->astream);
    delete s;
    pd_ctx_unref(ctx);
    return PD_OK;
}

extern "C" int pd_server_submit(pd_server s, const pd_request *q, int64_t *id) {
    if (!s) return PD_EINVAL;
    pd_ctx ctx = s->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (!q || !id) return pd_set_error(ctx, PD_EINVAL, "request and id must not be NULL");
    if (q->dim != 2 && q->dim != 3) return pd_set_error(ctx, PD_EINVAL, "dim must be 2 or 3");
    if (q->n <= 0 || !q->X || !q->V) return pd_set_error(ctx, PD_EINVAL, "need n > 0, X and V");
    if (q->bc_kind && !q->bc_vel)
        return pd_set_error(ctx, PD_EINVAL, "bc_vel is required with bc_kind");
    if (q->nseg < 0 || q->nseg > 8 || (q->nseg > 0 && !q->notch))
        return pd_set_error(ctx, PD_EINVAL, "nseg must be in [0, 8] with a notch array");
    if (q->nsteps < 0) return pd_set_error(ctx, PD_EINVAL, "nsteps must be >= 0");
    if (!(q->dt > 0.0) || !std::isfinite(q->dt))
        return pd_set_error(ctx, PD_EINVAL, "dt must be > 0");
    if (q->mat.dim != q->dim) return pd_set_error(ctx, PD_EINVAL, "material dim != dim");
    Req *r = new (std::nothrow) Req();
    if (!r) return PD_ENOMEM;
    const size_t nd = (size_t)q->n * q->dim;
    r->id = s->next_id++;
    r->dim = q->dim;
    r->n = q->n;
    r->X.assign(q->X, q->X + nd);
    r->V.assign(q->V, q->V + q->n);
    if (q->u0) r->u0.assign(q->u0, q->u0 + nd);
    if (q->v0) r->v0.assign(q->v0, q->v0 + nd);
    if (q->bc_kind) {
        r->bc_kind.assign(q->bc_kind, q->bc_kind + q->n);
        r->bc_vel.assign(q->bc_vel, q->bc_vel + nd);
    }
    if (q->nseg > 0) r->notch.assign(q->notch, q->notch + 4 * q->nseg);
    r->nseg = q->nseg;
    r->delta = q->delta;
    r->dt = q->dt;
    r->mat = q->mat;
    r->nsteps = q->nsteps;
    r->ramp = q->ramp_steps;
    r->keep = q->keep_state;
    r->estimate = estimate(*r);
    r->info.id = r->id;
    r->info.state = PD_REQ_QUEUED;
    r->info.t_submit = q->t_arrival > 0 ? q->t_arrival : now_s();
    r->info.status = PD_OK;
    s->all[r->id] = r;
    s->queue.push_back(r);
    *id = r->id;
    return PD_OK;
}

// builds the request's neighbour list and simulation on the device, on
// context bctx (the server's own or its admission context; the simulation
// ends up on the server's)
static int admit(pd_server s, Req *r, pd_ctx bctx) {
    pd_ctx ctx = bctx;
    const size_t n = (size_t)r->n, nd = n * r->dim;
    double *X = nullptr, *V = nullptr, *u0 = nullptr, *v0 = nullptr, *bv = nullptr;
    uint8_t *bk = nullptr;
    int st = pd_alloc(ctx, &X, nd);
    if (st == PD_OK) st = pd_alloc(ctx, &V, n);
    if (st == PD_OK && !r->u0.empty()) st = pd_alloc(ctx, &u0, nd);
    if (st == PD_OK && !r->v0.empty()) st = pd_alloc(ctx, &v0, nd);
    if (st == PD_OK && !r->bc_kind.empty()) st = pd_alloc(ctx, &bk, n);
    if (st == PD_OK && !r->bc_kind.empty()) st = pd_alloc(ctx, &bv, nd);
    auto up = [&](void *d, const void *h, size_t bytes) {
        if (st != PD_OK || !d) return;
        const hipError_t e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) st = pd_hip_error(ctx, e, "request upload", __FILE__, __LINE__);
    };
    up(X, r->X.data(), nd * 8);
    up(V, r->V.data(), n * 8);
    up(u0, r->u0.data(), nd * 8);
    up(v0, r->v0.data(), nd * 8);
    up(bk, r->bc_kind.data(), n);
    up(bv, r->bc_vel.data(), nd * 8);
    if (ctx != s->ctx) {
        // the server context's launch choices and tuning results
        ctx->kernel = s->ctx->kernel;
        ctx->tile = s->ctx->tile;
        ctx->block = s->ctx->block;
        ctx->lanes = s->ctx->lanes;
        ctx->tuned = s->ctx->tuned;
    }
    const int saved = ctx->lanes;
    if (s->lanes) ctx->lanes = s->lanes;
    if (st == PD_OK) st = pd_build_neighbors(ctx, r->dim, r->n, X, r->delta, &r->nbr);
    if (st == PD_OK)
        st = pd_sim_create(ctx, r->nbr, &r->mat, X, V, u0, v0, bk, bv, nullptr,
                           r->nseg ? r->notch.data() : nullptr, r->nseg, r->ramp, &r->sim);
    ctx->lanes = saved;
    if (st == PD_OK) {
        const hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = pd_hip_error(ctx, e, "admission", __FILE__, __LINE__);
    }
    pd_free(X);
    pd_free(V);
    pd_free(u0);
    pd_free(v0);
    pd_free(bk);
    pd_free(bv);
    // built on the admission context: the simulation moves to the server's
    if (st == PD_OK && ctx != s->ctx) st = pd_sim_rehome(r->sim, s->ctx);
    if (st != PD_OK) {
        if (r->sim) pd_sim_destroy(r->sim);
        if (r->nbr) pd_nbr_destroy(r->nbr);
        r->sim = nullptr;
        r->nbr = nullptr;
        return st;
    }
    const pd_nbr b = r->nbr;
    r->info.bonds = (int64_t)b->nnz;
    r->info.bytes = std::max(r->estimate,
                             footprint(r->dim, r->n, (int64_t)b->nnz, (int64_t)b->halo_total,
                                       (int64_t)b->ntiles, !r->bc_vel.empty(),
                                       r->mat.law == PD_LAW_LPS));
    return PD_OK;
}

// final state of a finished request (close the last half-step), then free
static int retire(pd_server s, Req *r) {
    pd_ctx ctx = s->ctx;
    int st = PD_OK;
    if (r->keep) {
        const size_t nd = (size_t)r->n * r->dim;
        double *u = nullptr, *v = nullptr;
        st = pd_alloc(ctx, &u, nd);
        if (st == PD_OK) st = pd_alloc(ctx, &v, nd);
        if (st == PD_OK) st = pd_sim_get(r->sim, u, v, nullptr, nullptr, nullptr);
        if (st == PD_OK) {
            r->u_out.resize(nd);
            r->v_out.resize(nd);
            hipError_t e = hipMemcpyAsync(r->u_out.data(), u, nd * 8, hipMemcpyDeviceToHost,
                                          ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->v_out.data(), v, nd * 8, hipMemcpyDeviceToHost,
                                   ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) st = pd_hip_error(ctx, e, "result download", __FILE__, __LINE__);
        }
        pd_free(u);
        pd_free(v);
    }
    release_device(s, r);
    r->info.t_done = now_s();
    r->info.state = st == PD_OK ? PD_REQ_DONE : PD_REQ_FAILED;
    r->info.status = st;
    return st;
}

// admission in arrival order while the head fits the budget, on context
// bctx; returns a device error (the context is unusable), else PD_OK
static int admit_queued(pd_server s, pd_ctx bctx, bool overlapped) {
    while (!s->queue.empty()) {
        Req *r = s->queue.front();
        if (r->estimate > s->budget) {   // can never fit
            s->queue.pop_front();
            r->info.state = PD_REQ_FAILED;
            r->info.status = PD_ECAPACITY;
            r->info.t_done = now_s();
            continue;
        }
        if (s->used + r->estimate > s->budget) break;
        s->queue.pop_front();
        const double ta = now_s();
        const int st = admit(s, r, bctx);
        const double dt = now_s() - ta;
        s->stats.admit_s += dt;
        if (overlapped) s->stats.admit_overlap_s += dt;
        if (st != PD_OK) {
            r->info.state = PD_REQ_FAILED;
            r->info.status = st;
            r->info.t_done = now_s();
            if (st == PD_EDEVICE) return st;   // the context is unusable from here on
            continue;
        }
        if (s->used + r->info.bytes > s->budget) {
            // the estimate was low: free it again, keep the true size and
            // wait at the head of the queue (or fail if it can never fit)
            if (r->sim) pd_sim_destroy(r->sim);
            if (r->nbr) pd_nbr_destroy(r->nbr);
            r->sim = nullptr;
            r->nbr = nullptr;
            r->estimate = r->info.bytes;
            r->info.bytes = 0;
            r->info.bonds = 0;
            if (r->estimate > s->budget) {
                r->info.state = PD_REQ_FAILED;
                r->info.status = PD_ECAPACITY;
                r->info.t_done = now_s();
                continue;
            }
            s->queue.push_front(r);
            break;
        }
        s->used += r->info.bytes;
        s->peak = std::max(s->peak, s->used);
        s->stats.admitted += 1;
        r->info.t_admit = now_s();
        r->info.state = PD_REQ_RUNNING;
        s->running.push_back(r);
    }
    return PD_OK;
}

extern "C" int pd_server_pump(pd_server s, int *n_running, int *n_queued) {
    if (!s) return PD_EINVAL;
    pd_ctx ctx = s->ctx;
    PD_TRY(pd_check_ctx(ctx));
    // with nothing running the device is idle: admit first, on the server's
    // own context, so that the new requests take this round's chunk
    if (s->running.empty()) PD_TRY(admit_queued(s, ctx, false));
    // one chunk for every running simulation: one batched launch per step
    // for each group that can share the streamed kernel, single launches for
    // the rest
    struct Chunk {
        std::vector<pd_sim> sims;
        std::vector<int64_t> steps;
        std::vector<double> dts;
        int64_t nsteps = 0;
    };
    std::map<GroupKey, Chunk> chunks;
    const double t_step = now_s();
    const size_t stepping = s->running.size();
    for (Req *r : s->running) {
        const int64_t k = std::min(s->chunk, r->nsteps - r->done);
        if (k <= 0) continue;
        const pd_sim m = r->sim;
        if (m->stream && m->s_form != SK_LPS_FORCE) {
            Chunk &c = chunks[GroupKey(m->nbr->dim, m->lanes, m->nbr->tile_T,
                                       (int)m->mat.precision, m->mat.law)];
            c.sims.push_back(m);
            c.steps.push_back(k);
            c.dts.push_back(r->dt);
            c.nsteps = std::max(c.nsteps, k);
        } else {
            PD_TRY(pd_verlet_step(m, k, r->dt));
        }
        r->done += k;
    }
    for (auto &kv : chunks) {
        Group &g = s->groups[kv.first];
        if (!g.batch) PD_TRY(pd_batch_create(ctx, &g.batch));
        Chunk &c = kv.second;
        // replay the captured graph while the group keeps its shape
        const bool same = c.sims == g.last_sims && c.nsteps == g.last_nsteps;
        PD_TRY(pd_batch_step(g.batch, c.sims.data(), (int)c.sims.size(), c.steps.data(),
                             c.dts.data(), c.nsteps, same ? 1 : 0));
        s->stats.launches += 1;
        s->stats.replays += same ? 1 : 0;
        g.last_sims = c.sims;
        g.last_nsteps = c.nsteps;
    }
    // while the chunk runs, admit on the admission context (the requests
    // join at the next round); without one, after the chunk
    double t_adm = 0.0;
    if (stepping > 0 && s->actx) {
        const double ta = now_s();
        PD_TRY(admit_queued(s, s->actx, true));
        t_adm = now_s() - ta;
    }
    if (stepping > 0) PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    s->stats.step_s += now_s() - t_step - t_adm;
    s->stats.rounds += 1;
    const double t_ret = now_s();
    // retire the finished ones (those admitted during the chunk have not run)
    std::vector<Req *> keep;
    int dev_err = PD_OK;
    for (size_t k = 0; k < s->running.size(); ++k) {
        Req *r = s->running[k];
        if (k < stepping && r->done >= r->nsteps) {
            const int st = retire(s, r);
            if (st == PD_EDEVICE) dev_err = st;
        } else {
            keep.push_back(r);
        }
    }
    s->running.swap(keep);
    if (dev_err != PD_OK) return dev_err;
    s->stats.retire_s += now_s() - t_ret;
    if (stepping > 0 && !s->actx) PD_TRY(admit_queued(s, ctx, false));
    if (n_running) *n_running = (int)s->running.size();
    if (n_queued) *n_queued = (int)s->queue.size();
    return PD_OK;
}

extern "C" int pd_server_info(pd_server s, int64_t id, pd_request_info *info) {
    if (!s || !info) return PD_EINVAL;
    auto it = s->all.find(id);
    if (it == s->all.end()) return pd_set_error(s->ctx, PD_EINVAL, "unknown request %lld",
                                                (long long)id);
    *info = it->second->info;
    return PD_OK;
}

extern "C" int pd_server_usage(pd_server s, int64_t *used, int64_t *peak) {
    if (!s) return PD_EINVAL;
    if (used) *used = s->used;
    if (peak) *peak = s->peak;
    return PD_OK;
}

extern "C" int pd_server_get_stats(pd_server s, pd_server_stats *out) {
    if (!s || !out) return PD_EINVAL;
    *out = s->stats;
    return PD_OK;
}

extern "C" int pd_server_result(pd_server s, int64_t id, double *u, double *v) {
    if (!s) return PD_EINVAL;
    auto it = s->all.find(id);
    if (it == s->all.end()) return pd_set_error(s->ctx, PD_EINVAL, "unknown request %lld",
                                                (long long)id);
    const Req *r = it->second;
    if (r->info.state != PD_REQ_DONE || !r->keep)
        return pd_set_error(s->ctx, PD_EINVAL, "request %lld has no kept result", (long long)id);
    if (u) std::memcpy(u, r->u_out.data(), r->u_out.size() * 8);
    if (v) std::memcpy(v, r->v_out.data(), r->v_out.size() * 8);
    return PD_OK;
}
