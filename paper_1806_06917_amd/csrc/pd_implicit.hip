// Quasi-static solve (Section "Implicit time integration"): Newton steps
// H(u) du = r with r_i = V_i (f_i(u) + b_i) on free nodes, the tangent H(u)
// applied matrix-free at the current iterate (the paper assembles it by
// central differences; here it is the analytic derivative of the bond force,
// constant for the linearised law and c exp(-beta r)(1 - 2 beta r) per bond
// for the NP law), each Newton system solved by conjugate gradients.
//
// CG runs entirely on the device: per iteration one tangent launch and three
// small vector kernels; the scalars alpha, beta and r.r live in device memory
// and every reduction is a fixed two-level tree (block partials, then the
// same ordered sum in every consumer block), so runs are bit-reproducible.
// A device `done` flag turns the remaining launches of a chunk into no-ops;
// the host looks at the state once per chunk.
//
// Precision: PD_FP64 runs every part in float64.  PD_MIXED applies the
// tangent with the unrefined reciprocal-square-root estimate inside the CG
// (float64 vectors and dot products) and wraps it in iterative refinement
// with full-precision float64 residuals.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pd_kernels.hpp"

namespace {

struct CgState {
    double rr[2];   // r.r, double-buffered by iteration parity
    double tol2;    // stop when r.r <= tol2
    int done;
    int iters;
};

__device__ double reduce_partials(const double *part) {
    // every block computes the same ordered tree over PD_RED_BLOCKS values
    __shared__ double sh[PD_BLOCK];
    double acc = 0.0;
    for (int k = threadIdx.x; k < PD_RED_BLOCKS; k += PD_BLOCK) acc += part[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ void block_partial(double acc, double *part) {
    __shared__ double sh[PD_BLOCK];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void dot_k(const double *a, const double *b, uint64_t m, double *part,
                      const CgState *st) {
    if (st && st->done) return;
    double acc = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        acc += a[k] * b[k];
    block_partial(acc, part);
}

__global__ void cg_update_k(double *x, double *r, const double *p, const double *q, uint64_t m,
                            const double *part_pq, double *part_rr, CgState *st, int parity) {
    if (st->done) return;
    const double pq = reduce_partials(part_pq);
    const double alpha = st->rr[parity] / pq;
    double acc = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x) {
        x[k] = x[k] + alpha * p[k];
        const double rk = r[k] - alpha * q[k];
        r[k] = rk;
        acc += rk * rk;
    }
    block_partial(acc, part_rr);
}

__global__ void cg_direction_k(double *p, const double *r, uint64_t m, const double *part_rr,
                               CgState *st, int parity) {
    if (st->done) return;
    const double rr_new = reduce_partials(part_rr);
    const double beta = rr_new / st->rr[parity];
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        p[k] = r[k] + beta * p[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[parity ^ 1] = rr_new;
        st->iters += 1;
        if (rr_new <= st->tol2) st->done = 1;
    }
}

// r_i = V_i (f_i + b_i) on free nodes, 0 on fixed ones; vectors padded to us
__global__ void residual_k(uint32_t n, int us, int dim, const double *xv, const double *f,
                           const double *b, const uint8_t *fixed, double *r) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (uint64_t)n * us) return;
    const uint32_t i = (uint32_t)(k / us);
    const int c = (int)(k % us);
    const double V = xv[4 * (uint64_t)i + (dim == 3 ? 3 : 2)];
    double v = 0.0;
    if (c < dim && !(fixed && fixed[i])) v = V * (f[k] + (b ? b[k] : 0.0));
    r[k] = v;
}

__global__ void rhs_norm_k(uint32_t n, int us, int dim, const double *xv, const double *b,
                           const uint8_t *fixed, double *out) {
    // out[k] = (V_i b_i)_c on free nodes, 0 otherwise (same layout as r)
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (uint64_t)n * us) return;
    const uint32_t i = (uint32_t)(k / us);
    const int c = (int)(k % us);
    const double V = xv[4 * (uint64_t)i + (dim == 3 ? 3 : 2)];
    out[k] = (c < dim && !(fixed && fixed[i])) ? V * b[k] : 0.0;
}

__global__ void axpy_k(double *y, const double *x, uint64_t m) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) y[k] = y[k] + x[k];
}

__global__ void copy_k(double *y, const double *x, uint64_t m) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) y[k] = x[k];
}

__global__ void zero_k(double *y, uint64_t m) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) y[k] = 0.0;
}

struct Work {
    double *xv = nullptr, *u = nullptr, *b = nullptr, *f = nullptr, *r = nullptr, *x = nullptr,
           *p = nullptr, *q = nullptr, *part_a = nullptr, *part_b = nullptr;
    uint8_t *alive = nullptr, *fixed = nullptr;
    uint16_t *bw = nullptr;
    int block = 0;
    CgState *st = nullptr;
    CgState *st_host = nullptr;
    ~Work() {
        pd_free(xv); pd_free(u); pd_free(b); pd_free(f); pd_free(r); pd_free(x); pd_free(p);
        pd_free(q); pd_free(part_a); pd_free(part_b); pd_free(alive); pd_free(fixed); pd_free(bw); pd_free(st);
        if (st_host) (void)hipHostFree(st_host);
    }
};

int dot_host(pd_ctx ctx, const double *a, const double *b, uint64_t m, double *part,
             double *out) {
    dot_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, ctx->stream>>>(a, b, m, part, nullptr);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(ctx->red_host, part, sizeof(double) * PD_RED_BLOCKS,
                               hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double acc = 0.0;
    for (int k = 0; k < PD_RED_BLOCKS; ++k) acc += ctx->red_host[k];
    *out = acc;
    return PD_OK;
}

// Solves H x = r (x starts at 0) until ||r_k|| <= tol or `budget` iterations.
int cg_solve(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, Work &w, uint64_t m,
             double tol, int budget, int *iters) {
    hipStream_t s = ctx->stream;
    const unsigned gm = pd_blocks(m);
    zero_k<<<gm, PD_BLOCK, 0, s>>>(w.x, m);
    copy_k<<<gm, PD_BLOCK, 0, s>>>(w.p, w.r, m);
    PD_LAUNCH_CHECK(ctx);
    double rr = 0.0;
    PD_TRY(dot_host(ctx, w.r, w.r, m, w.part_a, &rr));
    w.st_host->rr[0] = rr;
    w.st_host->rr[1] = 0.0;
    w.st_host->tol2 = tol * tol;
    w.st_host->done = rr <= tol * tol;
    w.st_host->iters = 0;
    PD_HIP(ctx, hipMemcpyAsync(w.st, w.st_host, sizeof(CgState), hipMemcpyHostToDevice, s));
    const int chunk = 32;
    int done = w.st_host->done;
    int it = 0;
    while (!done && it < budget) {
        const int nrun = std::min(chunk, budget - it);
        for (int k = 0; k < nrun; ++k) {
            const int parity = (it + k) & 1;
            PD_TRY(pd_tangent_sfc(ctx, nbr, mat, w.xv, w.alive, w.bw, w.block, w.fixed, w.p,
                                  w.q, &w.st->done, w.u));
            dot_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, s>>>(w.p, w.q, m, w.part_a, w.st);
            cg_update_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, s>>>(w.x, w.r, w.p, w.q, m, w.part_a,
                                                          w.part_b, w.st, parity);
            cg_direction_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, s>>>(w.p, w.r, m, w.part_b, w.st,
                                                             parity);
            PD_LAUNCH_CHECK(ctx);
        }
        it += nrun;
        PD_HIP(ctx, hipMemcpyAsync(w.st_host, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        PD_HIP(ctx, hipStreamSynchronize(s));
        done = w.st_host->done;
        it = w.st_host->iters;
    }
    *iters = w.st_host->iters;
    return PD_OK;
}

}  // namespace

extern "C" int pd_solve_implicit(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                                 const double *V, const uint8_t *alive, const uint8_t *fixed,
                                 const double *b, double *u, double rtol, int maxit,
                                 pd_solve_info *info) {
    if (!nbr) return pd_set_error(ctx, PD_EINVAL, "nbr must not be NULL");
    if (nbr->closing) return pd_set_error(ctx, PD_EINVAL, "nbr has been destroyed");
    if (nbr->nnz == 0)
        return pd_set_error(ctx, PD_EINVAL, "the mesh has no bonds (no two nodes within delta)");
    PD_TRY(pd_check_ctx(ctx));
    if (nbr->ctx != ctx) return pd_set_error(ctx, PD_EINVAL, "nbr belongs to another context");
    if (!mat || mat->dim != nbr->dim) return pd_set_error(ctx, PD_EINVAL, "bad material");
    if (mat->precision != PD_FP64 && mat->precision != PD_MIXED)
        return pd_set_error(ctx, PD_EINVAL, "bad precision");
    PD_TRY(pd_check_law(ctx, mat));
    if (mat->stretch != PD_STRETCH_LINEARISED || mat->law == PD_LAW_LPS || mat->pv_h > 0.0 ||
        mat->j_c2 > 0.0)
        return pd_set_error(ctx, PD_EINVAL,
                            "the implicit solve takes a pairwise law with the linearised stretch");
    if (!(rtol > 0.0) || !(rtol < 1.0)) return pd_set_error(ctx, PD_EINVAL, "rtol must be in (0,1)");
    if (maxit <= 0) return pd_set_error(ctx, PD_EINVAL, "maxit must be positive");
    PD_TRY(pd_check_dev_ptr(ctx, X, "X"));
    PD_TRY(pd_check_dev_ptr(ctx, V, "V"));
    PD_TRY(pd_check_dev_ptr(ctx, b, "b"));
    PD_TRY(pd_check_dev_ptr(ctx, u, "u"));
    if (alive) PD_TRY(pd_check_dev_ptr(ctx, alive, "alive"));
    if (fixed) PD_TRY(pd_check_dev_ptr(ctx, fixed, "fixed"));

    const uint32_t n = nbr->n;
    const int dim = nbr->dim, us = dim == 3 ? 4 : 2;
    const uint64_t m = (uint64_t)n * us;
    Work w;
    PD_TRY(pd_alloc(ctx, &w.xv, (size_t)n * 4));
    PD_TRY(pd_alloc(ctx, &w.u, m));
    PD_TRY(pd_alloc(ctx, &w.b, m));
    PD_TRY(pd_alloc(ctx, &w.f, m));
    PD_TRY(pd_alloc(ctx, &w.r, m));
    PD_TRY(pd_alloc(ctx, &w.x, m));
    PD_TRY(pd_alloc(ctx, &w.p, m));
    PD_TRY(pd_alloc(ctx, &w.q, m));
    PD_TRY(pd_alloc(ctx, &w.part_a, PD_RED_BLOCKS));
    PD_TRY(pd_alloc(ctx, &w.part_b, PD_RED_BLOCKS));
    PD_TRY(pd_alloc(ctx, &w.st, 1));
    if (hipHostMalloc((void **)&w.st_host, sizeof(CgState)) != hipSuccess) {
        (void)hipGetLastError();
        return pd_set_error(ctx, PD_ENOMEM, "pinned allocation failed");
    }
    if (alive) {
        PD_TRY(pd_alloc(ctx, &w.alive, nbr->nnz));
        PD_TRY(pd_alive_in(ctx, nbr, alive, w.alive));
    }
    if (fixed) {
        PD_TRY(pd_alloc(ctx, &w.fixed, n));
        PD_TRY(pd_gather_u8(ctx, nbr, fixed, w.fixed, 0));
    }
    int block = 0;
    const bool np = mat->law == PD_LAW_NP;
    if (!pd_general_law(mat))
        PD_TRY(pd_plan_kernel(ctx, nbr, pd_auto_lanes(ctx, nbr->nnz, nbr->n), &block));
    w.block = block;
    if (block > 0) {
        PD_TRY(pd_alloc(ctx, &w.bw, nbr->nnz + PD_BW_PAD));
        PD_TRY(pd_bw_compose(ctx, nbr, w.alive, w.bw));
    }
    PD_TRY(pd_gather_xv(ctx, nbr, X, V, w.xv));
    PD_TRY(pd_gather_vec(ctx, nbr, u, w.u, false));
    PD_TRY(pd_gather_vec(ctx, nbr, b, w.b, false));

    // ||V b|| over free nodes
    const unsigned gm = pd_blocks(m);
    rhs_norm_k<<<gm, PD_BLOCK, 0, ctx->stream>>>(n, us, dim, w.xv, w.b, w.fixed, w.r);
    PD_LAUNCH_CHECK(ctx);
    double bn2 = 0.0;
    PD_TRY(dot_host(ctx, w.r, w.r, m, w.part_a, &bn2));
    const double bnorm = bn2 > 0.0 ? std::sqrt(bn2) : 1.0;

    pd_material inner = *mat;
    const bool mixed = mat->precision == PD_MIXED;
    // Newton steps: one suffices for the linearised law (a few more for
    // iterative refinement); NP converges quadratically near the solution
    const int max_outer = np ? 60 : (mixed ? 30 : 4);
    int outer = 0, inner_total = 0, status = PD_ENOCONV;
    double rel = 0.0;
    while (true) {
        PD_TRY(pd_force_sfc(ctx, nbr, mat, w.xv, w.alive, w.bw, w.block, w.u, w.f));
        residual_k<<<gm, PD_BLOCK, 0, ctx->stream>>>(n, us, dim, w.xv, w.f, w.b, w.fixed, w.r);
        PD_LAUNCH_CHECK(ctx);
        double rr = 0.0;
        PD_TRY(dot_host(ctx, w.r, w.r, m, w.part_a, &rr));
        rel = std::sqrt(rr) / bnorm;
        if (!std::isfinite(rel)) {
            status = pd_set_error(ctx, PD_ENONFINITE, "non-finite residual");
            break;
        }
        if (rel <= rtol) {
            status = PD_OK;
            break;
        }
        if (outer >= max_outer || inner_total >= maxit) break;
        // inner target: FP64 solves straight to the requested accuracy (with a
        // small margin); mixed solves each correction to 1e-5 relative
        // (NP: the Newton system to 1e-6 relative or the final target, the
        // looser of the two, keeps Newton's convergence fast)
        double target = mixed ? 1e-5 * std::sqrt(rr) : 0.5 * rtol * bnorm;
        if (np) target = std::max(target, 1e-6 * std::sqrt(rr));
        int k = 0;
        PD_TRY(cg_solve(ctx, nbr, &inner, w, m, target, maxit - inner_total, &k));
        inner_total += k;
        axpy_k<<<gm, PD_BLOCK, 0, ctx->stream>>>(w.u, w.x, m);
        PD_LAUNCH_CHECK(ctx);
        ++outer;
    }
    PD_TRY(pd_scatter_vec(ctx, nbr, w.u, u));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (info) {
        info->outer_iters = outer;
        info->inner_iters = inner_total;
        info->rel_residual = rel;
    }
    if (status == PD_ENOCONV)
        return pd_set_error(ctx, PD_ENOCONV, "relative residual %.3e above %.3e after %d CG steps",
                            rel, rtol, inner_total);
    return status;
}
