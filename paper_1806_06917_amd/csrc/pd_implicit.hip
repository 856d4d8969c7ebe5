// Quasi-static solve (Section "Implicit time integration"): Newton steps
// H(u) du = r with r_i = V_i (f_i(u) + b_i) on free nodes, the tangent H(u)
// applied matrix-free at the current iterate (the paper assembles it by
// central differences; here it is the analytic derivative of the bond force,
// constant for the linearised law and c exp(-beta r)(1 - 2 beta r) per bond
// for the NP law), each Newton system solved by conjugate gradients.
//
// CG runs on the device in one launch per iteration, in the form of
// Chronopoulos and Gear (1989), which needs one fused reduction per iteration
// instead of two: with w = H r kept beside r, gamma = r.r and delta = w.r
// give beta = gamma / gamma_old and alpha = gamma / (delta - beta gamma /
// alpha_old), then p = r + beta p, s = w + beta s, x += alpha p,
// r -= alpha s, and the next w = H r.  The launch forms the new r on the fly
// for every neighbour it reads (r, w and s are double-buffered, so no block
// overwrites a value another block still reads), applies the tangent to it,
// stores its own nodes' vectors and sums gamma and delta per block.  Every
// block reduces the previous launch's block sums in one fixed order, so all
// blocks derive the same alpha, beta and stopping decision and runs are
// bit-reproducible; a device state word records gamma, alpha and the
// iteration count, and the host looks at it once per chunk of iterations.
// The float32 corrections of the mixed solve keep the classic form in two
// launches per iteration (p = r + beta p and q = H p with the sum of p.q,
// then x, r and the sum of r.r): in float32 the one-launch recurrences let r
// drift from the true residual, which cost more iterations (2253 against
// 1204 on the 400 x 40 bar) than the shorter iterations saved.
//
// Precision: PD_FP64 runs every part in float64.  PD_MIXED solves each
// correction with float32 CG vectors (x, r, w, p, s) and float32 bond
// arithmetic in the tangent, with float64 dot products, inside iterative
// refinement on float64 residuals (the force in float64) until the relative
// residual reaches the requested tolerance.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "pd_kernels.hpp"

namespace {

using namespace pdk;

struct CgState {
    double rr[2];      // r.r at the start of iteration m, in slot m & 1
    double alpha[2];   // alpha of iteration m, in slot m & 1
    double tol2;       // stop when r.r <= tol2
    int done;
    int iters;
};

// ordered tree over nparts block sums (the same in every block)
__device__ double reduce_partials(const double *part, int nparts) {
    __shared__ double sh[PD_BLOCK];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nparts; k += PD_BLOCK) acc += part[k];
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

// both sums of a launch: block sums of a and b in one tree
__device__ void block_partial2(double a, double b, double *part_a, double *part_b) {
    __shared__ double sa[PD_BLOCK], sb[PD_BLOCK];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sa[threadIdx.x] += sa[threadIdx.x + off];
            sb[threadIdx.x] += sb[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_a[blockIdx.x] = sa[0];
        part_b[blockIdx.x] = sb[0];
    }
}

// the totals of both block-sum arrays, each by an ordered tree over the nparts
// block sums (the same in every block)
__device__ void reduce_partials2(const double *part_a, const double *part_b, int nparts,
                                 double &ta, double &tb) {
    __shared__ double sa[PD_BLOCK], sb[PD_BLOCK];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nparts; k += PD_BLOCK) {
        a += part_a[k];
        b += part_b[k];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sa[threadIdx.x] += sa[threadIdx.x + off];
            sb[threadIdx.x] += sb[threadIdx.x + off];
        }
        __syncthreads();
    }
    ta = sa[0];
    tb = sb[0];
    __syncthreads();
}

__global__ void dot_k(const double *a, const double *b, uint64_t m, double *part) {
    double acc = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        acc += a[k] * b[k];
    block_partial(acc, part);
}

// Tangent factor of each bond at the linearisation point u (NP law):
// k = exp(-beta r)(1 - 2 beta r), r = |xi| S^2, S = (eta.xi)/|xi|^2 -- the
// factor psi'(r) + 2 r psi''(r) over psi'(0) of the tangent
template <int DIM>
__global__ void bond_factor_k(uint32_t n, const uint32_t *row_ptr, const int32_t *col,
                              const double *xv, const double *u, double beta, double *kb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int US = DIM == 3 ? 4 : 2;
    const double xix = xv[4 * (size_t)i], xiy = xv[4 * (size_t)i + 1];
    const double xiz = DIM == 3 ? xv[4 * (size_t)i + 2] : 0.0;
    const double uix = u[(size_t)i * US], uiy = u[(size_t)i * US + 1];
    const double uiz = DIM == 3 ? u[(size_t)i * US + 2] : 0.0;
    for (uint32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const uint32_t j = (uint32_t)col[p];
        const double dx = xv[4 * (size_t)j] - xix, dy = xv[4 * (size_t)j + 1] - xiy;
        const double dz = DIM == 3 ? xv[4 * (size_t)j + 2] - xiz : 0.0;
        const double ex = u[(size_t)j * US] - uix, ey = u[(size_t)j * US + 1] - uiy;
        const double ez = DIM == 3 ? u[(size_t)j * US + 2] - uiz : 0.0;
        const double r2 = dotf<DIM>(dx, dy, dz, dx, dy, dz);
        const double S = dotf<DIM>(ex, ey, ez, dx, dy, dz) / r2;
        const double r = sqrt(r2) * S * S;
        kb[p] = exp(-beta * r) * (1.0 - 2.0 * beta * r);
    }
}

// one CG solve's arrays; vectors in sfc order, [n][US] like u
template <class T>
struct CgArgs {
    uint32_t n;
    const uint32_t *row_ptr;
    const int32_t *col;
    const double *xv;            // {x, y, z, V} / {x, y, V, 0}
    const uint8_t *alive;        // NULL: all intact
    const uint8_t *fixed;        // NULL: none
    const double *kb;            // per-bond tangent factor (NP), NULL: 1
    double c;
    T *x, *p;                    // own nodes only: updated in place
    T *r[2], *w[2], *s[2];       // read in slot k & 1, written in slot (k + 1) & 1
    double *part_g, *part_d;     // block sums of r.r and w.r
    int nparts;
    CgState *st;
};

__device__ __forceinline__ double rsq_of(double r2) { return rsqrt_pos(r2); }
__device__ __forceinline__ float rsq_of(float r2) { return __builtin_amdgcn_rsqf(r2); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_of(float a, float b, float c) { return fmaf(a, b, c); }

// Launch k.  k = 0 starts the solve: alpha = beta = 0, so it only forms
// w_0 = H r_0 and the sums of r_0.r_0 and w_0.r_0.  Launch k >= 1 is
// iteration m = k - 1: it reduces gamma_m and delta_m (the stopping test),
// derives beta_m and alpha_m, updates its own nodes (s_m = w_m + beta s,
// p_m = r_m + beta p, x += alpha p_m, r_{m+1} = r_m - alpha s_m), applies
// the tangent to r_{m+1}, forming it for every neighbour read the same way
// (fixed rows identity, r read as 0 at fixed nodes, dead bonds skipped), and
// sums r_{m+1}.r_{m+1} and w_{m+1}.r_{m+1} per block.  L lanes per node.
template <int DIM, int L, class T>
__global__ __launch_bounds__(PD_BLOCK) void cg_step_k(CgArgs<T> a, int k) {
    CgState *st = a.st;
    if (st->done) return;
    constexpr int US = DIM == 3 ? 4 : 2;
    double alpha = 0.0, beta = 0.0;
    if (k > 0) {
        const int m = k - 1;
        double g, d;
        reduce_partials2(a.part_g, a.part_d, a.nparts, g, d);
        double den = d;
        if (m > 0) {
            beta = g / st->rr[(m - 1) & 1];
            den = d - beta * g / st->alpha[(m - 1) & 1];
        }
        // converged, or the curvature p.Hp (= den in exact arithmetic) no
        // longer positive: every block takes the same decision
        if (g <= st->tol2 || !(den > 0.0)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->rr[m & 1] = g;
                st->iters = m;
                st->done = 1;
            }
            return;
        }
        alpha = g / den;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->rr[m & 1] = g;
            st->alpha[m & 1] = alpha;
        }
    }
    const T ta = (T)alpha, tb = (T)beta;
    const T *__restrict__ rc = a.r[k & 1];
    const T *__restrict__ wc = a.w[k & 1];
    const T *__restrict__ sc = a.s[k & 1];
    T *__restrict__ rn = a.r[(k + 1) & 1];
    T *__restrict__ wn = a.w[(k + 1) & 1];
    T *__restrict__ sn = a.s[(k + 1) & 1];
    // s_m and r_{m+1} of node j, component d (the same operations wherever
    // they are formed)
    auto s_of = [&](uint32_t j, int d) -> T {
        return fma_of(tb, sc[(size_t)j * US + d], wc[(size_t)j * US + d]);
    };
    auto r_of = [&](uint32_t j, int d, T sj) -> T {
        return fma_of(-ta, sj, rc[(size_t)j * US + d]);
    };
    const int lane = threadIdx.x & (L - 1);
    const uint32_t per = (uint32_t)(gridDim.x * PD_BLOCK / L);
    double gp = 0.0, dp = 0.0;
    for (uint32_t i = (blockIdx.x * PD_BLOCK + threadIdx.x) / L; i < a.n; i += per) {
        const bool fi = a.fixed && a.fixed[i];
        const T six = s_of(i, 0), siy = s_of(i, 1), siz = DIM == 3 ? s_of(i, 2) : (T)0;
        const T rix = r_of(i, 0, six), riy = r_of(i, 1, siy), riz = DIM == 3 ? r_of(i, 2, siz) : (T)0;
        const double xix = a.xv[4 * (size_t)i], xiy = a.xv[4 * (size_t)i + 1];
        const double xiz = DIM == 3 ? a.xv[4 * (size_t)i + 2] : 0.0;
        const double Vi = a.xv[4 * (size_t)i + (DIM == 3 ? 3 : 2)];
        T hx = 0, hy = 0, hz = 0;
        if (!fi) {
            for (uint32_t e = a.row_ptr[i] + lane; e < a.row_ptr[i + 1]; e += L) {
                if (a.alive && !a.alive[e]) continue;
                const uint32_t j = (uint32_t)a.col[e];
                const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
                const T dx = (T)(xj.x - xix), dy = (T)(xj.y - xiy);
                const T dz = DIM == 3 ? (T)(xj.z - xiz) : (T)0;
                T vx, vy, vz = 0;
                if (!(a.fixed && a.fixed[j])) {
                    vx = r_of(j, 0, s_of(j, 0)) - rix;
                    vy = r_of(j, 1, s_of(j, 1)) - riy;
                    if (DIM == 3) vz = r_of(j, 2, s_of(j, 2)) - riz;
                } else {
                    vx = -rix;
                    vy = -riy;
                    if (DIM == 3) vz = -riz;
                }
                const T r2 = DIM == 3 ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
                const T ev = DIM == 3 ? vx * dx + vy * dy + vz * dz : vx * dx + vy * dy;
                const T inv = rsq_of(r2);
                T g = (T)(a.c * (DIM == 3 ? xj.w : xj.z)) * (ev * inv * inv) * inv;
                if (a.kb) g *= (T)a.kb[e];
                hx += g * dx;
                hy += g * dy;
                if (DIM == 3) hz += g * dz;
            }
        }
        // lane sums (neighbouring lanes first)
        for (int o = 1; o < L; o <<= 1) {
            hx += __shfl_xor(hx, o, L);
            hy += __shfl_xor(hy, o, L);
            if (DIM == 3) hz += __shfl_xor(hz, o, L);
        }
        if (lane == 0) {
            const size_t b = (size_t)i * US;
            const T wx = fi ? rix : (T)(-Vi) * hx, wy = fi ? riy : (T)(-Vi) * hy;
            const T wz = fi ? riz : (T)(-Vi) * hz;
            const T px = fma_of(tb, a.p[b], rc[b]), py = fma_of(tb, a.p[b + 1], rc[b + 1]);
            a.p[b] = px;
            a.p[b + 1] = py;
            a.x[b] = fma_of(ta, px, a.x[b]);
            a.x[b + 1] = fma_of(ta, py, a.x[b + 1]);
            sn[b] = six;
            sn[b + 1] = siy;
            rn[b] = rix;
            rn[b + 1] = riy;
            wn[b] = wx;
            wn[b + 1] = wy;
            if (DIM == 3) {
                const T pz = fma_of(tb, a.p[b + 2], rc[b + 2]);
                a.p[b + 2] = pz;
                a.x[b + 2] = fma_of(ta, pz, a.x[b + 2]);
                sn[b + 2] = siz;
                rn[b + 2] = riz;
                wn[b + 2] = wz;
            }
            gp += (double)rix * (double)rix + (double)riy * (double)riy +
                  (DIM == 3 ? (double)riz * (double)riz : 0.0);
            dp += (double)wx * (double)rix + (double)wy * (double)riy +
                  (DIM == 3 ? (double)wz * (double)riz : 0.0);
        }
    }
    block_partial2(gp, dp, a.part_g, a.part_d);
}

// The two-launch form (the mixed solve's float32 corrections): one solve's
// arrays, vectors in sfc order, [n][US] like u
template <class T>
struct Cg2Args {
    uint32_t n;
    const uint32_t *row_ptr;
    const int32_t *col;
    const double *xv;            // {x, y, z, V} / {x, y, V, 0}
    const uint8_t *alive;        // NULL: all intact
    const uint8_t *fixed;        // NULL: none
    const double *kb;            // per-bond tangent factor (NP), NULL: 1
    double c;
    T *x, *r, *q;
    T *p[2];                     // search direction, double-buffered
    double *part_pq, *part_rr;   // block sums
    int nparts;
    CgState *st;
};

// First launch of iteration `it`: beta from the previous update's r.r (and
// the stopping test), p = r + beta p_old for every node read, q = H p for
// the block's nodes (fixed rows identity, p read as 0 at fixed nodes, dead
// bonds skipped), and the block's sum of p.q.  L lanes per node.
template <int DIM, int L, class T>
__global__ __launch_bounds__(PD_BLOCK) void cg_apply_k(Cg2Args<T> a, int it) {
    CgState *st = a.st;
    if (st->done) return;
    constexpr int US = DIM == 3 ? 4 : 2;
    double beta = 0.0;
    if (it > 0) {
        const double rr = reduce_partials(a.part_rr, a.nparts);
        beta = rr / st->rr[(it - 1) & 1];
        if (rr <= st->tol2) {          // every block takes the same decision
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->rr[it & 1] = rr;
                st->iters = it;
                st->done = 1;
            }
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) st->rr[it & 1] = rr;
    }
    const T tb = (T)beta;
    const T *__restrict__ pold = a.p[it & 1];
    T *__restrict__ pnew = a.p[(it + 1) & 1];
    const T *__restrict__ r = a.r;
    auto dir = [&](uint32_t j, int d) -> T {
        return it == 0 ? r[(size_t)j * US + d] : r[(size_t)j * US + d] + tb * pold[(size_t)j * US + d];
    };
    const int lane = threadIdx.x & (L - 1);
    const uint32_t per = (uint32_t)(gridDim.x * PD_BLOCK / L);
    double pq = 0.0;
    for (uint32_t i = (blockIdx.x * PD_BLOCK + threadIdx.x) / L; i < a.n; i += per) {
        const bool fi = a.fixed && a.fixed[i];
        const T pix = dir(i, 0), piy = dir(i, 1), piz = DIM == 3 ? dir(i, 2) : (T)0;
        const double xix = a.xv[4 * (size_t)i], xiy = a.xv[4 * (size_t)i + 1];
        const double xiz = DIM == 3 ? a.xv[4 * (size_t)i + 2] : 0.0;
        const double Vi = a.xv[4 * (size_t)i + (DIM == 3 ? 3 : 2)];
        T sx = 0, sy = 0, sz = 0;
        if (!fi) {
            for (uint32_t e = a.row_ptr[i] + lane; e < a.row_ptr[i + 1]; e += L) {
                if (a.alive && !a.alive[e]) continue;
                const uint32_t j = (uint32_t)a.col[e];
                const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
                const T dx = (T)(xj.x - xix), dy = (T)(xj.y - xiy);
                const T dz = DIM == 3 ? (T)(xj.z - xiz) : (T)0;
                T wx = 0, wy = 0, wz = 0;
                if (!(a.fixed && a.fixed[j])) {
                    wx = dir(j, 0) - pix;
                    wy = dir(j, 1) - piy;
                    if (DIM == 3) wz = dir(j, 2) - piz;
                } else {
                    wx = -pix;
                    wy = -piy;
                    if (DIM == 3) wz = -piz;
                }
                const T r2 = DIM == 3 ? dx * dx + dy * dy + dz * dz : dx * dx + dy * dy;
                const T ew = DIM == 3 ? wx * dx + wy * dy + wz * dz : wx * dx + wy * dy;
                const T inv = rsq_of(r2);
                T g = (T)(a.c * (DIM == 3 ? xj.w : xj.z)) * (ew * inv * inv) * inv;
                if (a.kb) g *= (T)a.kb[e];
                sx += g * dx;
                sy += g * dy;
                if (DIM == 3) sz += g * dz;
            }
        }
        // lane sums (neighbouring lanes first)
        for (int o = 1; o < L; o <<= 1) {
            sx += __shfl_xor(sx, o, L);
            sy += __shfl_xor(sy, o, L);
            if (DIM == 3) sz += __shfl_xor(sz, o, L);
        }
        if (lane == 0) {
            const T qx = fi ? pix : (T)(-Vi) * sx, qy = fi ? piy : (T)(-Vi) * sy;
            const T qz = fi ? piz : (T)(-Vi) * sz;
            a.q[(size_t)i * US] = qx;
            a.q[(size_t)i * US + 1] = qy;
            pnew[(size_t)i * US] = pix;
            pnew[(size_t)i * US + 1] = piy;
            if (DIM == 3) {
                a.q[(size_t)i * US + 2] = qz;
                pnew[(size_t)i * US + 2] = piz;
            }
            pq += (double)pix * (double)qx + (double)piy * (double)qy +
                  (DIM == 3 ? (double)piz * (double)qz : 0.0);
        }
    }
    block_partial(pq, a.part_pq);
}

// Second launch: alpha = r.r / p.q, x += alpha p, r -= alpha q, block sums
// of the new r.r.
template <int DIM, class T>
__global__ __launch_bounds__(PD_BLOCK) void cg_update_k(Cg2Args<T> a, int it) {
    CgState *st = a.st;
    if (st->done) return;
    constexpr int US = DIM == 3 ? 4 : 2;
    const double pq = reduce_partials(a.part_pq, a.nparts);
    const T alpha = (T)(st->rr[it & 1] / pq);
    const T *__restrict__ p = a.p[(it + 1) & 1];
    double acc = 0.0;
    const uint64_t m = (uint64_t)a.n * US;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x) {
        if (DIM == 3 && (k & 3) == 3) continue;   // padding
        a.x[k] = a.x[k] + alpha * p[k];
        const T rk = a.r[k] - alpha * a.q[k];
        a.r[k] = rk;
        acc += (double)rk * (double)rk;
    }
    block_partial(acc, a.part_rr);
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

// y += (double) x
template <class T>
__global__ void add_k(double *y, const T *x, uint64_t m) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) y[k] = y[k] + (double)x[k];
}

// CG start: x = 0, r = (T) rhs, p = w = s = 0 (the slots launch 0 reads)
template <class T>
__global__ void cg_init_k(const double *rhs, T *x, T *p, T *r, T *w, T *s, uint64_t m) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    x[k] = 0;
    p[k] = 0;
    r[k] = (T)rhs[k];
    w[k] = 0;
    s[k] = 0;
}

template <class T>
__global__ void r_dot_k(const T *r, uint64_t m, double *part) {
    double acc = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        acc += (double)r[k] * (double)r[k];
    block_partial(acc, part);
}

template <class T>
struct CgVecs {
    T *x = nullptr, *p = nullptr, *r[2] = {nullptr, nullptr}, *w[2] = {nullptr, nullptr},
      *s[2] = {nullptr, nullptr};
    ~CgVecs() {
        pd_free(x);
        pd_free(p);
        for (int k = 0; k < 2; ++k) {
            pd_free(r[k]);
            pd_free(w[k]);
            pd_free(s[k]);
        }
    }
    int alloc(pd_ctx ctx, uint64_t m) {
        PD_TRY(pd_alloc(ctx, &x, m));
        PD_TRY(pd_alloc(ctx, &p, m));
        for (int k = 0; k < 2; ++k) {
            PD_TRY(pd_alloc(ctx, &r[k], m));
            PD_TRY(pd_alloc(ctx, &w[k], m));
            PD_TRY(pd_alloc(ctx, &s[k], m));
        }
        return PD_OK;
    }
};

struct Work {
    double *xv = nullptr, *u = nullptr, *b = nullptr, *f = nullptr, *r = nullptr,
           *part_a = nullptr, *part_b = nullptr, *kb = nullptr;
    uint8_t *alive = nullptr, *fixed = nullptr;
    uint16_t *bw = nullptr;
    int block = 0;
    CgVecs<double> v64;
    CgVecs<float> v32;
    CgState *st = nullptr;
    CgState *st_host = nullptr;
    ~Work() {
        pd_free(xv); pd_free(u); pd_free(b); pd_free(f); pd_free(r); pd_free(part_a);
        pd_free(part_b); pd_free(kb); pd_free(alive); pd_free(fixed); pd_free(bw); pd_free(st);
        if (st_host) (void)hipHostFree(st_host);
    }
};

int dot_host(pd_ctx ctx, const double *a, const double *b, uint64_t m, double *part,
             double *out) {
    dot_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, ctx->stream>>>(a, b, m, part);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(ctx->red_host, part, sizeof(double) * PD_RED_BLOCKS,
                               hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double acc = 0.0;
    for (int k = 0; k < PD_RED_BLOCKS; ++k) acc += ctx->red_host[k];
    *out = acc;
    return PD_OK;
}

template <int DIM, class T>
int launch_cg_lanes(pd_ctx ctx, const CgArgs<T> &a, int k, unsigned grid, int L) {
    hipStream_t s = ctx->stream;
    switch (L) {
    case 1: cg_step_k<DIM, 1, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    case 2: cg_step_k<DIM, 2, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    case 4: cg_step_k<DIM, 4, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    case 8: cg_step_k<DIM, 8, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    case 16: cg_step_k<DIM, 16, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    default: cg_step_k<DIM, 32, T><<<grid, PD_BLOCK, 0, s>>>(a, k); break;
    }
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

template <int DIM, int L, class T>
void launch_cg2_iter(const Cg2Args<T> &a, int it, unsigned grid, hipStream_t s) {
    cg_apply_k<DIM, L, T><<<grid, PD_BLOCK, 0, s>>>(a, it);
    cg_update_k<DIM, T><<<grid, PD_BLOCK, 0, s>>>(a, it);
}

template <int DIM, class T>
int launch_cg2_lanes(pd_ctx ctx, const Cg2Args<T> &a, int it, unsigned grid, int L) {
    hipStream_t s = ctx->stream;
    switch (L) {
    case 1: launch_cg2_iter<DIM, 1, T>(a, it, grid, s); break;
    case 2: launch_cg2_iter<DIM, 2, T>(a, it, grid, s); break;
    case 4: launch_cg2_iter<DIM, 4, T>(a, it, grid, s); break;
    case 8: launch_cg2_iter<DIM, 8, T>(a, it, grid, s); break;
    case 16: launch_cg2_iter<DIM, 16, T>(a, it, grid, s); break;
    default: launch_cg2_iter<DIM, 32, T>(a, it, grid, s); break;
    }
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

// Solves H x = rhs (x from 0) until ||r|| <= tol or `budget` iterations, in
// the vector precision T; x is left in v.x.
template <class T>
int cg_solve(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, Work &w, CgVecs<T> &v,
             const double *rhs, uint64_t m, double tol, int budget, int *iters) {
    hipStream_t s = ctx->stream;
    const unsigned gm = pd_blocks(m);
    cg_init_k<T><<<gm, PD_BLOCK, 0, s>>>(rhs, v.x, v.p, v.r[0], v.w[0], v.s[0], m);
    r_dot_k<T><<<PD_RED_BLOCKS, PD_BLOCK, 0, s>>>(v.r[0], m, w.part_a);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(ctx->red_host, w.part_a, sizeof(double) * PD_RED_BLOCKS,
                               hipMemcpyDeviceToHost, s));
    PD_HIP(ctx, hipStreamSynchronize(s));
    double rr = 0.0;
    for (int k = 0; k < PD_RED_BLOCKS; ++k) rr += ctx->red_host[k];
    w.st_host->rr[0] = rr;
    w.st_host->rr[1] = 0.0;
    w.st_host->alpha[0] = w.st_host->alpha[1] = 0.0;
    w.st_host->tol2 = tol * tol;
    w.st_host->done = rr <= tol * tol;
    w.st_host->iters = 0;
    PD_HIP(ctx, hipMemcpyAsync(w.st, w.st_host, sizeof(CgState), hipMemcpyHostToDevice, s));
    // about four bonds per lane: the tangent launch of a small system is
    // latency-bound (each bond a chain of dependent loads), so it takes many
    // short lanes
    const double k = nbr->n ? (double)nbr->nnz / (double)nbr->n : 0.0;
    int L = 1;
    while (L < 32 && L * 4 < k) L *= 2;
    // one grid for every launch: enough blocks for every node's lane group
    // (at most the partial-sum slots)
    uint64_t need = ((uint64_t)nbr->n * L + PD_BLOCK - 1) / PD_BLOCK;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(need, PD_RED_BLOCKS));
    const int chunk = 32;
    int done = w.st_host->done;
    if constexpr (std::is_same<T, float>::value) {
        // float32 corrections: the two-launch form (its float32 recurrences
        // keep r close to the true residual; the one-launch form's drift apart
        // and cost more iterations than its shorter launches save)
        Cg2Args<T> a{};
        a.n = nbr->n;
        a.row_ptr = nbr->row_ptr;
        a.col = nbr->col;
        a.xv = w.xv;
        a.alive = w.alive;
        a.fixed = w.fixed;
        a.kb = mat->law == PD_LAW_NP ? w.kb : nullptr;
        a.c = mat->c;
        a.x = v.x;
        a.r = v.r[0];
        a.q = v.w[0];
        a.p[0] = v.p;        // both direction buffers start at 0
        a.p[1] = v.s[0];
        a.part_pq = w.part_a;
        a.part_rr = w.part_b;
        a.nparts = (int)grid;
        a.st = w.st;
        int it = 0;
        while (!done && it < budget) {
            const int nrun = std::min(chunk, budget - it);
            for (int k = 0; k < nrun; ++k) {
                const int st = nbr->dim == 3 ? launch_cg2_lanes<3, T>(ctx, a, it + k, grid, L)
                                             : launch_cg2_lanes<2, T>(ctx, a, it + k, grid, L);
                if (st != PD_OK) return st;
            }
            it += nrun;
            PD_HIP(ctx, hipMemcpyAsync(w.st_host, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            PD_HIP(ctx, hipStreamSynchronize(s));
            done = w.st_host->done;
            if (done) it = w.st_host->iters;
        }
        *iters = it;
        return PD_OK;
    }
    CgArgs<T> a{};
    a.n = nbr->n;
    a.row_ptr = nbr->row_ptr;
    a.col = nbr->col;
    a.xv = w.xv;
    a.alive = w.alive;
    a.fixed = w.fixed;
    a.kb = mat->law == PD_LAW_NP ? w.kb : nullptr;
    a.c = mat->c;
    a.x = v.x;
    a.p = v.p;
    for (int k = 0; k < 2; ++k) {
        a.r[k] = v.r[k];
        a.w[k] = v.w[k];
        a.s[k] = v.s[k];
    }
    a.part_g = w.part_a;
    a.part_d = w.part_b;
    a.nparts = (int)grid;
    a.st = w.st;
    // launch 0 forms w_0 = H r_0; launch k >= 1 is iteration k - 1, so
    // launches 0..budget run at most `budget` iterations
    int launched = 0;
    while (!done && launched <= budget) {
        const int nrun = std::min(chunk, budget + 1 - launched);
        for (int k = 0; k < nrun; ++k) {
            const int st = nbr->dim == 3 ? launch_cg_lanes<3, T>(ctx, a, launched + k, grid, L)
                                         : launch_cg_lanes<2, T>(ctx, a, launched + k, grid, L);
            if (st != PD_OK) return st;
        }
        launched += nrun;
        PD_HIP(ctx, hipMemcpyAsync(w.st_host, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        PD_HIP(ctx, hipStreamSynchronize(s));
        done = w.st_host->done;
    }
    *iters = done ? w.st_host->iters : budget;
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
    if (mat->precision != PD_FP64 && mat->precision != PD_MIXED && mat->precision != PD_FP32)
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
    // PD_FP32 solves like PD_MIXED: float32 corrections, float64 residuals
    const bool mixed = mat->precision != PD_FP64;
    if (mixed) PD_TRY(w.v32.alloc(ctx, m));
    else PD_TRY(w.v64.alloc(ctx, m));
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
    if (np) PD_TRY(pd_alloc(ctx, &w.kb, nbr->nnz));
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
        // small margin).  Mixed, linearised law: each correction of the
        // iterative refinement to 1e-2 relative (a float32 CG converges ever
        // more slowly as it nears its stall near 1e-5, so shallow corrections
        // take the fewest iterations in total: on the 400 x 40 bar 1204
        // against 1453 at 1e-3 or 1e-4 and 1654 at 3e-2).  Mixed, NP law: each
        // Newton system to 1e-4 relative (looser systems cost Newton steps:
        // 6 steps and 1887 iterations at 1e-2 against 4 and 1588).  NP: the
        // Newton system to 1e-6 relative or the final target, the looser of
        // the two, keeps Newton's convergence fast.
        double target = mixed ? (np ? 1e-4 : 1e-2) * std::sqrt(rr) : 0.5 * rtol * bnorm;
        if (np) target = std::max(target, 1e-6 * std::sqrt(rr));
        if (np) {
            // the tangent's bond factors at this Newton iterate
            if (dim == 3)
                bond_factor_k<3><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(
                    n, nbr->row_ptr, nbr->col, w.xv, w.u, mat->beta, w.kb);
            else
                bond_factor_k<2><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(
                    n, nbr->row_ptr, nbr->col, w.xv, w.u, mat->beta, w.kb);
            PD_LAUNCH_CHECK(ctx);
        }
        int k = 0;
        if (mixed) {
            PD_TRY(cg_solve(ctx, nbr, mat, w, w.v32, w.r, m, target, maxit - inner_total, &k));
            add_k<float><<<gm, PD_BLOCK, 0, ctx->stream>>>(w.u, w.v32.x, m);
        } else {
            PD_TRY(cg_solve(ctx, nbr, mat, w, w.v64, w.r, m, target, maxit - inner_total, &k));
            add_k<double><<<gm, PD_BLOCK, 0, ctx->stream>>>(w.u, w.v64.x, m);
        }
        PD_LAUNCH_CHECK(ctx);
        inner_total += k;
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
