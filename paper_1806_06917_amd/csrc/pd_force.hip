// Bond-force gather (Algorithm 1, linearised law, J = 1) with the fused
// critical-stretch damage test, and the velocity-Verlet step built on it
// (Section "Explicit time integration").
//
// One group of L lanes (L | 64, so a group never straddles a wavefront)
// owns one node i in sfc order.  Lane l walks bonds row_ptr[i] + l,
// + l + L, ... : the column and flag streams are read contiguously by the
// group, the neighbour records XV[j], u[j] are gathered (neighbours of
// consecutive sfc nodes overlap, so these mostly hit L2).  The L partial sums
// are combined pairwise (neighbouring lanes first, group_reduce), so the
// order of the per-node sum depends only on L and on the row, never on the
// rest of the mesh.  Lane 0 then applies the node update selected by `mode`;
// the kernel boundary is the global synchronisation between the drift of one
// step and the gather of the next (the displacement is double-buffered).
//
// FP64 mode: every bond operation in float64.  Mixed mode: the same float64
// arithmetic except 1/|xi|, which is the hardware reciprocal-square-root
// estimate (relative error below 2^-22).
#include <cmath>

#include "pd_kernels.hpp"

namespace {

using namespace pdk;

// Gather kernel: bond columns are sfc ids, neighbour records come straight
// from global memory (L2).  Used for rows too long for the LDS tiles and as
// the reference layout.
template <int DIM, int L, bool MIXED, bool WANT_E>
__global__ __launch_bounds__(PD_BLOCK) void node_kernel(NodeArgs a) {
    if (a.done && *a.done) return;
    const uint32_t tile = pd_xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t gid = tile * PD_BLOCK + threadIdx.x;
    const uint32_t i = gid / L;
    const int lane = threadIdx.x & (L - 1);
    const bool valid = i < a.n;
    const bool tangent = a.mode == M_TANGENT;

    double xix = 0, xiy = 0, xiz = 0, Vi = 0, uix = 0, uiy = 0, uiz = 0;
    Acc64 s64;
    bool fixed_i = false;
    if (valid) {
        const double4 q = reinterpret_cast<const double4 *>(a.xv)[i];
        xix = q.x; xiy = q.y;
        if (DIM == 3) { xiz = q.z; Vi = q.w; } else { Vi = q.z; }
        load_vec<DIM>(a.u, i, uix, uiy, uiz);
        if (tangent && a.bc) fixed_i = a.bc[i] != 0;
        if (tangent && fixed_i) { uix = 0; uiy = 0; uiz = 0; }
        const uint32_t rs = a.row_ptr[i], re = a.row_ptr[i + 1];
        if (a.law == PD_LAW_LINEAR && a.stretch == PD_STRETCH_LINEARISED && !(a.pv_h > 0.0) &&
            !(a.j_c2 > 0.0)) {
            for (uint32_t p = rs + lane; p < re; p += L) {
                // a dead bond adds exact zeros, like the tile kernel's dummy record
                const uint32_t j = (uint32_t)a.col[p];
                const bool live = !a.alive || a.alive[p];
                const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
                double ujx, ujy, ujz;
                load_vec<DIM>(a.u, j, ujx, ujy, ujz);
                if (tangent && a.bc && a.bc[j]) { ujx = 0; ujy = 0; ujz = 0; }
                const double cVj = a.cv_uniform != 0.0 ? a.cv_uniform : a.c * (DIM == 3 ? xj.w : xj.z);
                const double dxz = DIM == 3 ? xj.z - xiz : 0.0, duz = DIM == 3 ? ujz - uiz : 0.0;
                if (bond<DIM, MIXED, WANT_E>(a.damage, a.s_c, xj.x - xix, xj.y - xiy, dxz, ujx - uix,
                                             ujy - uiy, duz, cVj, !live, s64))
                    a.alive[p] = 0;
            }
        } else if (DIM == 3 && a.law == PD_LAW_LPS) {
            // linear peridynamic solid: the scatter of the paper read from
            // node i, f_i = sum_j (t_ij + t_ji) M V_j, with {m, theta} of
            // both ends from the state pass
            const double2 si = reinterpret_cast<const double2 *>(a.lps)[i];
            const LpsCoef qi = lps_coef<MIXED>(si.x, si.y, a.bulk, a.shear);
            const double hi = si.x > 0.0 ? si.y / 3.0 : 0.0;    // theta_i / 3
            for (uint32_t p = rs + lane; p < re; p += L) {
                const uint32_t j = (uint32_t)a.col[p];
                const bool live = !a.alive || a.alive[p];
                const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
                double ujx, ujy, ujz;
                load_vec<DIM>(a.u, j, ujx, ujy, ujz);
                const double dxx = xj.x - xix, dxy = xj.y - xiy, dxz = xj.z - xiz;
                const double dux = ujx - uix, duy = ujy - uiy, duz = ujz - uiz;
                double r2, qb, w;
                lps_terms<MIXED>(dxx, dxy, dxz, dux, duy, duz, r2, qb, w);
                const double2 sj = reinterpret_cast<const double2 *>(a.lps)[j];
                const LpsCoef qj = lps_coef<MIXED>(sj.x, sj.y, a.bulk, a.shear);
                // |xi| for partial volumes and the energy only
                const double len = (a.pv_h > 0.0 || WANT_E) ? lps_len<MIXED>(r2) : 0.0;
                const double Vj =
                    a.vol_uniform > 0.0 ? 1.0 : xj.w * pv_weight(len, a.pv_R, a.pv_h);
                const double g = lps_force_weight(qi, qj, r2, qb, w, Vj, live);
                s64.x = fma(g, dxx + dux, s64.x);
                s64.y = fma(g, dxy + duy, s64.y);
                s64.z = fma(g, dxz + duz, s64.z);
                if (WANT_E) {
                    const double edi = w / len - hi * len;    // e - theta_i |xi| / 3
                    s64.e += live ? edi * edi * Vj : 0.0;
                }
            }
        } else {
            // general law; the tangent's linearisation point, if any
            const bool lin = tangent && a.u_lin;
            double lix = 0, liy = 0, liz = 0;
            if (lin) load_vec<DIM>(a.u_lin, i, lix, liy, liz);
            for (uint32_t p = rs + lane; p < re; p += L) {
                const uint32_t j = (uint32_t)a.col[p];
                const bool live = !a.alive || a.alive[p];
                const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
                double ujx, ujy, ujz, ljx = 0, ljy = 0, ljz = 0;
                load_vec<DIM>(a.u, j, ujx, ujy, ujz);
                if (tangent && a.bc && a.bc[j]) { ujx = 0; ujy = 0; ujz = 0; }
                if (lin) load_vec<DIM>(a.u_lin, j, ljx, ljy, ljz);
                const double cVj = a.cv_uniform != 0.0 ? a.cv_uniform : a.c * (DIM == 3 ? xj.w : xj.z);
                const double dxz = DIM == 3 ? xj.z - xiz : 0.0, duz = DIM == 3 ? ujz - uiz : 0.0;
                if (bond_law<DIM, MIXED, WANT_E>(a.law, a.stretch, a.beta, a.damage, a.s_c, tangent,
                                                 xj.x - xix, xj.y - xiy, dxz, ujx - uix, ujy - uiy,
                                                 duz, ljx - lix, ljy - liy, ljz - liz, cVj, !live,
                                                 s64, a.pv_h, a.pv_R, a.j_c1, a.j_c2,
                                                 a.j_idelta))
                    a.alive[p] = 0;
            }
        }
    }
    double fx, fy, fz, Ue;
    group_reduce<DIM, L, WANT_E>(s64, fx, fy, fz, Ue);
    if (!valid || lane != 0) return;
    if (DIM == 3 && a.law == PD_LAW_LPS && a.vol_uniform > 0.0) {
        // the solid's bond terms left the uniform volume out
        fx = fx * a.vol_uniform;
        fy = fy * a.vol_uniform;
        fz = fz * a.vol_uniform;
        Ue = Ue * a.vol_uniform;
    }
    if (WANT_E && DIM == 3 && a.law == PD_LAW_LPS) {
        const double2 si = reinterpret_cast<const double2 *>(a.lps)[i];
        Ue = si.x > 0.0 ? 0.5 * a.bulk * si.y * si.y + 7.5 * a.shear / si.x * Ue : 0.0;
    }
    double vx = 0, vy = 0, vz = 0;
    if (mode_reads_v(a.mode)) load_vec<DIM>(a.v, i, vx, vy, vz);
    const int kind = a.bc ? a.bc[i] : PD_BC_FREE;
    node_update<DIM>(a, i, fx, fy, fz, Ue, Vi, uix, uiy, uiz, fixed_i, vx, vy, vz, kind);
}

// The gather kernel in PD_FP32 (linearised law only): float32 bond terms
// after the float64 differences, compensated float32 lane sums, the same
// rows, lanes and reduction order, then the float64 node update.
template <int DIM, int L, bool WANT_E>
__global__ __launch_bounds__(PD_BLOCK) void node_kernel32(NodeArgs a) {
    if (a.done && *a.done) return;
    const uint32_t tile = pd_xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t i = (tile * PD_BLOCK + threadIdx.x) / L;
    const int lane = threadIdx.x & (L - 1);
    const bool valid = i < a.n;
    double xix = 0, xiy = 0, xiz = 0, Vi = 0, uix = 0, uiy = 0, uiz = 0;
    AccC acc;
    if (valid) {
        const double4 q = reinterpret_cast<const double4 *>(a.xv)[i];
        xix = q.x; xiy = q.y;
        if (DIM == 3) { xiz = q.z; Vi = q.w; } else { Vi = q.z; }
        load_vec<DIM>(a.u, i, uix, uiy, uiz);
        const float sc = (float)a.s_c;
        // bond p's float32 terms (all +0 past the row's end)
        auto terms = [&](uint32_t p, uint32_t pe, float &tx, float &ty, float &tz, float &te) {
            if (p >= pe) {
                tx = ty = tz = te = 0.0f;
                return;
            }
            const uint32_t j = (uint32_t)a.col[p];
            const bool live = !a.alive || a.alive[p];
            const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
            double ujx, ujy, ujz;
            load_vec<DIM>(a.u, j, ujx, ujy, ujz);
            const float cVj = (float)(a.cv_uniform != 0.0 ? a.cv_uniform
                                                           : a.c * (DIM == 3 ? xj.w : xj.z));
            const double dxz = DIM == 3 ? xj.z - xiz : 0.0, duz = DIM == 3 ? ujz - uiz : 0.0;
            if (bond32<DIM, WANT_E>(a.damage, sc, xj.x - xix, xj.y - xiy, dxz, ujx - uix,
                                    ujy - uiy, duz, cVj, !live, tx, ty, tz, te))
                a.alive[p] = 0;
        };
        // the lane's bonds two at a time (p and p + L), as the streamed kernel
        const uint32_t pe = a.row_ptr[i + 1];
        for (uint32_t p = a.row_ptr[i] + lane; p < pe; p += 2 * L) {
            float ax, ay, az, ae, bx, by, bz, be;
            terms(p, pe, ax, ay, az, ae);
            terms(p + L, pe, bx, by, bz, be);
            pair_into<DIM, WANT_E>(acc, ax, ay, az, ae, bx, by, bz, be);
        }
    }
    double fx, fy, fz, Ue;
    group_reduce_c<DIM, L, WANT_E>(acc, fx, fy, fz, Ue);
    if (!valid || lane != 0) return;
    double vx = 0, vy = 0, vz = 0;
    if (mode_reads_v(a.mode)) load_vec<DIM>(a.v, i, vx, vy, vz);
    const int kind = a.bc ? a.bc[i] : PD_BC_FREE;
    node_update<DIM>(a, i, fx, fy, fz, Ue, Vi, uix, uiy, uiz, false, vx, vy, vz, kind);
}

// Linear peridynamic solid, first pass (Algorithm 2, weighted volume and
// dilatation): per node m_i = sum |xi|^2 V_j and theta_i = (3/m_i) sum |xi| e V_j
// over live bonds, stored as {m, theta} in a.lps.
template <int L, bool MIXED>
__global__ __launch_bounds__(PD_BLOCK) void lps_state_k(NodeArgs a) {
    const uint32_t tile = pd_xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t i = (tile * PD_BLOCK + threadIdx.x) / L;
    const int lane = threadIdx.x & (L - 1);
    const bool valid = i < a.n;
    double m = 0.0, s = 0.0;
    if (valid) {
        const double4 q = reinterpret_cast<const double4 *>(a.xv)[i];
        double uix, uiy, uiz;
        load_vec<3>(a.u, i, uix, uiy, uiz);
        for (uint32_t p = a.row_ptr[i] + lane; p < a.row_ptr[i + 1]; p += L) {
            if (a.alive && !a.alive[p]) continue;
            const uint32_t j = (uint32_t)a.col[p];
            const double4 xj = reinterpret_cast<const double4 *>(a.xv)[j];
            double ujx, ujy, ujz;
            load_vec<3>(a.u, j, ujx, ujy, ujz);
            double r2, qb, w;
            lps_terms<MIXED>(xj.x - q.x, xj.y - q.y, xj.z - q.z, ujx - uix, ujy - uiy,
                             ujz - uiz, r2, qb, w);
            const double Vj = a.vol_uniform > 0.0
                                  ? 1.0
                                  : xj.w * pv_weight(a.pv_h > 0.0 ? lps_len<MIXED>(r2) : 0.0,
                                                     a.pv_R, a.pv_h);
            lps_state_terms(r2, w, Vj, m, s);
        }
    }
    m = lane_sum<L>(m);
    s = lane_sum<L>(s);
    if (a.vol_uniform > 0.0) {      // the uniform volume, applied once per node
        m = m * a.vol_uniform;
        s = s * a.vol_uniform;
    }
    if (valid && lane == 0)
        reinterpret_cast<double2 *>(a.lps)[i] = make_double2(m, m > 0.0 ? 3.0 / m * s : 0.0);
}

template <int L>
int launch_lps_l(pd_ctx ctx, const NodeArgs &a, bool mixed) {
    const unsigned grid = pd_blocks((uint64_t)a.n * L);
    if (grid == 0) return PD_OK;
    if (mixed) lps_state_k<L, true><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
    else lps_state_k<L, false><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int launch_lps_state(pd_ctx ctx, const NodeArgs &a, int lanes, bool mixed) {
    switch (lanes) {
    case 1: return launch_lps_l<1>(ctx, a, mixed);
    case 2: return launch_lps_l<2>(ctx, a, mixed);
    case 4: return launch_lps_l<4>(ctx, a, mixed);
    case 8: return launch_lps_l<8>(ctx, a, mixed);
    case 16: return launch_lps_l<16>(ctx, a, mixed);
    case 32: return launch_lps_l<32>(ctx, a, mixed);
    case 64: return launch_lps_l<64>(ctx, a, mixed);
    default: return pd_set_error(ctx, PD_EINVAL, "unsupported lane count %d", lanes);
    }
}

// notch pre-crack: orientation tests in float64 without contraction, end
// points of the bond in lexicographic order so (i,j) and (j,i) agree
__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx,
                                         double cy) {
#pragma clang fp contract(off)
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}
__device__ __forceinline__ int sgn(double x) { return (x > 0.0) - (x < 0.0); }

__device__ bool segments_meet(double px, double py, double qx, double qy, double ax, double ay,
                              double bx, double by) {
    if (qx < px || (qx == px && qy < py)) {
        double t = px; px = qx; qx = t;
        t = py; py = qy; qy = t;
    }
    const int o1 = sgn(orient(ax, ay, bx, by, px, py));
    const int o2 = sgn(orient(ax, ay, bx, by, qx, qy));
    const int o3 = sgn(orient(px, py, qx, qy, ax, ay));
    const int o4 = sgn(orient(px, py, qx, qy, bx, by));
    if (o1 == 0 && o2 == 0 && o3 == 0 && o4 == 0)
        return fmax(fmin(px, qx), fmin(ax, bx)) <= fmin(fmax(px, qx), fmax(ax, bx)) &&
               fmax(fmin(py, qy), fmin(ay, by)) <= fmin(fmax(py, qy), fmax(ay, by));
    return o1 * o2 <= 0 && o3 * o4 <= 0;
}

struct NotchSegs {
    double s[8][4];
};

__global__ void notch_k(uint32_t n, const double *xv, const uint32_t *row_ptr, const int32_t *col,
                        int nseg, NotchSegs segs, uint8_t *alive) {
    const uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const uint32_t lane = threadIdx.x % 64;
    if (i >= n) return;
    const double4 P = reinterpret_cast<const double4 *>(xv)[i];
    for (uint32_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) {
        const double4 Q = reinterpret_cast<const double4 *>(xv)[col[p]];
        for (int s = 0; s < nseg; ++s)
            if (segments_meet(P.x, P.y, Q.x, Q.y, segs.s[s][0], segs.s[s][1], segs.s[s][2],
                              segs.s[s][3]))
                alive[p] = 0;
    }
}

template <int DIM, int L>
int launch_t(pd_ctx ctx, const NodeArgs &a, bool mixed) {
    const unsigned grid = pd_blocks((uint64_t)a.n * L);
    if (grid == 0) return PD_OK;
    const bool e = mode_wants_energy(a);
    if (a.fp32) {
        if (e) node_kernel32<DIM, L, true><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
        else node_kernel32<DIM, L, false><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
    } else if (mixed) {
        if (e) node_kernel<DIM, L, true, true><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
        else node_kernel<DIM, L, true, false><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
    } else {
        if (e) node_kernel<DIM, L, false, true><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
        else node_kernel<DIM, L, false, false><<<grid, PD_BLOCK, 0, ctx->stream>>>(a);
    }
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

template <int DIM>
int launch_d(pd_ctx ctx, const NodeArgs &a, int lanes, bool mixed) {
    switch (lanes) {
    case 1: return launch_t<DIM, 1>(ctx, a, mixed);
    case 2: return launch_t<DIM, 2>(ctx, a, mixed);
    case 4: return launch_t<DIM, 4>(ctx, a, mixed);
    case 8: return launch_t<DIM, 8>(ctx, a, mixed);
    case 16: return launch_t<DIM, 16>(ctx, a, mixed);
    case 32: return launch_t<DIM, 32>(ctx, a, mixed);
    case 64: return launch_t<DIM, 64>(ctx, a, mixed);
    default: return pd_set_error(ctx, PD_EINVAL, "unsupported lane count %d", lanes);
    }
}

}  // namespace

int pd_launch_gather(pd_ctx ctx, int dim, const NodeArgs &a, int lanes, bool mixed) {
    return dim == 3 ? launch_d<3>(ctx, a, lanes, mixed) : launch_d<2>(ctx, a, lanes, mixed);
}

static bool tile_fits(pd_ctx ctx, const pd_nbr nbr, int lanes, int block) {
    return pd_tile_resident(nbr->dim, nbr->ntiles, nbr->tile_T, pd_tile_hcap(nbr),
                            pd_tile_bcap(nbr), lanes, block, ctx->num_cu);
}

// the streamed kernel of this form can run on the tiles nbr holds now
static bool stream_form_fits(pd_ctx ctx, const pd_nbr nbr, int lanes, int prec, int form) {
    int b = 0;
    unsigned g = 0;
    uint32_t m = 0;
    size_t l = 0;
    return nbr->lcol && pd_stream_fits(nbr->dim, nbr->n, nbr->nnz, nbr->halo_total) &&
           pd_stream_geometry(ctx, nbr->dim, nbr->ntiles, nbr->tile_T, pd_tile_hcap(nbr),
                              pd_tile_bcap(nbr), lanes, prec, false, form, &b, &g, &m, &l);
}

// threads per tile workgroup for the tiles nbr holds now: the tuning value,
// else one lane group per tile node (measured best on the 1M-node cube and
// the 512^2 plate), doubled while the halo or the bond words of the largest
// tile need more threads than that to stage
static int tile_block(pd_ctx ctx, const pd_nbr nbr, int lanes) {
    if (ctx->block) return ctx->block;
    int block = (int)nbr->tile_T * lanes;
    block = block < 256 ? 256 : (block > 1024 ? 1024 : block);
    while (block < 1024 && !tile_fits(ctx, nbr, lanes, block)) block *= 2;
    return block;
}

// Chooses the kernel for one call site: *block > 0 selects the LDS tile
// kernel with that many threads per workgroup (tiles built, or rebuilt at the
// requested or automatic size and then halved, until one layout fits),
// *block = 0 the plain gather kernel.  A layout used by live simulations is
// never rebuilt.
int pd_plan_kernel(pd_ctx ctx, pd_nbr nbr, int lanes, int *block) {
    *block = 0;
    const bool forced = ctx->kernel == 2;
    if (ctx->kernel == 1) return PD_OK;
    if (lanes < 2 || lanes > 32) {
        if (forced) return pd_set_error(ctx, PD_EINVAL, "the tile kernel needs 2..32 lanes");
        return PD_OK;
    }
    if (nbr->lcol && nbr->users > 0) {
        const int B = tile_block(ctx, nbr, lanes);
        if (tile_fits(ctx, nbr, lanes, B)) *block = B;
        else if (forced) return pd_set_error(ctx, PD_ECAPACITY, "tile layout does not fit");
        return PD_OK;
    }
    const uint64_t key = ((uint64_t)(uint32_t)ctx->tile << 32) ^ ((uint64_t)ctx->block << 8) ^
                         (uint64_t)lanes;
    if (nbr->fail_key == key + 1) {
        if (forced) return pd_set_error(ctx, PD_ECAPACITY, "tile layout does not fit in LDS");
        return PD_OK;
    }
    uint32_t T = ctx->tile ? (uint32_t)ctx->tile : 128u;
    for (; T >= 16; T >>= 1) {
        if (!(nbr->lcol && nbr->tile_T == T)) {
            const int st = pd_nbr_build_tiles(ctx, nbr, T);
            if (st != PD_OK && st != PD_ECAPACITY) return st;
            if (st == PD_ECAPACITY) {
                if (ctx->tile) break;
                continue;
            }
        }
        const int B = tile_block(ctx, nbr, lanes);
        if (tile_fits(ctx, nbr, lanes, B)) {
            *block = B;
            return PD_OK;
        }
        if (ctx->tile) break;
    }
    nbr->fail_key = key + 1;
    if (forced) return pd_set_error(ctx, PD_ECAPACITY, "tile layout does not fit in LDS");
    return PD_OK;
}

namespace {

// block > 0 (with a.bw set): tile kernel; otherwise the gather kernel
int launch_node(pd_ctx ctx, const pd_nbr nbr, NodeArgs a, int lanes, bool mixed, int block) {
    if (block > 0 && a.bw && !a.fp32) {
        a.halo_ptr = nbr->halo_ptr;
        a.halo = nbr->halo;
        a.self_off = nbr->self_off;
        a.tile = nbr->tile_T;
        a.ntiles = nbr->ntiles;
        a.hcap = pd_tile_hcap(nbr);
        a.bcap = pd_tile_bcap(nbr);
        return pd_launch_tile(ctx, nbr->dim, a, lanes, mixed, block);
    }
    a.bw = nullptr;
    // the solid's state pass at the same displacement, then the force pass
    if (nbr->dim == 3 && a.law == PD_LAW_LPS) PD_TRY(launch_lps_state(ctx, a, lanes, mixed));
    return pd_launch_gather(ctx, nbr->dim, a, lanes, mixed);
}

int check_material(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat) {
    if (!mat) return pd_set_error(ctx, PD_EINVAL, "material must not be NULL");
    if (mat->dim != nbr->dim) return pd_set_error(ctx, PD_EINVAL, "material dim != neighbour dim");
    if (mat->precision != PD_FP64 && mat->precision != PD_MIXED && mat->precision != PD_FP32)
        return pd_set_error(ctx, PD_EINVAL, "precision must be PD_FP64, PD_MIXED or PD_FP32");
    if (mat->precision == PD_FP32 && pd_general_law(mat))
        return pd_set_error(ctx, PD_EINVAL, "PD_FP32 takes the linearised law only");
    if (!std::isfinite(mat->c) || !std::isfinite(mat->s_c))
        return pd_set_error(ctx, PD_EINVAL, "c and s_c must be finite");
    if (mat->j_c2 > 0.0 && !(nbr->delta - 0.5 * mat->pv_h > 0.0))
        return pd_set_error(ctx, PD_EINVAL, "the influence function needs radius - pv_h/2 > 0");
    return pd_check_law(ctx, mat);
}

NodeArgs base_args(const pd_nbr nbr, const pd_material *mat) {
    NodeArgs a{};
    a.fp32 = mat->precision == PD_FP32;
    a.row_ptr = nbr->row_ptr;
    a.col = nbr->col;
    a.n = nbr->n;
    a.c = mat->c;
    a.s_c = mat->s_c;
    a.rho = mat->rho;
    a.law = mat->law;
    a.stretch = mat->stretch;
    a.beta = mat->beta;
    a.bulk = mat->bulk;
    a.shear = mat->shear;
    a.pv_h = mat->pv_h;
    a.pv_R = nbr->delta;
    a.j_c1 = mat->j_c1;
    a.j_c2 = mat->j_c2;
    a.j_idelta = mat->j_c2 > 0.0 ? 1.0 / (nbr->delta - 0.5 * mat->pv_h) : 0.0;
    return a;
}

int ensure_scratch(pd_ctx ctx, pd_nbr nbr) {
    const int us = nbr->dim == 3 ? 4 : 2;
    if (!nbr->s_xv) PD_TRY(pd_alloc(ctx, &nbr->s_xv, (size_t)nbr->n * 4));
    if (!nbr->s_u) PD_TRY(pd_alloc(ctx, &nbr->s_u, (size_t)nbr->n * us));
    if (!nbr->s_f) PD_TRY(pd_alloc(ctx, &nbr->s_f, (size_t)nbr->n * us));
    if (!nbr->s_U) PD_TRY(pd_alloc(ctx, &nbr->s_U, (size_t)nbr->n));
    if (!nbr->s_alive) PD_TRY(pd_alloc(ctx, &nbr->s_alive, nbr->nnz));
    if (!nbr->s_fixed) PD_TRY(pd_alloc(ctx, &nbr->s_fixed, (size_t)nbr->n));
    if (!nbr->s_bw && nbr->lcol) PD_TRY(pd_alloc(ctx, &nbr->s_bw, nbr->nnz + PD_BW_PAD));
    return PD_OK;
}

double ramp_factor(double s, int64_t ramp) {
    if (ramp <= 0) return 1.0;
    const double r = s / (double)ramp;
    return r < 1.0 ? r : 1.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// stateless force evaluation
// ---------------------------------------------------------------------------
int pd_check_force_args(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                        const double *V, const double *u, const uint8_t *alive, const double *f,
                        const double *U) {
    if (!nbr) return pd_set_error(ctx, PD_EINVAL, "nbr must not be NULL");
    if (nbr->closing) return pd_set_error(ctx, PD_EINVAL, "nbr has been destroyed");
    if (nbr->nnz == 0)
        return pd_set_error(ctx, PD_EINVAL, "the mesh has no bonds (no two nodes within delta)");
    PD_TRY(pd_check_ctx(ctx));
    if (nbr->ctx != ctx) return pd_set_error(ctx, PD_EINVAL, "nbr belongs to another context");
    PD_TRY(check_material(ctx, nbr, mat));
    PD_TRY(pd_check_dev_ptr(ctx, X, "X"));
    PD_TRY(pd_check_dev_ptr(ctx, V, "V"));
    PD_TRY(pd_check_dev_ptr(ctx, u, "u"));
    PD_TRY(pd_check_dev_ptr(ctx, f, "f"));
    if (alive) PD_TRY(pd_check_dev_ptr(ctx, alive, "alive"));
    if (U) PD_TRY(pd_check_dev_ptr(ctx, U, "U"));
    return PD_OK;
}

size_t pd_force_bufs_bytes(const pd_nbr nbr, const pd_material *mat) {
    const size_t n = nbr->n, us = nbr->dim == 3 ? 4 : 2;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = up(n * 4 * 8) + 2 * up(n * us * 8) + up(n * 8) + up(nbr->nnz);
    if (mat->law == PD_LAW_LPS) bytes += up(n * 2 * 8);
    return bytes;
}

pd_force_bufs pd_force_bufs_carve(const pd_nbr nbr, const pd_material *mat, void *base) {
    const size_t n = nbr->n, us = nbr->dim == 3 ? 4 : 2;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    unsigned char *q = static_cast<unsigned char *>(base);
    pd_force_bufs b{};
    b.xv = reinterpret_cast<double *>(q);
    q += up(n * 4 * 8);
    b.u = reinterpret_cast<double *>(q);
    q += up(n * us * 8);
    b.f = reinterpret_cast<double *>(q);
    q += up(n * us * 8);
    b.U = reinterpret_cast<double *>(q);
    q += up(n * 8);
    b.alive = q;
    q += up(nbr->nnz);
    b.lps = mat->law == PD_LAW_LPS ? reinterpret_cast<double *>(q) : nullptr;
    return b;
}

// The force evaluation of pd_internal_force on the gather kernel, with the
// internal-order copies in the caller's buffers (allocates nothing; arguments
// already checked)
int pd_force_gather(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                    const double *V, const double *u, uint8_t *alive, double *f, double *U,
                    const pd_force_bufs &b) {
    const int lanes = pd_auto_lanes(ctx, nbr->nnz, nbr->n);
    PD_TRY(pd_gather_xv(ctx, nbr, X, V, b.xv));
    PD_TRY(pd_gather_vec(ctx, nbr, u, b.u, false));
    if (alive) PD_TRY(pd_alive_in(ctx, nbr, alive, b.alive));
    NodeArgs a = base_args(nbr, mat);
    a.xv = b.xv;
    a.u = b.u;
    a.alive = alive ? b.alive : nullptr;
    a.bw = nullptr;
    a.damage = alive && mat->s_c > 0.0;
    a.f_out = b.f;
    a.e_out = U ? b.U : nullptr;
    a.mode = M_FORCE;
    a.lps = b.lps;
    PD_TRY(launch_node(ctx, nbr, a, lanes, mat->precision == PD_MIXED, 0));
    PD_TRY(pd_scatter_vec(ctx, nbr, b.f, f));
    if (U) PD_TRY(pd_scatter_scalar(ctx, nbr, b.U, U));
    if (alive && a.damage) PD_TRY(pd_alive_out(ctx, nbr, b.alive, alive));
    return PD_OK;
}

extern "C" int pd_internal_force(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                                 const double *V, const double *u, uint8_t *alive, double *f,
                                 double *U) {
    PD_TRY(pd_check_force_args(ctx, nbr, mat, X, V, u, alive, f, U));
    const int lanes = pd_auto_lanes(ctx, nbr->nnz, nbr->n);
    int block = 0;
    if (!pd_general_law(mat) && mat->precision != PD_FP32)
        PD_TRY(pd_plan_kernel(ctx, nbr, lanes, &block));
    PD_TRY(ensure_scratch(ctx, nbr));
    const bool tiled = block > 0;
    PD_TRY(pd_gather_xv(ctx, nbr, X, V, nbr->s_xv));
    PD_TRY(pd_gather_vec(ctx, nbr, u, nbr->s_u, false));
    if (alive) PD_TRY(pd_alive_in(ctx, nbr, alive, nbr->s_alive));
    if (tiled) PD_TRY(pd_bw_compose(ctx, nbr, alive ? nbr->s_alive : nullptr, nbr->s_bw));
    NodeArgs a = base_args(nbr, mat);
    a.xv = nbr->s_xv;
    a.u = nbr->s_u;
    a.alive = alive ? nbr->s_alive : nullptr;
    a.bw = tiled ? nbr->s_bw : nullptr;
    a.damage = alive && mat->s_c > 0.0;
    a.f_out = nbr->s_f;
    a.e_out = U ? nbr->s_U : nullptr;
    a.mode = M_FORCE;
    if (mat->law == PD_LAW_LPS) {
        if (!nbr->s_lps) PD_TRY(pd_alloc(ctx, &nbr->s_lps, (size_t)nbr->n * 2));
        a.lps = nbr->s_lps;
    }
    PD_TRY(launch_node(ctx, nbr, a, lanes, mat->precision == PD_MIXED, block));
    PD_TRY(pd_scatter_vec(ctx, nbr, nbr->s_f, f));
    if (U) PD_TRY(pd_scatter_scalar(ctx, nbr, nbr->s_U, U));
    if (alive && a.damage) {
        if (tiled) PD_TRY(pd_bw_to_alive(ctx, nbr, nbr->s_bw, nbr->s_alive));
        PD_TRY(pd_alive_out(ctx, nbr, nbr->s_alive, alive));
    }
    return PD_OK;
}

// ---------------------------------------------------------------------------
// tangent operator (used by the implicit solver as well)
// ---------------------------------------------------------------------------
int pd_tangent_sfc(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, const double *xv,
                   const uint8_t *alive_sfc, uint16_t *bw, int block, const uint8_t *fixed_sfc,
                   const double *w, double *y, const int *done, const double *u_lin) {
    NodeArgs a = base_args(nbr, mat);
    a.done = done;
    a.u_lin = mat->law == PD_LAW_NP ? u_lin : nullptr;
    a.xv = xv;
    a.u = w;
    a.alive = const_cast<uint8_t *>(alive_sfc);
    a.bw = bw;
    a.damage = 0;
    a.bc = fixed_sfc;
    a.f_out = y;
    a.mode = M_TANGENT;
    return launch_node(ctx, nbr, a, pd_auto_lanes(ctx, nbr->nnz, nbr->n),
                       mat->precision == PD_MIXED, block);
}

// internal force in sfc order, no damage: f = force(u) (implicit residuals)
int pd_force_sfc(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, const double *xv,
                 const uint8_t *alive_sfc, uint16_t *bw, int block, const double *u, double *f) {
    NodeArgs a = base_args(nbr, mat);
    a.xv = xv;
    a.u = u;
    a.alive = const_cast<uint8_t *>(alive_sfc);
    a.bw = bw;
    a.damage = 0;
    a.f_out = f;
    a.mode = M_FORCE;
    return launch_node(ctx, nbr, a, pd_auto_lanes(ctx, nbr->nnz, nbr->n), false, block);
}

static int apply_tangent(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                         const double *V, const double *u, const uint8_t *alive,
                         const uint8_t *fixed, const double *w, double *y) {
    if (!nbr) return pd_set_error(ctx, PD_EINVAL, "nbr must not be NULL");
    if (nbr->closing) return pd_set_error(ctx, PD_EINVAL, "nbr has been destroyed");
    if (nbr->nnz == 0)
        return pd_set_error(ctx, PD_EINVAL, "the mesh has no bonds (no two nodes within delta)");
    PD_TRY(pd_check_ctx(ctx));
    if (nbr->ctx != ctx) return pd_set_error(ctx, PD_EINVAL, "nbr belongs to another context");
    PD_TRY(check_material(ctx, nbr, mat));
    if (mat->precision == PD_FP32)
        return pd_set_error(ctx, PD_EINVAL, "the tangent takes PD_FP64 or PD_MIXED");
    if (mat->stretch != PD_STRETCH_LINEARISED || mat->law == PD_LAW_LPS || mat->pv_h > 0.0 ||
        mat->j_c2 > 0.0)
        return pd_set_error(ctx, PD_EINVAL,
                            "the tangent takes a pairwise law with the linearised stretch only");
    PD_TRY(pd_check_dev_ptr(ctx, X, "X"));
    PD_TRY(pd_check_dev_ptr(ctx, V, "V"));
    PD_TRY(pd_check_dev_ptr(ctx, w, "w"));
    PD_TRY(pd_check_dev_ptr(ctx, y, "y"));
    if (u) PD_TRY(pd_check_dev_ptr(ctx, u, "u"));
    if (alive) PD_TRY(pd_check_dev_ptr(ctx, alive, "alive"));
    if (fixed) PD_TRY(pd_check_dev_ptr(ctx, fixed, "fixed"));
    const bool np = mat->law == PD_LAW_NP;
    int block = 0;
    if (!pd_general_law(mat))
        PD_TRY(pd_plan_kernel(ctx, nbr, pd_auto_lanes(ctx, nbr->nnz, nbr->n), &block));
    PD_TRY(ensure_scratch(ctx, nbr));
    const bool tiled = block > 0;
    if (np && !nbr->s_ulin) PD_TRY(pd_alloc(ctx, &nbr->s_ulin, (size_t)nbr->n * (nbr->dim == 3 ? 4 : 2)));
    PD_TRY(pd_gather_xv(ctx, nbr, X, V, nbr->s_xv));
    PD_TRY(pd_gather_vec(ctx, nbr, w, nbr->s_u, false));
    if (np) PD_TRY(pd_gather_vec(ctx, nbr, u, nbr->s_ulin, true));
    if (alive) PD_TRY(pd_alive_in(ctx, nbr, alive, nbr->s_alive));
    if (tiled) PD_TRY(pd_bw_compose(ctx, nbr, alive ? nbr->s_alive : nullptr, nbr->s_bw));
    if (fixed) PD_TRY(pd_gather_u8(ctx, nbr, fixed, nbr->s_fixed, 0));
    PD_TRY(pd_tangent_sfc(ctx, nbr, mat, nbr->s_xv, alive ? nbr->s_alive : nullptr,
                          tiled ? nbr->s_bw : nullptr, block, fixed ? nbr->s_fixed : nullptr,
                          nbr->s_u, nbr->s_f, nullptr, np ? nbr->s_ulin : nullptr));
    PD_TRY(pd_scatter_vec(ctx, nbr, nbr->s_f, y));
    return PD_OK;
}

extern "C" int pd_apply_tangent(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                                const double *V, const uint8_t *alive, const uint8_t *fixed,
                                const double *w, double *y) {
    return apply_tangent(ctx, nbr, mat, X, V, nullptr, alive, fixed, w, y);
}

extern "C" int pd_apply_tangent_at(pd_ctx ctx, pd_nbr nbr, const pd_material *mat,
                                   const double *X, const double *V, const double *u,
                                   const uint8_t *alive, const uint8_t *fixed, const double *w,
                                   double *y) {
    if (!u) return pd_set_error(ctx, PD_EINVAL, "u must not be NULL");
    return apply_tangent(ctx, nbr, mat, X, V, u, alive, fixed, w, y);
}

// ---------------------------------------------------------------------------
// resident explicit simulation
// ---------------------------------------------------------------------------
static void sim_release(pd_sim s) {
    if (!s) return;
    pd_free(s->xv);
    pd_free(s->u[0]);
    pd_free(s->u[1]);
    pd_free(s->v);
    pd_free(s->bc_vel);
    pd_free(s->b);
    pd_free(s->bc);
    pd_free(s->alive);
    pd_free(s->bw);
    pd_free(s->scratch);
    pd_free(s->rec[0]);
    pd_free(s->rec[1]);
    pd_free(s->lps);
    pd_free(s->lpsc);
    if (s->nbr && s->tiled) s->nbr->users -= 1;
    pd_ctx ctx = s->ctx;
    pd_nbr nbr = s->nbr;
    delete s;
    pd_nbr_unref(nbr);
    pd_ctx_unref(ctx);
}

static int lps_mass(pd_sim s);

extern "C" int pd_sim_create(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                             const double *V, const double *u0, const double *v0,
                             const uint8_t *bc_kind, const double *bc_vel, const double *b,
                             const double *notch, int nseg, int64_t ramp_steps, pd_sim *out) {
    if (!out) return pd_set_error(ctx, PD_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!nbr) return pd_set_error(ctx, PD_EINVAL, "nbr must not be NULL");
    if (nbr->closing) return pd_set_error(ctx, PD_EINVAL, "nbr has been destroyed");
    if (nbr->nnz == 0)
        return pd_set_error(ctx, PD_EINVAL, "the mesh has no bonds (no two nodes within delta)");
    PD_TRY(pd_check_ctx(ctx));
    if (nbr->ctx != ctx) return pd_set_error(ctx, PD_EINVAL, "nbr belongs to another context");
    PD_TRY(check_material(ctx, nbr, mat));
    if (!(mat->rho > 0.0) || !std::isfinite(mat->rho))
        return pd_set_error(ctx, PD_EINVAL, "rho must be finite and positive");
    PD_TRY(pd_check_dev_ptr(ctx, X, "X"));
    PD_TRY(pd_check_dev_ptr(ctx, V, "V"));
    if (u0) PD_TRY(pd_check_dev_ptr(ctx, u0, "u0"));
    if (v0) PD_TRY(pd_check_dev_ptr(ctx, v0, "v0"));
    if (bc_kind) PD_TRY(pd_check_dev_ptr(ctx, bc_kind, "bc_kind"));
    if (bc_kind && !bc_vel)
        return pd_set_error(ctx, PD_EINVAL, "bc_vel is required with bc_kind");
    if (bc_vel) PD_TRY(pd_check_dev_ptr(ctx, bc_vel, "bc_vel"));
    if (b) PD_TRY(pd_check_dev_ptr(ctx, b, "b"));
    if (nseg < 0 || nseg > 8) return pd_set_error(ctx, PD_EINVAL, "nseg must be in [0, 8]");
    if (nseg > 0 && (!notch || nbr->dim != 2))
        return pd_set_error(ctx, PD_EINVAL, "notch segments need dim 2 and a host array");
    if (ramp_steps < 0) return pd_set_error(ctx, PD_EINVAL, "ramp_steps must be >= 0");
    NotchSegs segs{};
    for (int s = 0; s < nseg; ++s)
        for (int k = 0; k < 4; ++k) {
            segs.s[s][k] = notch[4 * s + k];
            if (!std::isfinite(segs.s[s][k]))
                return pd_set_error(ctx, PD_EINVAL, "notch coordinates must be finite");
        }

    // automatic tuning: the autotuner's tile size and lane count for meshes
    // like this one, if it measured any (else the built-in heuristics); a
    // tuned tile size that does not fit this mesh falls back to automatic
    int lanes = pd_auto_lanes(ctx, nbr->nnz, nbr->n);
    int block = 0;
    const pd_tune_entry *te = nullptr;
    bool layout_only = false;
    // the NP law without damage also runs on the streamed kernel (its other
    // calls, and every other general law, on the gather kernel)
    const bool np_stream = mat->law == PD_LAW_NP && mat->stretch == PD_STRETCH_LINEARISED &&
                           !(mat->s_c > 0.0) && !(mat->pv_h > 0.0) && !(mat->j_c2 > 0.0);
    // so does the solid's explicit step (its two passes) without partial volumes
    const bool lps_stream = mat->law == PD_LAW_LPS && !(mat->pv_h > 0.0);
    const bool general = pd_general_law(mat) && !np_stream && !lps_stream;
    if (ctx->lanes == 0 && ctx->kernel == 0 && ctx->tile == 0 && ctx->block == 0 && nbr->n > 0)
        te = pd_tune_find(ctx, nbr->dim, (double)nbr->nnz / (double)nbr->n, mat->precision);
    if ((np_stream || lps_stream) && ctx->kernel == 2)
        return pd_set_error(ctx, PD_ECAPACITY, "the LDS tile kernel takes the linearised law only");
    if (mat->precision == PD_FP32 && ctx->kernel == 2)
        return pd_set_error(ctx, PD_ECAPACITY, "the LDS tile kernel has no PD_FP32 form");
    if (general) {
        if (ctx->kernel == 2 || ctx->kernel == 3)
            return pd_set_error(ctx, PD_ECAPACITY, "the tiled kernels take the linearised law only");
    } else if (te) {
        lanes = te->lanes;
        ctx->tile = te->tile;
        const int st = pd_plan_kernel(ctx, nbr, lanes, &block);
        ctx->tile = 0;
        PD_TRY(st);
        // tiles held at another size by a live simulation are not the tuned shape
        if (block > 0 && nbr->tile_T != (uint32_t)te->tile) block = 0;
        layout_only = block == 0 && nbr->lcol && nbr->tile_T == (uint32_t)te->tile;
        // the tuned shape (timed on the linearised law) must also fit this
        // material's streamed form (the solid stages more per halo node);
        // else the automatic choice
        if ((block > 0 || layout_only) && !stream_form_fits(ctx, nbr, lanes, mat->precision,
                                                            lps_stream ? SK_LPS_FORCE
                                                                       : (np_stream ? SK_NP
                                                                                    : SK_LINEAR))) {
            block = 0;
            layout_only = false;
        }
        // the tuned shape does not apply (it does not fit, or the tiles are
        // held at another size): the automatic lanes as well as tile size,
        // since the tuned lane count was timed with the tuned tiles
        if (block == 0 && !layout_only) {
            lanes = pd_auto_lanes(ctx, nbr->nnz, nbr->n);
            PD_TRY(pd_plan_kernel(ctx, nbr, lanes, &block));
        }
    } else {
        PD_TRY(pd_plan_kernel(ctx, nbr, lanes, &block));
        layout_only = block == 0 && ctx->tile != 0 && nbr->lcol &&
                      nbr->tile_T == (uint32_t)ctx->tile;
    }
    // tiles built at the requested size whose tile kernel cannot be resident
    // there still serve the streamed steps; the simulation's other calls then
    // run on the gather kernel (layout_only, dropped again if it cannot stream)
    if (general || !(ctx->kernel == 0 || ctx->kernel == 3)) layout_only = false;
    pd_sim s = new (std::nothrow) pd_sim_s();
    if (!s) return PD_ENOMEM;
    s->ctx = ctx;
    s->nbr = nbr;
    ctx->refs += 1;
    nbr->refs += 1;
    s->mat = *mat;
    s->ramp = ramp_steps;
    const size_t n = nbr->n, us = nbr->dim == 3 ? 4 : 2;
    int st = PD_OK;
    if (st == PD_OK) st = pd_alloc(ctx, &s->xv, n * 4);
    if (st == PD_OK) st = pd_alloc(ctx, &s->u[0], n * us);
    if (st == PD_OK) st = pd_alloc(ctx, &s->u[1], n * us);
    if (st == PD_OK) st = pd_alloc(ctx, &s->v, n * us);
    if (st == PD_OK) st = pd_alloc(ctx, &s->bc, n + 16);   // whole 32-bit words for copies
    if (st == PD_OK) st = pd_alloc(ctx, &s->alive, nbr->nnz);
    if (st == PD_OK) st = pd_alloc(ctx, &s->scratch, 2 * n);
    if (st == PD_OK && bc_vel) st = pd_alloc(ctx, &s->bc_vel, n * us);
    if (st == PD_OK && b) st = pd_alloc(ctx, &s->b, n * us);
    if (st == PD_OK && mat->law == PD_LAW_LPS) st = pd_alloc(ctx, &s->lps, n * 2);
    if (st == PD_OK) st = pd_gather_xv(ctx, nbr, X, V, s->xv);
    if (st == PD_OK) st = pd_gather_vec(ctx, nbr, u0, s->u[0], true);
    if (st == PD_OK) st = pd_gather_vec(ctx, nbr, v0, s->v, true);
    if (st == PD_OK) st = pd_gather_u8(ctx, nbr, bc_kind, s->bc, PD_BC_FREE);
    if (st == PD_OK && bc_vel) st = pd_gather_vec(ctx, nbr, bc_vel, s->bc_vel, true);
    if (st == PD_OK && b) st = pd_gather_vec(ctx, nbr, b, s->b, true);
    if (st == PD_OK) st = pd_alive_in(ctx, nbr, nullptr, s->alive);
    if (st == PD_OK && nseg > 0) {
        notch_k<<<pd_blocks((uint64_t)n * 64), PD_BLOCK, 0, ctx->stream>>>(
            nbr->n, s->xv, nbr->row_ptr, nbr->col, nseg, segs, s->alive);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = pd_hip_error(ctx, e, "notch_k", __FILE__, __LINE__);
    }
    s->lanes = lanes;
    // the tile kernel for the other calls (those of the NP law and the solid
    // run on the gather kernel)
    s->block = (np_stream || lps_stream || mat->precision == PD_FP32) ? 0 : block;
    if (st == PD_OK && (block > 0 || layout_only)) {
        s->tiled = true;
        nbr->users += 1;
        st = pd_alloc(ctx, &s->bw, nbr->nnz + PD_BW_PAD);
        if (st == PD_OK) st = pd_bw_compose(ctx, nbr, s->alive, s->bw);
    }
    if (st == PD_OK) {
        double Vu = 0.0;
        st = pd_uniform_volume(ctx, nbr, s->xv, &Vu);
        s->cv_uniform = mat->c * Vu;
        s->vol_uniform = Vu;
    }
    s->s_form = lps_stream ? SK_LPS_FORCE : (np_stream ? SK_NP : SK_LINEAR);
    if (st == PD_OK && s->tiled && (lps_stream ? s->vol_uniform > 0.0 : s->cv_uniform != 0.0) &&
        (ctx->kernel == 0 || ctx->kernel == 3) &&
        pd_stream_fits(nbr->dim, nbr->n, nbr->nnz, nbr->halo_total) &&
        pd_stream_geometry(ctx, nbr->dim, nbr->ntiles, nbr->tile_T, pd_tile_hcap(nbr),
                           pd_tile_bcap(nbr), lanes, mat->precision, false, s->s_form,
                           &s->s_block, &s->s_grid, &s->s_mmax, &s->s_lds) &&
        (!lps_stream ||
         pd_stream_geometry(ctx, nbr->dim, nbr->ntiles, nbr->tile_T, pd_tile_hcap(nbr),
                            pd_tile_bcap(nbr), lanes, mat->precision, false,
                            SK_LPS_STATE, &s->s2_block, &s->s2_grid, &s->s2_mmax,
                            &s->s2_lds))) {
        const size_t rd = nbr->dim == 3 ? 6 : 4;
        st = pd_alloc(ctx, &s->rec[0], n * rd);
        if (st == PD_OK) st = pd_alloc(ctx, &s->rec[1], n * rd);
        if (st == PD_OK && lps_stream) st = pd_alloc(ctx, &s->lpsc, n * 2);
        // both buffers carry the positions; u is rewritten every step
        if (st == PD_OK) st = pd_rec_pack(ctx, nbr->dim, nbr->n, s->xv, s->u[0], s->rec[0]);
        if (st == PD_OK) st = pd_rec_pack(ctx, nbr->dim, nbr->n, s->xv, s->u[0], s->rec[1]);
        s->stream = true;
        s->rec_stale = false;
    }
    if (st == PD_OK && block == 0 && s->tiled && !s->stream) {
        // tiles without a resident tile kernel and no streamed steps: all
        // calls on the gather kernel, with the flags (not bond words)
        nbr->users -= 1;
        pd_free(s->bw);
        s->bw = nullptr;
        s->tiled = false;
    }
    if (st == PD_OK && ctx->kernel == 3 && !s->stream)
        st = pd_set_error(ctx, PD_ECAPACITY, "the streamed kernel cannot run this simulation");
    if (st == PD_OK && s->stream && s->s_form == SK_LPS_FORCE) st = lps_mass(s);
    if (st == PD_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = pd_hip_error(ctx, e, "sim_create", __FILE__, __LINE__);
    }
    if (st != PD_OK) {
        sim_release(s);
        return st;
    }
    *out = s;
    return PD_OK;
}

static NodeArgs sim_args(pd_sim s);

// The solid's weighted volume m per node, fixed while the bond flags are (the
// solid takes no damage): the gather kernel's state pass at the current u
// leaves {m, theta} in s->lps, whose m the streamed state pass reads.  Run
// whenever the flags are set (creation, pd_sim_set).
static int lps_mass(pd_sim s) {
    NodeArgs a = sim_args(s);
    a.u = s->u[s->cur];
    return launch_lps_state(s->ctx, a, s->lanes, s->mat.precision == PD_MIXED);
}

static NodeArgs sim_args(pd_sim s) {
    NodeArgs a = base_args(s->nbr, &s->mat);
    a.xv = s->xv;
    a.v = s->v;
    a.alive = s->alive;
    a.bw = s->tiled ? s->bw : nullptr;
    a.cv_uniform = s->cv_uniform;
    a.damage = s->mat.s_c > 0.0;
    a.bc = s->bc;
    a.bc_vel = s->bc_vel;
    a.b = s->b;
    a.flag = s->ctx->flag;
    a.lps = s->lps;
    a.vol_uniform = s->mat.law == PD_LAW_LPS && !(s->mat.pv_h > 0.0) ? s->vol_uniform : 0.0;
    return a;
}

// static part of a simulation's streamed-batch descriptor
StreamInst pd_stream_inst(const pd_sim s) {
    const pd_nbr nbr = s->nbr;
    StreamInst d{};
    d.row_ptr = nbr->row_ptr;
    d.halo_ptr = nbr->halo_ptr;
    d.halo = nbr->halo;
    d.self_off = nbr->self_off;
    d.bw = s->bw;
    d.rec[0] = s->rec[0];
    d.rec[1] = s->rec[1];
    d.v = s->v;
    d.bc = s->bc;
    d.bc_vel = s->bc_vel;
    d.b = s->b;
    d.n = nbr->n;
    d.tile_begin = 0;
    d.cv = s->cv_uniform;
    d.s_c = s->mat.s_c;
    d.rho = s->mat.rho;
    d.damage = s->mat.s_c > 0.0;
    d.beta = s->mat.beta;
    d.lps = s->lpsc;
    d.lpsm = s->lps;
    d.vol = s->vol_uniform;
    d.bulk = s->mat.bulk;
    d.shear = s->mat.shear;
    d.ramp = s->ramp;
    return d;
}

// launch arguments shared by every instance of a batch shaped like sim
StreamArgs pd_stream_args(const pd_sim sim, const StreamInst *inst, uint32_t ninst,
                          uint32_t ntiles) {
    const pd_nbr nbr = sim->nbr;
    StreamArgs sa{};
    sa.inst = inst;
    sa.ninst = ninst;
    sa.ntiles = ntiles;
    sa.tile = nbr->tile_T;
    sa.hcap = pd_tile_hcap(nbr);
    sa.bcap = pd_tile_bcap(nbr);
    sa.mmax = sim->s_mmax;
    return sa;
}

// nsteps launches of the streamed kernel (the solid: state pass, then force
// pass, per step), the k-th told it is step k
static int stream_steps(pd_sim sim, StreamArgs &sa, int64_t nsteps) {
    const pd_ctx ctx = sim->ctx;
    const int prec = sim->mat.precision;
    const int dim = sim->nbr->dim;
    StreamArgs sb = sa;          // the state pass: its own grid and tiles per workgroup
    sb.mmax = sim->s2_mmax;
    for (int64_t k = 0; k < nsteps; ++k) {
        sa.step = k;
        sb.step = k;
        if (sim->s_form == SK_LPS_FORCE)
            PD_TRY(pd_launch_stream(ctx, ctx->stream, dim, sb, sim->lanes, prec, SK_LPS_STATE,
                                    sim->s2_block, sim->s2_grid, sim->s2_lds));
        PD_TRY(pd_launch_stream(ctx, ctx->stream, dim, sa, sim->lanes, prec, sim->s_form,
                                sim->s_block, sim->s_grid, sim->s_lds));
    }
    return PD_OK;
}

// host state after nsteps streamed steps at dt
void pd_sim_advanced(pd_sim sim, int64_t nsteps, double dt) {
    if (nsteps <= 0) return;
    sim->step += nsteps;
    sim->cur ^= (int)(nsteps & 1);
    sim->v_half = true;
    sim->u_stale = true;
    sim->last_dt = dt;
}

extern "C" int pd_verlet_step(pd_sim sim, int64_t nsteps, double dt) {
    if (!sim) return PD_EINVAL;
    pd_ctx ctx = sim->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (nsteps < 0) return pd_set_error(ctx, PD_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return pd_set_error(ctx, PD_EINVAL, "dt must be > 0");
    if (sim->v_half && dt != sim->last_dt)
        return pd_set_error(ctx, PD_EINVAL,
                            "dt changed mid-trajectory: read the state (pd_sim_get) first");
    NodeArgs a = sim_args(sim);
    a.dt = dt;
    const bool mixed = sim->mat.precision == PD_MIXED;
    if (sim->stream) {
        const pd_nbr nbr = sim->nbr;
        if (nsteps > 0 && sim->rec_stale) {
            PD_TRY(pd_rec_pack(ctx, nbr->dim, nbr->n, sim->xv, sim->u[sim->cur],
                               sim->rec[sim->cur]));
            sim->rec_stale = false;
        }
        StreamArgs sa = pd_stream_args(sim, nullptr, 1, nbr->ntiles);
        sa.one = pd_stream_inst(sim);
        sa.one.cur0 = sim->cur;
        sa.one.vhalf0 = sim->v_half ? 1 : 0;
        sa.one.dt = dt;
        sa.one.step0 = sim->step;
        sa.one.limit = nsteps;
        PD_TRY(stream_steps(sim, sa, nsteps));
        pd_sim_advanced(sim, nsteps, dt);
        return PD_OK;
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        a.mode = sim->v_half ? M_STEP_CONT : M_STEP_FIRST;
        a.u = sim->u[sim->cur];
        a.u_out = sim->u[sim->cur ^ 1];
        a.r_half = ramp_factor((double)sim->step + 0.5, sim->ramp);
        PD_TRY(launch_node(ctx, sim->nbr, a, sim->lanes, mixed, sim->block));
        sim->cur ^= 1;
        sim->v_half = true;
        sim->step += 1;
    }
    sim->last_dt = dt;
    return PD_OK;
}

// u[cur] from the records after streamed steps
static int sim_sync_u(pd_sim sim) {
    if (!sim->u_stale) return PD_OK;
    PD_TRY(pd_rec_unpack(sim->ctx, sim->nbr->dim, sim->nbr->n, sim->rec[sim->cur],
                         sim->u[sim->cur]));
    sim->u_stale = false;
    return PD_OK;
}

// completes the last step: force at u^N with the damage test, second half-kick
// A force evaluation of a simulation outside its steps: on the tile kernel,
// or, for tiles without a resident tile kernel (sim->block == 0), on the
// gather kernel, which reads and writes the bond flags: the bond words' dead
// bits go to the flags first and come back after
static int sim_launch(pd_sim sim, const NodeArgs &a, bool mixed) {
    const pd_ctx ctx = sim->ctx;
    if (sim->tiled && sim->block == 0) {
        PD_TRY(pd_bw_to_alive(ctx, sim->nbr, sim->bw, sim->alive));
        PD_TRY(launch_node(ctx, sim->nbr, a, sim->lanes, mixed, 0));
        return pd_bw_compose(ctx, sim->nbr, sim->alive, sim->bw);
    }
    return launch_node(ctx, sim->nbr, a, sim->lanes, mixed, sim->block);
}

static int sim_close(pd_sim sim) {
    PD_TRY(sim_sync_u(sim));
    if (!sim->v_half) return PD_OK;
    NodeArgs a = sim_args(sim);
    a.dt = sim->last_dt;
    a.mode = M_CLOSE;
    a.u = sim->u[sim->cur];
    a.r_full = ramp_factor((double)sim->step, sim->ramp);
    PD_TRY(sim_launch(sim, a, sim->mat.precision == PD_MIXED));
    sim->v_half = false;
    return PD_OK;
}

// Central-difference steps: the first step of the call is a velocity-Verlet
// step (the scheme's start), the others u^{k+1} = 2 u^k - u^{k-1} + dt^2 a^k
// with u^{k-1} in the other half of the ping-pong pair (of records on the
// streamed kernel, of u arrays on the tile and gather kernels).
extern "C" int pd_central_step(pd_sim sim, int64_t nsteps, double dt) {
    if (!sim) return PD_EINVAL;
    pd_ctx ctx = sim->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (nsteps < 0) return pd_set_error(ctx, PD_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return pd_set_error(ctx, PD_EINVAL, "dt must be > 0");
    if (sim->v_half && dt != sim->last_dt)
        return pd_set_error(ctx, PD_EINVAL,
                            "dt changed mid-trajectory: read the state (pd_sim_get) first");
    if (nsteps == 0) return PD_OK;
    const bool mixed = sim->mat.precision == PD_MIXED;
    if (sim->stream) {
        // on the streamed kernel: the first launch a Verlet step, the others
        // central differences from the record pair
        const pd_nbr nbr = sim->nbr;
        if (sim->rec_stale) {
            PD_TRY(pd_rec_pack(ctx, nbr->dim, nbr->n, sim->xv, sim->u[sim->cur],
                               sim->rec[sim->cur]));
            sim->rec_stale = false;
        }
        StreamArgs sa = pd_stream_args(sim, nullptr, 1, nbr->ntiles);
        sa.one = pd_stream_inst(sim);
        sa.one.cur0 = sim->cur;
        sa.one.vhalf0 = sim->v_half ? 1 : 0;
        sa.one.dt = dt;
        sa.one.step0 = sim->step;
        sa.one.limit = nsteps;
        sa.one.cd = 1;
        PD_TRY(stream_steps(sim, sa, nsteps));
        pd_sim_advanced(sim, nsteps, dt);
        return PD_OK;
    }
    PD_TRY(sim_sync_u(sim));
    NodeArgs a = sim_args(sim);
    a.dt = dt;
    for (int64_t k = 0; k < nsteps; ++k) {
        a.mode = k > 0 ? M_STEP_CD : (sim->v_half ? M_STEP_CONT : M_STEP_FIRST);
        a.u = sim->u[sim->cur];
        a.u_out = sim->u[sim->cur ^ 1];
        a.r_half = ramp_factor((double)sim->step + 0.5, sim->ramp);
        PD_TRY(launch_node(ctx, sim->nbr, a, sim->lanes, mixed, sim->block));
        sim->cur ^= 1;
        sim->v_half = true;
        sim->step += 1;
    }
    sim->last_dt = dt;
    return PD_OK;
}

extern "C" int pd_sim_get(pd_sim sim, double *u, double *v, uint8_t *alive, double *ke_pe,
                          int64_t *step) {
    if (!sim) return PD_EINVAL;
    pd_ctx ctx = sim->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (u) PD_TRY(pd_check_dev_ptr(ctx, u, "u"));
    if (v) PD_TRY(pd_check_dev_ptr(ctx, v, "v"));
    if (alive) PD_TRY(pd_check_dev_ptr(ctx, alive, "alive"));
    PD_TRY(pd_flag_clear(ctx));
    PD_TRY(sim_close(sim));
    if (u) PD_TRY(pd_scatter_vec(ctx, sim->nbr, sim->u[sim->cur], u));
    if (v) PD_TRY(pd_scatter_vec(ctx, sim->nbr, sim->v, v));
    if (alive) {
        if (sim->tiled) PD_TRY(pd_bw_to_alive(ctx, sim->nbr, sim->bw, sim->alive));
        PD_TRY(pd_alive_out(ctx, sim->nbr, sim->alive, alive));
    }
    if (ke_pe) {
        NodeArgs a = sim_args(sim);
        a.mode = M_ENERGY;
        a.damage = 0;
        a.u = sim->u[sim->cur];
        a.e_out = sim->scratch;
        PD_TRY(sim_launch(sim, a, false));
        PD_TRY(pd_sum(ctx, sim->scratch, sim->nbr->n, 2, ke_pe));
    }
    if (step) *step = sim->step;
    int flag = 0;
    PD_TRY(pd_flag_read(ctx, &flag));
    if (flag & 1) return pd_set_error(ctx, PD_ENONFINITE, "non-finite displacement or velocity");
    return PD_OK;
}

extern "C" int pd_sim_set(pd_sim sim, const double *u, const double *v, const uint8_t *alive,
                          int64_t step) {
    if (!sim) return PD_EINVAL;
    pd_ctx ctx = sim->ctx;
    PD_TRY(pd_check_ctx(ctx));
    if (u) PD_TRY(pd_check_dev_ptr(ctx, u, "u"));
    if (v) PD_TRY(pd_check_dev_ptr(ctx, v, "v"));
    if (alive) PD_TRY(pd_check_dev_ptr(ctx, alive, "alive"));
    if (step < 0) return pd_set_error(ctx, PD_EINVAL, "step must be >= 0");
    PD_TRY(sim_close(sim));
    if (u) {
        PD_TRY(pd_gather_vec(ctx, sim->nbr, u, sim->u[sim->cur], false));
        sim->rec_stale = true;
    }
    if (v) PD_TRY(pd_gather_vec(ctx, sim->nbr, v, sim->v, false));
    if (alive) {
        PD_TRY(pd_alive_in(ctx, sim->nbr, alive, sim->alive));
        if (sim->tiled) PD_TRY(pd_bw_compose(ctx, sim->nbr, sim->alive, sim->bw));
        if (sim->stream && sim->s_form == SK_LPS_FORCE) PD_TRY(lps_mass(sim));
    }
    sim->step = step;
    return PD_OK;
}

int pd_sim_rehome(pd_sim s, pd_ctx to) {
    const pd_ctx from = s->ctx;
    const pd_nbr nb = s->nbr;
    if (from == to) return PD_OK;
    if (from->device != to->device || nb->ctx != from || nb->refs != 1 || nb->users > 1)
        return pd_set_error(to, PD_EINVAL, "the simulation cannot move to this context");
    PD_HIP(from, hipStreamSynchronize(from->stream));
    pd_mem_restream(from->stream, to->stream, from->red, from->flag);
    s->ctx = to;
    nb->ctx = to;
    from->refs -= 2;
    to->refs += 2;
    return PD_OK;
}

extern "C" int pd_sim_info(pd_sim sim, int *kernel, int *tile, int *block, int *lanes) {
    if (!sim) return PD_EINVAL;
    if (kernel) *kernel = sim->stream ? 3 : (sim->tiled && sim->block > 0 ? 2 : 1);
    if (tile) *tile = sim->stream || (sim->tiled && sim->block > 0) ? (int)sim->nbr->tile_T : 0;
    if (block) *block = sim->stream ? sim->s_block : (sim->block > 0 ? sim->block : PD_BLOCK);
    if (lanes) *lanes = sim->lanes;
    return PD_OK;
}

extern "C" int pd_sim_destroy(pd_sim sim) {
    if (!sim) return PD_EINVAL;
    (void)hipSetDevice(sim->ctx->device);
    (void)hipStreamSynchronize(sim->ctx->stream);
    sim_release(sim);
    return PD_OK;
}
