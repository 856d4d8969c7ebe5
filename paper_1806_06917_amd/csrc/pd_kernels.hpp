// Device code shared by the node kernels: the bond laws (Algorithm 1,
// linearised or general: the NP potential, the exact stretch, partial
// volumes and the influence function; the linear peridynamic solid's bond
// terms of Algorithm 2), the damage test, the per-node lane reduction and
// the node update (force output, tangent output, energies, velocity-Verlet
// half-kicks and drift with boundary data, central differences).
#pragma once

#include <type_traits>

#include "pd_internal.hpp"

namespace pdk {

enum Mode {
    M_FORCE = 0, M_STEP_FIRST = 1, M_STEP_CONT = 2, M_CLOSE = 3, M_ENERGY = 4, M_TANGENT = 5,
    M_STEP_CD = 6   // central-difference step: u_out holds u^{k-1} on entry
};

struct NodeArgs {
    const double *__restrict__ xv;     // [n][4]
    const double *__restrict__ u;      // [n][US]
    double *__restrict__ u_out;        // [n][US]
    double *__restrict__ v;            // [n][US]
    const uint32_t *__restrict__ row_ptr;
    const int32_t *__restrict__ col;   // sfc ids (gather kernel)
    uint16_t *__restrict__ bw;         // tile kernel bond words: local id | 0x8000 once broken
    const uint32_t *__restrict__ halo_ptr;
    const int32_t *__restrict__ halo;
    const uint32_t *__restrict__ self_off;
    uint8_t *__restrict__ alive;       // NULL: all intact, no damage
    const uint8_t *__restrict__ bc;    // NULL: all free (tangent mode: fixed flags)
    const double *__restrict__ bc_vel; // [n][US]
    const double *__restrict__ b;      // [n][US] or NULL
    double *__restrict__ f_out;        // [n][US] force (M_FORCE) or y (M_TANGENT)
    double *__restrict__ e_out;        // M_FORCE: U_i; M_ENERGY: {KE_i, V_i U_i} pairs
    int *__restrict__ flag;            // non-finite report
    int fp32;                          // PD_FP32: float32 bond terms, compensated sums
    const int *__restrict__ done;      // if set and *done != 0 the launch is a no-op
    const double *__restrict__ rec;    // streamed kernel: records {X, u} per node
    double *__restrict__ rec_out;      // streamed kernel: u^{k+1} goes into these records
    uint32_t n;
    uint32_t tile;                     // nodes per tile (tile kernel)
    uint32_t hcap;                     // halo records held in LDS (tile kernel)
    uint32_t bcap;                     // bonds per tile held in LDS (tile kernel)
    uint32_t ntiles;                   // tiles (tile kernel)
    uint32_t mmax;                     // tiles per workgroup, upper bound (tile kernel)
    int mode;
    int damage;
    double c, s_c, rho, dt, r_half, r_full;
    double cv_uniform;                 // c V when every node has volume V, else 0
    // general pairwise law (gather kernel): PD_LAW_*, PD_STRETCH_*, NP beta,
    // and the linearisation point of the tangent ([n][US], sfc order)
    int law, stretch;
    double beta;
    const double *__restrict__ u_lin;
    // linear peridynamic solid: moduli and {m, theta} per node ([n][2], sfc);
    // vol_uniform: V when every node has volume V and there are no partial
    // volumes (the bond sums then leave V out and each node's sums are scaled
    // by V once, as in the streamed kernel), else 0
    double bulk, shear;
    double *__restrict__ lps;
    double vol_uniform;
    // partial volumes: band width h (0 = off) and the neighbour radius R
    double pv_h, pv_R;
    // influence function J = j_c1 r exp(-r^2/j_c2), r = |xi| j_idelta
    // (j_c2 = 0: off)
    double j_c1, j_c2, j_idelta;
};

// partial-volume weight of a bond of length len: min(1, max(0, (R - len)/h)),
// 1 when h = 0
__device__ __forceinline__ double pv_weight(double len, double R, double h) {
    return h > 0.0 ? fmin(1.0, fmax(0.0, (R - len) / h)) : 1.0;
}

// per-lane FP64 running sums of the bond forces (and bond energies)
struct Acc64 {
    double x = 0, y = 0, z = 0, e = 0;
};

template <int DIM>
__device__ __forceinline__ void load_vec(const double *p, uint32_t i, double &x, double &y,
                                         double &z) {
    if (DIM == 3) {
        const double4 q = reinterpret_cast<const double4 *>(p)[i];
        x = q.x; y = q.y; z = q.z;
    } else {
        const double2 q = reinterpret_cast<const double2 *>(p)[i];
        x = q.x; y = q.y; z = 0.0;
    }
}

template <int DIM>
__device__ __forceinline__ void store_vec(double *p, uint32_t i, double x, double y, double z) {
    if (DIM == 3) reinterpret_cast<double4 *>(p)[i] = make_double4(x, y, z, 0.0);
    else reinterpret_cast<double2 *>(p)[i] = make_double2(x, y);
}

// 1/sqrt(r2) for finite r2 > 0: the hardware estimate refined by one
// third-order correction, y = y0 + y0 e (1/2 + 3/8 e), e = 1 - r2 y0^2
__device__ __forceinline__ double rsqrt_pos(double r2) {
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = fma(y0 * -r2, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// Dot products with a fixed fused order, a.x*b.x first, then each further
// product fused into the sum: every kernel rounds a bond's arithmetic the
// same way whatever the compiler's contraction choices around it (the tile,
// streamed and gather kernels must agree bit for bit).
template <int DIM>
__device__ __forceinline__ double dotf(double ax, double ay, double az, double bx, double by,
                                       double bz) {
    return DIM == 3 ? fma(az, bz, fma(ay, by, ax * bx)) : fma(ay, by, ax * bx);
}

// One bond: xi = X_j - X_i, eta = u_j - u_i, cVj = c V_j; `dead` marks a bond
// broken earlier; damage on/off and the critical stretch s_c.  Returns true if
// the bond breaks now (S > s_c); a bond that is dead or breaks now contributes
// nothing.  Otherwise adds
// c V_j S xi/|xi| (and (c/4) V_j S^2 |xi| if WANT_E) to the lane's sums.
// Everything runs in float64; mixed precision takes 1/|xi| from the hardware
// reciprocal-square-root estimate alone (relative error below 2^-22), the
// FP64 mode refines it to full double precision.
// With NP the force carries the factor exp(-beta r), r = |xi| S^2, of the
// NP potential (linearised stretch; the streamed kernel's NP form).  Mixed
// precision takes the factor from the hardware float32 exp2 (relative error
// about 1e-7 for the exponents that matter; the factor underflows to 0 below
// exp(-87), where the bond carries no force anyway).
template <int DIM, bool MIXED, bool WANT_E, bool NP = false>
__device__ __forceinline__ bool bond(int damage, double s_c, double dxx, double dxy, double dxz,
                                     double dux, double duy, double duz, double cVj, bool dead,
                                     Acc64 &s, double beta = 0.0) {
    const double r2 = dotf<DIM>(dxx, dxy, dxz, dxx, dxy, dxz);
    const double ex = dotf<DIM>(dux, duy, duz, dxx, dxy, dxz);
    const double inv = MIXED ? __builtin_amdgcn_rsq(r2) : rsqrt_pos(r2);
    const double S = ex * (inv * inv);
    const bool brk = damage && !dead && S > s_c;
    // a dead or breaking bond leaves the sums untouched (they are never -0);
    // the empty volatile statement keeps this a masked block rather than
    // selects after the sums
    if (!(brk || dead)) {
        asm volatile("" ::: "memory");
        double g = cVj * S * inv;
        if (NP) {
            const double x = -beta * ((r2 * inv) * S * S);
            g *= MIXED ? (double)__builtin_amdgcn_exp2f((float)(x * 1.4426950408889634)) : exp(x);
        }
        s.x = fma(g, dxx, s.x);
        s.y = fma(g, dxy, s.y);
        if (DIM == 3) s.z = fma(g, dxz, s.z);
        if (WANT_E && !NP) s.e += 0.25 * cVj * S * S * (r2 * inv);
        if (WANT_E && NP) s.e += 0.25 * cVj * (-expm1(-beta * ((r2 * inv) * S * S)) / beta);
    }
    return brk;
}

// ---------------------------------------------------------------------------
// PD_FP32: the bond terms of the linearised law in float32 after the float64
// differences, with compensated float32 per-node sums
// ---------------------------------------------------------------------------
// running sums as unevaluated pairs hi + lo (TwoSum keeps every addition's
// rounding error in lo)
struct AccC {
    float hx = 0, lx = 0, hy = 0, ly = 0, hz = 0, lz = 0, he = 0, le = 0;
};

// h + v as the pair (s, e) with s = fl(h + v) and s + e = h + v exactly
// (Knuth's TwoSum); the error goes into l
__device__ __forceinline__ void two_sum_into(float &h, float &l, float v) {
#pragma clang fp contract(off)
    const float s = h + v;
    const float bp = s - h;
    const float e = (h - (s - bp)) + (v - bp);
    h = s;
    l = l + e;
}

// One bond as in `bond`, in float32: xi and eta arrive as float64
// differences and are rounded to float32; |xi|^2 and eta.xi are fused
// float32 sums, |xi|^-1 is the hardware float32 reciprocal square root; S,
// the damage test (against s_c rounded to float32) and the bond force are
// float32.  The force terms (and the energy) come back in t, exactly +0 for
// a dead or breaking bond; the return value says whether the bond breaks.
template <int DIM, bool WANT_E>
__device__ __forceinline__ bool bond32(int damage, float s_c, double dxx, double dxy, double dxz,
                                       double dux, double duy, double duz, float cVj, bool dead,
                                       float &tx, float &ty, float &tz, float &te) {
    const float x = (float)dxx, y = (float)dxy, z = DIM == 3 ? (float)dxz : 0.0f;
    const float ex = (float)dux, ey = (float)duy, ez = DIM == 3 ? (float)duz : 0.0f;
    const float r2 = DIM == 3 ? __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x))
                              : __builtin_fmaf(y, y, x * x);
    const float et = DIM == 3 ? __builtin_fmaf(ez, z, __builtin_fmaf(ey, y, ex * x))
                              : __builtin_fmaf(ey, y, ex * x);
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float S = et * (inv * inv);
    const bool brk = damage && !dead && S > s_c;
    const bool live = !(brk || dead);
    const float g = cVj * S * inv;
    tx = live ? g * x : 0.0f;
    ty = live ? g * y : 0.0f;
    tz = DIM == 3 && live ? g * z : 0.0f;
    te = WANT_E && live ? 0.25f * cVj * S * S * (r2 * inv) : 0.0f;
    return brk;
}

// The terms of two consecutive bonds of a lane (a before b; a lane's last
// bond, if its count is odd, pairs with terms +0) are added in float32 and
// the pair sum goes into the compensated sums: one TwoSum per pair and
// component.  The pair sum adds one rounding of the size of the terms' own,
// so the sums stay free of error growth with the bond count.
template <int DIM, bool WANT_E>
__device__ __forceinline__ void pair_into(AccC &s, float ax, float ay, float az, float ae, float bx,
                                          float by, float bz, float be) {
#pragma clang fp contract(off)
    two_sum_into(s.hx, s.lx, ax + bx);
    two_sum_into(s.hy, s.ly, ay + by);
    if (DIM == 3) two_sum_into(s.hz, s.lz, az + bz);
    if (WANT_E) two_sum_into(s.he, s.le, ae + be);
}

// A float moved across lanes by a DPP pattern
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL,
                                                              0xF, 0xF, false));
}

// one reduction level of a compensated pair over blocks of 2M lanes whose
// halves are uniform (the partners of level_sum); both partners compute the
// same pair (TwoSum's error is exact, so operand order does not matter)
template <int M>
__device__ __forceinline__ void level_sum_c(float &h, float &l) {
    float hp, lp;
    if constexpr (M == 1) { hp = dpp_f32<0xB1>(h); lp = dpp_f32<0xB1>(l); }
    else if constexpr (M == 2) { hp = dpp_f32<0x4E>(h); lp = dpp_f32<0x4E>(l); }
    else if constexpr (M == 4) { hp = dpp_f32<0x141>(h); lp = dpp_f32<0x141>(l); }
    else if constexpr (M == 8) { hp = dpp_f32<0x140>(h); lp = dpp_f32<0x140>(l); }
    else { hp = __shfl_xor(h, M, 2 * M); lp = __shfl_xor(l, M, 2 * M); }
    {
#pragma clang fp contract(off)
        const float sum = h + hp;
        const float bp = sum - h;
        const float e = (h - (sum - bp)) + (hp - bp);
        h = sum;
        l = (l + lp) + e;
    }
}

// group reduction of the compensated sums (the order of group_reduce), then
// each pair hi + lo in float64
template <int DIM, int L, bool WANT_E>
__device__ __forceinline__ void group_reduce_c(AccC &s, double &fx, double &fy, double &fz,
                                               double &Ue) {
    auto level = [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if constexpr (M < L) {
            level_sum_c<M>(s.hx, s.lx);
            level_sum_c<M>(s.hy, s.ly);
            if (DIM == 3) level_sum_c<M>(s.hz, s.lz);
            if (WANT_E) level_sum_c<M>(s.he, s.le);
        }
    };
    level(std::integral_constant<int, 1>{});
    level(std::integral_constant<int, 2>{});
    level(std::integral_constant<int, 4>{});
    level(std::integral_constant<int, 8>{});
    level(std::integral_constant<int, 16>{});
    level(std::integral_constant<int, 32>{});
    fx = (double)s.hx + (double)s.lx;
    fy = (double)s.hy + (double)s.ly;
    fz = DIM == 3 ? (double)s.hz + (double)s.lz : 0.0;
    Ue = WANT_E ? (double)s.he + (double)s.le : 0.0;
}

// One bond under the general pairwise law of Algorithm 1 (gather kernel):
// the NP potential psi(r) = C (1 - exp(-beta r)) and/or the exact stretch.
// Force and damage as in `bond` with S the chosen stretch, e its direction
// (xi/|xi|, or (xi+eta)/|xi+eta| for the exact stretch) and the bond force
// c V_j exp(-beta r) S e (factor 1 for the linear law), r = |xi| S^2; energy
// c V_j/(4 beta) (1 - exp(-beta r)) (linear law: (c/4) V_j r).
// Tangent mode (du = w_j - w_i, linearised stretch): the bond acts with the
// stiffness c exp(-beta r)(1 - 2 beta r) of the linearisation point
// (dl = ulin_j - ulin_i), i.e. psi'(r) + 2 r psi''(r) over psi'(0).
template <int DIM, bool MIXED, bool WANT_E>
__device__ __forceinline__ bool bond_law(int law, int stretch, double beta, int damage,
                                         double s_c, bool tangent, double dxx, double dxy,
                                         double dxz, double dux, double duy, double duz,
                                         double dlx, double dly, double dlz, double cVj,
                                         bool dead, Acc64 &s, double pvh = 0.0,
                                         double pvR = 0.0, double jc1 = 0.0, double jc2 = 0.0,
                                         double jid = 0.0) {
    const double r2 = dotf<DIM>(dxx, dxy, dxz, dxx, dxy, dxz);
    const double inv = MIXED ? __builtin_amdgcn_rsq(r2) : rsqrt_pos(r2);
    const double len = r2 * inv;
    if (pvh > 0.0) cVj *= pv_weight(len, pvR, pvh);
    if (jc2 > 0.0) {
        const double r = len * jid;
        cVj *= jc1 * r * exp(-(r * r) / jc2);
    }
    const bool np = law == PD_LAW_NP;
    if (tangent) {
        const double el = dotf<DIM>(dlx, dly, dlz, dxx, dxy, dxz);
        const double Su = el * (inv * inv);
        const double r = len * Su * Su;
        const double k = np ? exp(-beta * r) * (1.0 - 2.0 * beta * r) : 1.0;
        const double ew = dotf<DIM>(dux, duy, duz, dxx, dxy, dxz);
        const double g = dead ? 0.0 : cVj * k * (ew * (inv * inv)) * inv;
        s.x = fma(g, dxx, s.x);
        s.y = fma(g, dxy, s.y);
        if (DIM == 3) s.z = fma(g, dxz, s.z);
        return false;
    }
    double S, ex, ey, ez;
    if (stretch == PD_STRETCH_EXACT) {
        // S = (|xi+eta| - |xi|)/|xi| in the cancellation-free form
        // (2 xi.eta + eta.eta)/((|xi+eta| + |xi|) |xi|)
        const double yx = dxx + dux, yy = dxy + duy, yz = DIM == 3 ? dxz + duz : 0.0;
        const double y2 = dotf<DIM>(yx, yy, yz, yx, yy, yz);
        const double iy = MIXED ? __builtin_amdgcn_rsq(y2) : rsqrt_pos(y2);
        const double xe = dotf<DIM>(dxx, dxy, dxz, dux, duy, duz);
        const double ee = dotf<DIM>(dux, duy, duz, dux, duy, duz);
        S = (2.0 * xe + ee) / (y2 * iy + len) * inv;
        ex = yx * iy; ey = yy * iy; ez = yz * iy;
    } else {
        const double e_ = dotf<DIM>(dux, duy, duz, dxx, dxy, dxz);
        S = e_ * (inv * inv);
        ex = dxx * inv; ey = dxy * inv; ez = dxz * inv;
    }
    const bool brk = damage && S > s_c;
    const bool off = brk || dead;
    const double r = len * S * S;
    const double phi = np ? exp(-beta * r) : 1.0;
    const double g = off ? 0.0 : cVj * phi * S;
    s.x = fma(g, ex, s.x);
    s.y = fma(g, ey, s.y);
    if (DIM == 3) s.z = fma(g, ez, s.z);
    if (WANT_E) s.e += off ? 0.0 : 0.25 * cVj * (np ? -expm1(-beta * r) / beta : r);
    return brk && !dead;
}

// Linear peridynamic solid, per bond, written so that it needs one
// reciprocal square root and one reciprocal (y = xi + eta):
//   r2 = |xi|^2,
//   q  = 1 / (|xi| |y|) = rsqrt(r2 |y|^2),
//   w  = |xi| e with the extension e = |y| - |xi| in the cancellation-free
//        form (|y|^2 - |xi|^2)/(|y| + |xi|): w = num / (1 + |y|^2 q), where
//        num = |y|^2 - |xi|^2 = eta.(xi + y) and |y|^2 q = |y|/|xi|.
// The state pass sums |xi|^2 = r2 and |xi| e = w; the force pass's weight
// t / |y| = (A |xi| + D e) / |y| is q (A r2 + D w) (|xi|/|y| = r2 q,
// e/|y| = w q).  Mixed precision takes both from the hardware estimates
// (relative error below 2^-22); the denominator is formed without
// contraction (every kernel rounds it alike).
template <bool MIXED>
__device__ __forceinline__ double lps_w(double num, double y2, double q) {
#pragma clang fp contract(off)
    const double den = y2 * q + 1.0;
    return MIXED ? num * __builtin_amdgcn_rcp(den) : num / den;
}

template <bool MIXED>
__device__ __forceinline__ void lps_terms(double dxx, double dxy, double dxz, double dux,
                                          double duy, double duz, double &r2, double &q,
                                          double &w) {
    r2 = dotf<3>(dxx, dxy, dxz, dxx, dxy, dxz);
    const double yx = dxx + dux, yy = dxy + duy, yz = dxz + duz;
    const double y2 = dotf<3>(yx, yy, yz, yx, yy, yz);
    const double r2y2 = r2 * y2;
    q = MIXED ? __builtin_amdgcn_rsq(r2y2) : rsqrt_pos(r2y2);
    const double num = dotf<3>(dux, duy, duz, dxx + yx, dxy + yy, dxz + yz);
    w = lps_w<MIXED>(num, y2, q);
}

// |xi| from r2 (partial volumes, the energy)
template <bool MIXED>
__device__ __forceinline__ double lps_len(double r2) {
    return r2 * (MIXED ? __builtin_amdgcn_rsq(r2) : rsqrt_pos(r2));
}

// The solid's per-bond terms, shared by the gather and streamed kernels and
// written without contraction, so that both round every bond alike.
// First pass: m += |xi|^2 V_j, s += |xi| e V_j.
__device__ __forceinline__ void lps_state_terms(double r2, double w, double Vj, double &m,
                                                double &s) {
#pragma clang fp contract(off)
    m += r2 * Vj;
    s += w * Vj;
}
// A node's coefficients in the bond force state, from its {m, theta}:
// t_ij = (3 K theta_i / m_i) |xi| + (15 mu / m_i) (e - theta_i |xi| / 3)
//      = a_i |xi| + d_i e  with  a_i = (3 K - 5 mu) theta_i / m_i,
// d_i = 15 mu / m_i (both 0 where m_i = 0); mixed precision rounds both to
// float32 (the streamed force pass stages them so).
struct LpsCoef {
    double a, d;
};
template <bool MIXED>
__device__ __forceinline__ LpsCoef lps_coef(double m, double theta, double K, double mu) {
#pragma clang fp contract(off)
    LpsCoef q;
    q.a = m > 0.0 ? (3.0 * K - 5.0 * mu) * theta / m : 0.0;
    q.d = m > 0.0 ? 15.0 * mu / m : 0.0;
    if (MIXED) {
        q.a = (double)(float)q.a;
        q.d = (double)(float)q.d;
    }
    return q;
}
// Force: the weight g of M = (xi+eta) in f_i, (t_ij + t_ji) V_j / |xi+eta|
// = q ((a_i + a_j) r2 + (d_i + d_j) w) V_j, from the coefficients of both
// ends and the bond's r2, q, w (lps_terms).
__device__ __forceinline__ double lps_force_weight(const LpsCoef &qi, const LpsCoef &qj,
                                                   double r2, double q, double w, double Vj,
                                                   bool live) {
#pragma clang fp contract(off)
    const double t = (qi.a + qj.a) * r2 + (qi.d + qj.d) * w;
    return live ? t * q * Vj : 0.0;
}

// A double moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One reduction level over blocks of 2M lanes whose halves are each uniform:
// every lane adds the value of a lane in the other half.  M = 1, 2 take the
// xor partner (quad permutations), M = 4, 8 the mirror lane in the 8- or
// 16-lane row (uniform halves make that the same sum), M = 16 the xor
// partner through the LDS crossbar.  Both partners add the same two values,
// so the block ends uniform, bit for bit.
template <int M>
__device__ __forceinline__ double level_sum(double x) {
    if constexpr (M == 1) return x + dpp_f64<0xB1>(x);        // quad_perm [1,0,3,2]
    else if constexpr (M == 2) return x + dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
    else if constexpr (M == 4) return x + dpp_f64<0x141>(x);  // row_half_mirror
    else if constexpr (M == 8) return x + dpp_f64<0x140>(x);  // row_mirror
    else return x + __shfl_xor(x, M, 2 * M);
}

// Sum of one double over the L lanes of a group (aligned, L a power of two up
// to 64) in the order of group_reduce
template <int L>
__device__ __forceinline__ double lane_sum(double x) {
    if constexpr (L > 1) x = level_sum<1>(x);
    if constexpr (L > 2) x = level_sum<2>(x);
    if constexpr (L > 4) x = level_sum<4>(x);
    if constexpr (L > 8) x = level_sum<8>(x);
    if constexpr (L > 16) x = level_sum<16>(x);
    if constexpr (L > 32) x = level_sum<32>(x);
    return x;
}

// Sum over the L lanes of a group (aligned, L a power of two up to 64),
// pairing neighbours first: every lane ends with the same sum.
template <int DIM, int L, bool WANT_E>
__device__ __forceinline__ void group_reduce(Acc64 &s, double &fx, double &fy, double &fz,
                                             double &Ue) {
    auto level = [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if constexpr (M < L) {
            s.x = level_sum<M>(s.x);
            s.y = level_sum<M>(s.y);
            if (DIM == 3) s.z = level_sum<M>(s.z);
            if (WANT_E) s.e = level_sum<M>(s.e);
        }
    };
    level(std::integral_constant<int, 1>{});
    level(std::integral_constant<int, 2>{});
    level(std::integral_constant<int, 4>{});
    level(std::integral_constant<int, 8>{});
    level(std::integral_constant<int, 16>{});
    level(std::integral_constant<int, 32>{});
    fx = s.x; fy = s.y; fz = s.z; Ue = s.e;
}

// modes whose node update reads v
__host__ __device__ inline bool mode_reads_v(int mode) {
    return mode == M_STEP_FIRST || mode == M_STEP_CONT || mode == M_CLOSE || mode == M_ENERGY;
}

// Node update by one lane, after the force density f_i is known.  (vx, vy,
// vz) is v_i and `kind` the boundary kind of node i, both read by the caller
// (v only in the modes of mode_reads_v).
template <int DIM>
__device__ __forceinline__ void node_update(const NodeArgs &a, uint32_t i, double fx, double fy,
                                            double fz, double Ue, double Vi, double uix,
                                            double uiy, double uiz, bool fixed_i, double vx,
                                            double vy, double vz, int kind) {
    switch (a.mode) {
    case M_FORCE:
        store_vec<DIM>(a.f_out, i, fx, fy, fz);
        if (a.e_out) a.e_out[i] = Ue;
        return;
    case M_TANGENT: {
        if (fixed_i) {
            double wx, wy, wz;
            load_vec<DIM>(a.u, i, wx, wy, wz);
            store_vec<DIM>(a.f_out, i, wx, wy, wz);
        } else {
            store_vec<DIM>(a.f_out, i, -Vi * fx, -Vi * fy, -Vi * fz);
        }
        return;
    }
    case M_ENERGY: {
        const double vv = DIM == 3 ? vx * vx + vy * vy + vz * vz : vx * vx + vy * vy;
        a.e_out[2 * (size_t)i] = 0.5 * a.rho * Vi * vv;
        a.e_out[2 * (size_t)i + 1] = Vi * Ue;
        return;
    }
    default: break;
    }

    const double hdt = 0.5 * a.dt;
    if (a.mode == M_CLOSE) {   // second half-kick of the last step
        if (kind == PD_BC_FREE) {
            double bx = 0, by = 0, bz = 0;
            if (a.b) load_vec<DIM>(a.b, i, bx, by, bz);
            vx = vx + hdt * (fx + bx) / a.rho;
            vy = vy + hdt * (fy + by) / a.rho;
            vz = vz + hdt * (fz + bz) / a.rho;
        } else if (kind == PD_BC_CLAMPED) {
            vx = vy = vz = 0.0;
        } else {
            double wx, wy, wz;
            load_vec<DIM>(a.bc_vel, i, wx, wy, wz);
            vx = a.r_full * wx; vy = a.r_full * wy; vz = a.r_full * wz;
        }
        store_vec<DIM>(a.v, i, vx, vy, vz);
        const bool fin = isfinite(vx) && isfinite(vy) && isfinite(vz) && isfinite(uix) &&
                         isfinite(uiy) && isfinite(uiz);
        if (!fin) atomicOr(a.flag, 1);
        return;
    }
    double nx, ny, nz;
    if (kind == PD_BC_FREE && a.mode == M_STEP_CD) {
        // u^{k+1} = 2 u^k - u^{k-1} + dt^2 (f + b)/rho; v keeps the half-step
        // velocity (u^{k+1} - u^k)/dt, which a closing half-kick completes
        double bx = 0, by = 0, bz = 0, px, py, pz;
        if (a.b) load_vec<DIM>(a.b, i, bx, by, bz);
        load_vec<DIM>(a.u_out, i, px, py, pz);
        nx = (2.0 * uix - px) + a.dt * a.dt * (fx + bx) / a.rho;
        ny = (2.0 * uiy - py) + a.dt * a.dt * (fy + by) / a.rho;
        nz = (2.0 * uiz - pz) + a.dt * a.dt * (fz + bz) / a.rho;
        vx = (nx - uix) / a.dt;
        vy = (ny - uiy) / a.dt;
        vz = (nz - uiz) / a.dt;
    } else if (kind == PD_BC_FREE) {
        double bx = 0, by = 0, bz = 0;
        if (a.b) load_vec<DIM>(a.b, i, bx, by, bz);
        if (a.mode == M_STEP_CONT) {   // second half-kick of the previous step
            vx = vx + hdt * (fx + bx) / a.rho;
            vy = vy + hdt * (fy + by) / a.rho;
            vz = vz + hdt * (fz + bz) / a.rho;
        }
        vx = vx + hdt * (fx + bx) / a.rho;   // first half-kick of this step
        vy = vy + hdt * (fy + by) / a.rho;
        vz = vz + hdt * (fz + bz) / a.rho;
        nx = uix + a.dt * vx;                // drift
        ny = uiy + a.dt * vy;
        nz = uiz + a.dt * vz;
    } else if (kind == PD_BC_CLAMPED) {
        vx = vy = vz = 0.0;
        nx = ny = nz = 0.0;
    } else {
        double wx, wy, wz;
        load_vec<DIM>(a.bc_vel, i, wx, wy, wz);
        vx = a.r_half * wx; vy = a.r_half * wy; vz = a.r_half * wz;
        nx = uix + a.dt * vx;
        ny = uiy + a.dt * vy;
        nz = uiz + a.dt * vz;
    }
    store_vec<DIM>(a.v, i, vx, vy, vz);
    if (a.rec_out) {   // u part of the record {x y z ux uy uz} ({x y ux uy})
        double *r = a.rec_out + (size_t)i * (DIM == 3 ? 6 : 4);
        if (DIM == 3) {
            r[3] = nx;
            *reinterpret_cast<double2 *>(r + 4) = make_double2(ny, nz);
        } else {
            *reinterpret_cast<double2 *>(r + 2) = make_double2(nx, ny);
        }
    } else {
        store_vec<DIM>(a.u_out, i, nx, ny, nz);
    }
}

// modes that need the strain energy of every bond
__host__ __device__ inline bool mode_wants_energy(const NodeArgs &a) {
    return a.mode == M_ENERGY || (a.mode == M_FORCE && a.e_out != nullptr);
}

// one instance of a streamed batch (device memory).  The dynamic fields give
// the instance's state at batch step 0: its step count, which record buffer
// holds u, whether v holds v^{k-1/2}, and how many batch steps it takes.
struct StreamInst {
    const uint32_t *row_ptr;
    const uint32_t *halo_ptr;
    const int32_t *halo;
    const uint32_t *self_off;
    uint16_t *bw;
    double *rec[2];
    double *v;
    const uint8_t *bc;          // padded to whole 32-bit words
    const double *bc_vel;
    const double *b;
    uint32_t n, tile_begin;     // nodes; first tile in the batch numbering
    double cv, s_c, rho, dt;
    double beta;                // NP law (launches of the NP kernel only)
    double *lps;                // the solid: [n] {a, d} (lps_coef) from its state pass
    const double *lpsm;         // the solid: [n][2] {m, .}: m per node, fixed with the bonds
    double vol, bulk, shear;    // the solid: the (uniform) nodal volume and the moduli
    int damage, cur0, vhalf0;
    int cd;                     // central-difference steps after the chunk's first (Verlet) step
    int64_t ramp, step0, limit;
};

struct StreamArgs {
    const StreamInst *inst;     // batch launches: the instance descriptors
    uint32_t ninst, ntiles, tile, hcap, bcap, mmax;
    int64_t step;               // step of this launch within its chunk
    StreamInst one;             // single-simulation launches: the descriptor itself
};

}  // namespace pdk

// launchers (pd_force.hip, pd_tile.hip, pd_stream.hip)

int pd_launch_gather(pd_ctx ctx, int dim, const pdk::NodeArgs &a, int lanes, bool mixed);
int pd_launch_tile(pd_ctx ctx, int dim, const pdk::NodeArgs &a, int lanes, bool mixed,
                   int block);
// LDS bytes of one tile-kernel workgroup
size_t tile_lds_bytes(int dim, uint32_t hcap, uint32_t bcap, uint32_t tile, uint32_t mmax);
// the tile layout fits and every form of the tile kernel can be resident
bool pd_tile_resident(int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap, uint32_t bcap,
                      int lanes, int block, int num_cu);
// launch geometry of the persistent tile kernel; false if the layout does not fit
// (max_per_cu > 0 caps the workgroups per CU)
bool pd_tile_geometry(int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap, uint32_t bcap,
                      int block, int num_cu, int *rpt, unsigned *grid, uint32_t *mmax,
                      size_t *lds, int max_per_cu);
// streamed kernel (explicit steps with uniform volumes) ----------------------

// Forms of the streamed kernel: the linearised law, the NP law, and the two
// passes of the linear peridynamic solid (3-d, single simulation).  A solid
// step is a state-pass launch followed by a force-pass launch; its geometry
// is that of the force pass, whose LDS layout is the larger.
enum { SK_LINEAR = 0, SK_NP = 1, SK_LPS_STATE = 2, SK_LPS_FORCE = 3 };
// (batch: the kernel form that reads descriptors from device memory)
bool pd_stream_geometry(pd_ctx ctx, int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap,
                        uint32_t bcap, int lanes, int prec, bool batch, int form, int *block,
                        unsigned *grid, uint32_t *mmax, size_t *lds);
bool pd_stream_fits(int dim, uint32_t n, uint64_t nnz, uint64_t halo_total);
int pd_launch_stream(pd_ctx ctx, hipStream_t st, int dim, const pdk::StreamArgs &sa, int lanes,
                     int prec, int form, int block, unsigned grid, size_t lds);
// a simulation's streamed descriptor (static part), the launch arguments of a
// batch shaped like it (inst NULL: single-simulation form), and its host state
// after streamed steps
pdk::StreamInst pd_stream_inst(const pd_sim s);
pdk::StreamArgs pd_stream_args(const pd_sim sim, const pdk::StreamInst *inst, uint32_t ninst,
                               uint32_t ntiles);
void pd_sim_advanced(pd_sim sim, int64_t nsteps, double dt);
int pd_rec_pack(pd_ctx ctx, int dim, uint32_t n, const double *xv, const double *u, double *rec);
int pd_rec_unpack(pd_ctx ctx, int dim, uint32_t n, const double *rec, double *u);
// LDS halo capacity of a tiled neighbour list
inline uint32_t pd_tile_hcap(const pd_nbr nbr) { return (nbr->halo_max + 31u) & ~31u; }
inline uint32_t pd_tile_bcap(const pd_nbr nbr) { return (nbr->bonds_max + 63u) & ~63u; }
// bond words of a tiled neighbour list: bw = lcol | 0x8000 where alive == 0
// (bw arrays hold nnz + PD_BW_PAD entries, the pad marked dead, for the
// kernels' 32-bit reads, the streamed kernel's 16-byte copies and its bond
// loop's reads up to 6 L - 1 words past a row's end)
constexpr uint32_t PD_BW_PAD = 256;
int pd_bw_compose(pd_ctx ctx, const pd_nbr nbr, const uint8_t *alive_sfc, uint16_t *bw);
int pd_bw_to_alive(pd_ctx ctx, const pd_nbr nbr, const uint16_t *bw, uint8_t *alive_sfc);
