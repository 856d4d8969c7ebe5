// Streamed tiles: the explicit step (velocity Verlet with the bond-force
// gather, critical-stretch damage and boundary data; Algorithm 4 with the
// force of Algorithm 1) over LDS tiles whose staging runs asynchronously.
//
// Same tiles as the register-staged tile kernel (T consecutive sfc nodes,
// halo H_t, 16-bit tile-local bond words), but every global -> LDS copy is a
// gfx950 LDS DMA (global_load_lds_dword / _dwordx4): the data goes from L2
// straight into LDS without passing through registers, so the copies for tile
// k+1 stay in flight while the workgroup sums the bonds of tile k.  LDS holds
// one or two tile slots (records, bond words, row offsets, v and boundary
// kinds) plus the halo ids one tile further ahead.
//
// Node state lives in HBM as one record per node, {x y z ux uy uz} (2-d:
// {x y ux uy}); a record is 3 (2) 16-byte chunks, so a halo record is three
// (two) DMA lanes.  The node update writes u^{k+1} into the u part of the
// other record buffer (the positions are never rewritten).
//
// Per workgroup iteration k, with two slots (tile k in slot k mod 2):
//   wait for this wave's copies, barrier: tile k and the ids of tile k+1 are
//   in LDS, the sums of tile k-1 are done; write back the bond words of tile
//   k-1 that broke; issue the copies of tile k+1 into the other slot and of
//   the ids of tile k+2; sum the bonds of tile k, one lane group per node in
//   the gather kernel's summation order (so results are bit-identical to
//   it), and let lane 0 of each group update its node (kick, drift, boundary
//   data).  With one slot the copies of tile k+1 start after the sums of
//   tile k, and the other workgroups on the CU fill the wait.
#include <climits>

#include "pd_kernels.hpp"

namespace {

using namespace pdk;

typedef __attribute__((address_space(3))) char lds_char;

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const lds_char *)p;
}

// LDS DMA: lane l of the wave copies the 16 (4) bytes at base + voff into
// LDS at m0 + 16 l (m0 + 4 l).  m0 must be the same in every lane.  The copy
// is counted by the wave's vmcnt; dma_wait() waits for all of this wave's.
// The instructions are written out because the compiler's own form of them
// makes every later LDS read of the wave wait for the copy.
__device__ __forceinline__ void dma16(const void *base, uint32_t voff, uint32_t m0) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %1, %0"
                 :
                 : "s"(base), "v"(voff), "s"(m0)
                 : "memory", "m0");
}
__device__ __forceinline__ void dma4(const void *base, uint32_t voff, uint32_t m0) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dword %1, %0"
                 :
                 : "s"(base), "v"(voff), "s"(m0)
                 : "memory", "m0");
}
__device__ __forceinline__ void dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// barrier that orders LDS only (global traffic in flight stays in flight)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int META = 5;              // h0, hn, b0 (even), b1, self offset
constexpr uint16_t BW_DEAD = 0x8000;
constexpr uint32_t BRK_CAP = 256;    // broken bonds listed per tile (more: the whole tile)

inline __host__ __device__ uint32_t round4(uint32_t x) { return (x + 3u) & ~3u; }

// LDS layout, in this order (every region a multiple of 16 bytes).  NS tile
// slots (records, bond words, row offsets, v, boundary kinds), two halo-id
// slots, three break lists (tile k uses list k mod 3, so a list is cleared
// one tile before its next use without an extra barrier).
struct StreamLayout {
    uint32_t NS, H, T, WB, TP, TB, MM, RD, US;
    __host__ __device__ StreamLayout(int ns, int dim, uint32_t hcap, uint32_t bcap,
                                     uint32_t tile, uint32_t mmax) {
        NS = (uint32_t)ns;
        H = hcap;                      // multiple of 32
        T = tile;
        WB = round4(bcap / 2 + 2);     // 32-bit bond-word pairs per slot
        TP = round4(tile + 1);         // row offsets per slot
        TB = round4(tile / 4 + 1);     // 32-bit words of boundary kinds per slot
        MM = round4(mmax * META);
        RD = dim == 3 ? 6 : 4;         // doubles per record
        US = dim == 3 ? 4 : 2;         // doubles per node in v
    }
    __host__ __device__ size_t bytes() const {
        return (size_t)NS * H * RD * 8 + (size_t)2 * H * 4 + (size_t)NS * WB * 4 +
               (size_t)NS * TP * 4 + (size_t)NS * T * US * 8 + (size_t)NS * TB * 4 +
               (size_t)3 * (BRK_CAP + 4) * 4 + (size_t)MM * 4;
    }
};

// NS = 2: the copies of tile k+1 fly while tile k is summed (one workgroup
// holds both slots).  NS = 1: one slot, copies start after the sums, and the
// workgroups sharing a CU cover each other's waits.
template <int DIM, int L, bool MIXED, int NS>
__global__ __launch_bounds__(1024) void stream_kernel(NodeArgs a) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    constexpr uint32_t RD = DIM == 3 ? 6 : 4, NCH = RD / 2, US = DIM == 3 ? 4 : 2;
    const StreamLayout lay(NS, DIM, a.hcap, a.bcap, a.tile, a.mmax);
    const uint32_t H = lay.H, T = lay.T, WB = lay.WB, TP = lay.TP, TB = lay.TB;
    const uint32_t B = blockDim.x, tid = threadIdx.x, lane64 = tid & 63u, wbase = tid - lane64;
    double *recs = lds;                                                          // NS H RD
    int32_t *ids = reinterpret_cast<int32_t *>(recs + (size_t)NS * H * RD);      // 2 H
    uint32_t *words = reinterpret_cast<uint32_t *>(ids + (size_t)2 * H);         // NS WB
    uint32_t *rowp = words + (size_t)NS * WB;                                    // NS TP
    double *vbuf = reinterpret_cast<double *>(rowp + (size_t)NS * TP);           // NS T US
    uint32_t *bcb = reinterpret_cast<uint32_t *>(vbuf + (size_t)NS * T * US);    // NS TB
    uint32_t *brk = bcb + (size_t)NS * TB;                                       // 3 (4 + CAP)
    uint32_t *meta = brk + 3 * (BRK_CAP + 4);                                    // MM
    const bool wants_v = mode_reads_v(a.mode);
    auto slot = [&](uint32_t k) { return NS == 2 ? (k & 1u) : 0u; };

    // persistent schedule: the tiles of this XCD's contiguous range, strided
    // over the XCD's workgroups
    const uint32_t nb = gridDim.x, x = blockIdx.x % 8, l = blockIdx.x / 8;
    const uint32_t gx = nb / 8 + (x < nb % 8 ? 1u : 0u);
    const uint32_t tq = a.ntiles / 8, tr = a.ntiles % 8;
    const uint32_t tbeg = x * tq + (x < tr ? x : tr), tcnt = tq + (x < tr ? 1u : 0u);
    const uint32_t K = l < tcnt ? (tcnt - l + gx - 1) / gx : 0u;
    if (K == 0) return;
    auto tile_of = [&](uint32_t k) { return tbeg + l + k * gx; };

    for (uint32_t k = tid; k < K; k += B) {
        const uint32_t t = tile_of(k), t0 = t * T, tn = min(T, a.n - t0);
        const uint32_t h0 = a.halo_ptr[t];
        uint32_t *m = meta + (size_t)k * META;
        m[0] = h0;
        m[1] = a.halo_ptr[t + 1] - h0;
        m[2] = a.row_ptr[t0] & ~1u;
        m[3] = a.row_ptr[t0 + tn];
        m[4] = a.self_off[t];
    }
    auto blist = [&](uint32_t k) { return brk + (k % 3u) * (BRK_CAP + 4); };
    if (tid < 3) brk[tid * (BRK_CAP + 4)] = 0;
    __syncthreads();

    // halo ids of tile k -> ids slot k mod 2
    auto issue_ids = [&](uint32_t k) {
        const uint32_t h0 = meta[k * META], hn = meta[k * META + 1];
        int32_t *dst = ids + (size_t)(k & 1u) * H;
        for (uint32_t c0 = wbase; c0 < hn; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(dst + c0));
            if (c0 + lane64 < hn) dma4(a.halo, (h0 + c0 + lane64) * 4u, m0);
        }
    };
    // records, bond words, row offsets, v and boundary kinds of tile k ->
    // its slot (the ids of tile k are in ids slot k mod 2)
    auto issue_tile = [&](uint32_t k) {
        const uint32_t s = slot(k), t = tile_of(k), t0 = t * T, tn = min(T, a.n - t0);
        const uint32_t hn = meta[k * META + 1], b0 = meta[k * META + 2], b1 = meta[k * META + 3];
        const int32_t *hid = ids + (size_t)(k & 1u) * H;
        double *rdst = recs + (size_t)s * H * RD;
        const uint32_t nrc = hn * NCH;
        for (uint32_t c0 = wbase; c0 < nrc; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(rdst + 2 * (size_t)c0));
            const uint32_t c = c0 + lane64;
            if (c < nrc) {
                const uint32_t r = c / NCH, part = c - r * NCH;
                dma16(a.rec, (uint32_t)hid[r] * (RD * 8u) + part * 16u, m0);
            }
        }
        const uint32_t nw = (b1 - b0 + 1) / 2;
        uint32_t *wdst = words + (size_t)s * WB;
        for (uint32_t c0 = wbase; c0 < nw; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(wdst + c0));
            if (c0 + lane64 < nw) dma4(a.bw, (b0 / 2 + c0 + lane64) * 4u, m0);
        }
        uint32_t *pdst = rowp + (size_t)s * TP;
        for (uint32_t c0 = wbase; c0 <= tn; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(pdst + c0));
            if (c0 + lane64 <= tn) dma4(a.row_ptr, (t0 + c0 + lane64) * 4u, m0);
        }
        if (wants_v) {
            const uint32_t nvc = tn * US / 2;
            double *vdst = vbuf + (size_t)s * T * US;
            for (uint32_t c0 = wbase; c0 < nvc; c0 += B) {
                const uint32_t m0 =
                    __builtin_amdgcn_readfirstlane(lds_addr(vdst + 2 * (size_t)c0));
                if (c0 + lane64 < nvc) dma16(a.v, (t0 * US + 2 * (c0 + lane64)) * 8u, m0);
            }
        }
        if (a.bc) {
            const uint32_t nbw = (tn + 3) / 4;   // the array is padded to whole words
            uint32_t *bdst = bcb + (size_t)s * TB;
            for (uint32_t c0 = wbase; c0 < nbw; c0 += B) {
                const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(bdst + c0));
                if (c0 + lane64 < nbw) dma4(a.bc, t0 + 4 * (c0 + lane64), m0);
            }
        }
    };

    // bond sums of tile k; lane 0 of each node's group then updates the node
    // (kick, drift, boundary data).  A bond that breaks gets its dead bit in
    // the slot's copy of the words and goes on the tile's break list.
    auto sum_and_update = [&](uint32_t k) {
        const uint32_t s = slot(k), t = tile_of(k), t0 = t * T, tn = min(T, a.n - t0);
        const uint32_t b0 = meta[k * META + 2], so = meta[k * META + 4];
        const double *rec = recs + (size_t)s * H * RD;
        uint16_t *w16 = reinterpret_cast<uint16_t *>(words + (size_t)s * WB);
        const uint32_t *rp = rowp + (size_t)s * TP;
        uint32_t *bl = blist(k);
        const uint32_t groups = B / L, g = tid / L;
        const int lane = tid & (L - 1);
        const double cv = a.cv_uniform;
        for (uint32_t q = g; q < tn; q += groups) {
            const double *ri = rec + (size_t)(so + q) * RD;
            const double xix = ri[0], xiy = ri[1], xiz = DIM == 3 ? ri[2] : 0.0;
            const double uix = ri[DIM], uiy = ri[DIM + 1], uiz = DIM == 3 ? ri[DIM + 2] : 0.0;
            Acc64 acc;
            const uint32_t rs = rp[q] - b0, re = rp[q + 1] - b0;
            for (uint32_t p = rs + lane; p < re; p += L) {
                const uint32_t w = w16[p];
                const double2 *rj =
                    reinterpret_cast<const double2 *>(rec + (size_t)(w & 0x7fffu) * RD);
                const double2 c0 = rj[0], c1 = rj[1];
                double dxx, dxy, dxz, dux, duy, duz;
                if (DIM == 3) {
                    const double2 c2 = rj[2];
                    dxx = c0.x - xix; dxy = c0.y - xiy; dxz = c1.x - xiz;
                    dux = c1.y - uix; duy = c2.x - uiy; duz = c2.y - uiz;
                } else {
                    dxx = c0.x - xix; dxy = c0.y - xiy; dxz = 0.0;
                    dux = c1.x - uix; duy = c1.y - uiy; duz = 0.0;
                }
                if (bond<DIM, MIXED, false>(a, dxx, dxy, dxz, dux, duy, duz, cv,
                                            (w & BW_DEAD) != 0, acc)) {
                    // a break: dead bit in the slot's copy, entry on the list
                    const uint32_t nw = (uint32_t)(w | BW_DEAD);
                    w16[p] = (uint16_t)nw;
                    const uint32_t e = atomicAdd(bl, 1u);
                    if (e < BRK_CAP) bl[4 + e] = (p << 16) | nw;
                }
            }
            double fx, fy, fz, Ue;
            group_reduce<DIM, L, false>(acc, fx, fy, fz, Ue);
            // node update, one lane per component (the same arithmetic as
            // node_update's explicit-step branch, so results stay identical)
            if (lane < (int)DIM) {
                const uint32_t d = (uint32_t)lane, i = t0 + q;
                const double fd = d == 0 ? fx : (d == 1 ? fy : fz);
                const double ud = ri[DIM + d];
                double vd = wants_v ? vbuf[(size_t)s * T * US + (size_t)q * US + d] : 0.0;
                const int kind =
                    a.bc ? (int)reinterpret_cast<const uint8_t *>(bcb + (size_t)s * TB)[q]
                         : PD_BC_FREE;
                const double hdt = 0.5 * a.dt;
                double nd;
                if (kind == PD_BC_FREE) {
                    const double bd = a.b ? a.b[(size_t)i * US + d] : 0.0;
                    if (a.mode == M_STEP_CONT) vd = vd + hdt * (fd + bd) / a.rho;
                    vd = vd + hdt * (fd + bd) / a.rho;
                    nd = ud + a.dt * vd;
                } else if (kind == PD_BC_CLAMPED) {
                    vd = 0.0;
                    nd = 0.0;
                } else {
                    vd = a.r_half * a.bc_vel[(size_t)i * US + d];
                    nd = ud + a.dt * vd;
                }
                a.v[(size_t)i * US + d] = vd;
                a.rec_out[(size_t)i * RD + DIM + d] = nd;
            }
        }
    };

    // the bond words of tile k that broke go back to HBM; a tile with more
    // breaks than the list holds writes back all its words from its slot
    // (the caller guarantees that slot is still intact)
    auto write_back = [&](uint32_t k, bool from_slot) {
        const uint32_t *bl = blist(k);
        const uint32_t b0 = meta[k * META + 2];
        if (!from_slot) {
            const uint32_t ne = min(bl[0], BRK_CAP);
            for (uint32_t e = tid; e < ne; e += B) {
                const uint32_t v = bl[4 + e];
                a.bw[b0 + (v >> 16)] = (uint16_t)(v & 0xffffu);
            }
        } else {
            const uint32_t s = slot(k), t0 = tile_of(k) * T, tn = min(T, a.n - t0);
            const uint32_t *rp = rowp + (size_t)s * TP;
            const uint16_t *w16 = reinterpret_cast<const uint16_t *>(words + (size_t)s * WB);
            const uint32_t rs = rp[0] - b0, re = rp[tn] - b0;
            for (uint32_t q = rs + tid; q < re; q += B) a.bw[b0 + q] = w16[q];
        }
    };

    issue_ids(0);
    if (K > 1) issue_ids(1);
    dma_wait();
    __syncthreads();
    issue_tile(0);
    for (uint32_t k = 0; k < K; ++k) {
        dma_wait();
        lds_barrier();                       // tile k and the ids of tile k+1 are in LDS
        if (tid == 0) blist(k + 1)[0] = 0;   // last read for tile k-2
        if (NS == 2) {
            if (k > 0) {                     // breaks of tile k-1, whose slot is reused below
                const uint32_t nbk = blist(k - 1)[0];
                if (nbk) write_back(k - 1, nbk > BRK_CAP);
                if (nbk > BRK_CAP) lds_barrier();
            }
            if (k + 1 < K) issue_tile(k + 1);
            if (k + 2 < K) issue_ids(k + 2);
            sum_and_update(k);
        } else {
            sum_and_update(k);
            lds_barrier();                   // the slot is free once the sums are done
            const uint32_t nbk = blist(k)[0];
            if (nbk) write_back(k, nbk > BRK_CAP);
            if (nbk > BRK_CAP) lds_barrier();
            if (k + 1 < K) issue_tile(k + 1);
            if (k + 2 < K) issue_ids(k + 2);
        }
    }
    if (NS == 2) {
        lds_barrier();
        const uint32_t nbk = blist(K - 1)[0];
        if (nbk) write_back(K - 1, nbk > BRK_CAP);
    }
}

template <int DIM>
void *pick_stream(int lanes, bool mixed, int ns) {
#define PD_SK(Lv)                                                                          \
    case Lv:                                                                               \
        if (ns == 2)                                                                       \
            return mixed ? (void *)stream_kernel<DIM, Lv, true, 2>                         \
                         : (void *)stream_kernel<DIM, Lv, false, 2>;                       \
        return mixed ? (void *)stream_kernel<DIM, Lv, true, 1> : (void *)stream_kernel<DIM, Lv, false, 1>;
    switch (lanes) {
        PD_SK(2)
        PD_SK(4)
        PD_SK(8)
        PD_SK(16)
        PD_SK(32)
    default: return nullptr;
    }
#undef PD_SK
}

// records {x y z ux uy uz} (2-d {x y ux uy}) from xv and u
template <int DIM>
__global__ void rec_pack_k(uint32_t n, const double *xv, const double *u, double *rec) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int RD = DIM == 3 ? 6 : 4, US = DIM == 3 ? 4 : 2;
    for (int d = 0; d < DIM; ++d) {
        rec[(size_t)i * RD + d] = xv[4 * (size_t)i + d];
        rec[(size_t)i * RD + DIM + d] = u[(size_t)i * US + d];
    }
}

template <int DIM>
__global__ void rec_unpack_k(uint32_t n, const double *rec, double *u) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int RD = DIM == 3 ? 6 : 4, US = DIM == 3 ? 4 : 2;
    for (int d = 0; d < US; ++d) u[(size_t)i * US + d] = d < DIM ? rec[(size_t)i * RD + DIM + d] : 0.0;
}

}  // namespace

// tile slots per workgroup: 1 lets two or more workgroups share a CU
constexpr int STREAM_SLOTS = 1;

// Launch geometry of the streamed kernel; false if it cannot run this layout.
bool pd_stream_geometry(pd_ctx ctx, int dim, uint32_t n, uint64_t nnz, uint32_t ntiles,
                        uint32_t tile, uint32_t hcap, uint32_t bcap, uint64_t halo_total,
                        int lanes, bool mixed, int *block, unsigned *grid, uint32_t *mmax,
                        size_t *lds, int *slots) {
    const uint32_t B = tile * (uint32_t)lanes;
    if (B < 64 || B > 1024 || B % 64 != 0) return false;
    if (lanes < dim) return false;   // the node update takes one lane per component
    const uint32_t RB = dim == 3 ? 48u : 32u;
    // 32-bit byte offsets of every copy; 16-bit tile-local bond positions
    if ((uint64_t)n * RB >= (1ull << 32) || 2 * nnz + 16 >= (1ull << 32) ||
        halo_total * 4 >= (1ull << 32) || bcap >= (1u << 16))
        return false;
    const int ns = STREAM_SLOTS;
    void *k = dim == 3 ? pick_stream<3>(lanes, mixed, ns) : pick_stream<2>(lanes, mixed, ns);
    if (!k) return false;
    for (int pass = 0; pass < 2; ++pass) {
        // first pass: one workgroup per CU gives the tile bound; second pass:
        // as many per CU as LDS and registers allow
        unsigned g = (unsigned)ctx->num_cu;
        if (pass == 1) {
            int per_cu = 0;
            const size_t bytes = StreamLayout(ns, dim, hcap, bcap, tile, *mmax).bytes();
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, (int)B,
                                                             bytes) != hipSuccess)
                return false;
            if (per_cu < 1) return false;
            g = (unsigned)(ctx->num_cu * per_cu);
        }
        if (g > ntiles) g = ntiles;
        if (g < 8 && ntiles >= 8) g = 8;
        if (g < 1) g = 1;
        uint32_t m = 0;
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t gx = g / 8 + (x < g % 8 ? 1u : 0u);
            const uint32_t tc = ntiles / 8 + (x < ntiles % 8 ? 1u : 0u);
            if (gx == 0) {
                if (tc) return false;
                continue;
            }
            const uint32_t kk = (tc + gx - 1) / gx;
            if (kk > m) m = kk;
        }
        const size_t bytes = StreamLayout(ns, dim, hcap, bcap, tile, m).bytes();
        if (bytes > 160 * 1024) return false;
        *mmax = m;
        *lds = bytes;
        *grid = g;
    }
    *block = (int)B;
    *slots = ns;
    return true;
}

int pd_launch_stream(pd_ctx ctx, int dim, const NodeArgs &a, int lanes, bool mixed, int block,
                     unsigned grid, size_t lds, int slots) {
    void *k = dim == 3 ? pick_stream<3>(lanes, mixed, slots)
                       : pick_stream<2>(lanes, mixed, slots);
    if (!k) return pd_set_error(ctx, PD_EINVAL, "streamed kernel needs 2..32 lanes");
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    NodeArgs args = a;
    void *argv[] = {&args};
    PD_HIP(ctx, hipLaunchKernel(k, dim3(grid), dim3(block), argv, lds, ctx->stream));
    return PD_OK;
}

int pd_rec_pack(pd_ctx ctx, int dim, uint32_t n, const double *xv, const double *u, double *rec) {
    if (dim == 3) rec_pack_k<3><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, xv, u, rec);
    else rec_pack_k<2><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, xv, u, rec);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_rec_unpack(pd_ctx ctx, int dim, uint32_t n, const double *rec, double *u) {
    if (dim == 3) rec_unpack_k<3><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, rec, u);
    else rec_unpack_k<2><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, rec, u);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}
