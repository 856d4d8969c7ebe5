// LDS-staged tiles for the bond-force gather.
//
// A tile is T consecutive nodes in sfc order.  Its halo H_t is the sorted set
// of all nodes its bonds touch (its own nodes included).  Per launch, one
// workgroup per tile copies the records {X, V, u} of H_t from HBM/L2 into LDS
// (sorted ids come in long contiguous runs, so these loads coalesce), then
// every bond reads its neighbour from LDS through a 16-bit tile-local index
// (lcol), which also halves the per-bond index stream.  The per-node
// summation order is the gather kernel's (same lanes, same butterfly), so
// both kernels give bit-identical results.
//
// Build (once per neighbour list and tile size), one workgroup per tile:
// insert the ids into an LDS hash set, compact, bitonic-sort, then find each
// bond's local index by binary search.
#include <climits>
#include <vector>

#include "pd_kernels.hpp"

namespace {

using namespace pdk;

constexpr int TB_BUILD = 256;
constexpr int HASH_CAP = 8192;      // LDS hash slots (int32)
constexpr int HALO_MAX = 4096;      // largest halo a tile may have

__device__ __forceinline__ uint32_t hash_id(int32_t id) {
    return ((uint32_t)id * 2654435761u) & (HASH_CAP - 1);
}

// insert into the LDS hash set; counts new ids in *cnt (stops at HALO_MAX)
__device__ void hash_insert(int32_t *table, int *cnt, int32_t id) {
    if (*(volatile int *)cnt >= HALO_MAX) return;
    uint32_t h = hash_id(id);
    while (true) {
        const int32_t prev = atomicCAS(&table[h], -1, id);
        if (prev == -1) {
            atomicAdd(cnt, 1);
            return;
        }
        if (prev == id) return;
        h = (h + 1) & (HASH_CAP - 1);
    }
}

__device__ void fill_hash(int32_t *table, int *cnt, uint32_t t0, uint32_t t1,
                          const uint32_t *row_ptr, const int32_t *col) {
    for (int k = threadIdx.x; k < HASH_CAP; k += TB_BUILD) table[k] = -1;
    if (threadIdx.x == 0) *cnt = 0;
    __syncthreads();
    for (uint32_t i = t0 + threadIdx.x; i < t1; i += TB_BUILD) hash_insert(table, cnt, (int32_t)i);
    const uint32_t a = row_ptr[t0], e = row_ptr[t1];
    for (uint32_t p = a + threadIdx.x; p < e; p += TB_BUILD) hash_insert(table, cnt, col[p]);
    __syncthreads();
}

__global__ __launch_bounds__(TB_BUILD) void tile_count_k(uint32_t n, uint32_t T,
                                                         const uint32_t *row_ptr,
                                                         const int32_t *col, uint32_t *count,
                                                         uint32_t *bonds, int *overflow) {
    __shared__ int32_t table[HASH_CAP];
    __shared__ int cnt;
    const uint32_t t = blockIdx.x;
    const uint32_t t0 = t * T, t1 = min(n, t0 + T);
    fill_hash(table, &cnt, t0, t1, row_ptr, col);
    if (threadIdx.x == 0) {
        count[t] = (uint32_t)cnt;
        bonds[t] = row_ptr[t1] - row_ptr[t0];
        if (cnt >= HALO_MAX) atomicOr(overflow, 1);
    }
}

__device__ uint32_t lower_bound(const int32_t *a, uint32_t len, int32_t key) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(TB_BUILD) void tile_fill_k(uint32_t n, uint32_t T,
                                                        const uint32_t *row_ptr,
                                                        const int32_t *col,
                                                        const uint32_t *halo_ptr, int32_t *halo,
                                                        uint32_t *self_off, uint16_t *lcol) {
    __shared__ int32_t table[HASH_CAP];
    __shared__ int32_t keys[HALO_MAX];
    __shared__ int cnt, pos;
    const uint32_t t = blockIdx.x;
    const uint32_t t0 = t * T, t1 = min(n, t0 + T);
    fill_hash(table, &cnt, t0, t1, row_ptr, col);
    const int m = cnt;   // < HALO_MAX (checked by the count pass)
    int P = 1;
    while (P < m) P <<= 1;
    if (threadIdx.x == 0) pos = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < HASH_CAP; k += TB_BUILD)
        if (table[k] != -1) keys[atomicAdd(&pos, 1)] = table[k];
    __syncthreads();
    for (int k = m + threadIdx.x; k < P; k += TB_BUILD) keys[k] = INT_MAX;
    __syncthreads();
    // bitonic sort of keys[0, P)
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = threadIdx.x; k < P; k += TB_BUILD) {
                const int partner = k ^ stride;
                if (partner > k) {
                    const bool up = (k & size) == 0;
                    const int32_t x = keys[k], y = keys[partner];
                    if ((x > y) == up) {
                        keys[k] = y;
                        keys[partner] = x;
                    }
                }
            }
            __syncthreads();
        }
    const uint32_t h0 = halo_ptr[t];
    for (int k = threadIdx.x; k < m; k += TB_BUILD) halo[h0 + k] = keys[k];
    if (threadIdx.x == 0) self_off[t] = lower_bound(keys, (uint32_t)m, (int32_t)t0);
    const uint32_t a = row_ptr[t0], e = row_ptr[t1];
    for (uint32_t p = a + threadIdx.x; p < e; p += TB_BUILD)
        lcol[p] = (uint16_t)lower_bound(keys, (uint32_t)m, col[p]);
}

// ---------------------------------------------------------------------------
// tile kernel: stage the halo records and the tile's bond streams in LDS,
// then one group of L lanes per node
// ---------------------------------------------------------------------------
template <int DIM>
struct Rec {
    static constexpr int NC = DIM == 3 ? 7 : 5;   // {x y [z] V ux uy [uz]}
    static constexpr int V = DIM;                 // index of V
    static constexpr int U = DIM + 1;             // index of ux
};

template <int DIM, int L, bool MIXED, bool WANT_E>
__global__ void tile_kernel(NodeArgs a) {
    if (a.done && *a.done) return;
    extern __shared__ double lds[];
    constexpr int NC = Rec<DIM>::NC, IV = Rec<DIM>::V, IU = Rec<DIM>::U;
    double *rec = lds;                                            // [hcap][NC]
    uint16_t *sbw = reinterpret_cast<uint16_t *>(lds + (size_t)a.hcap * NC);
    const uint32_t t = pd_xcd_tile(blockIdx.x, gridDim.x);
    const bool tangent = a.mode == M_TANGENT;
    const uint32_t t0 = t * a.tile;
    const uint32_t tn = min(a.tile, a.n - t0);
    const uint32_t b0 = a.row_ptr[t0], bn = a.row_ptr[t0 + tn] - b0;

    // stage the halo records and the tile's bond words
    const uint32_t h0 = a.halo_ptr[t], hn = a.halo_ptr[t + 1] - h0;
    for (uint32_t k = threadIdx.x; k < hn; k += blockDim.x) {
        const uint32_t id = (uint32_t)a.halo[h0 + k];
        const double4 q = reinterpret_cast<const double4 *>(a.xv)[id];
        double ux, uy, uz;
        load_vec<DIM>(a.u, id, ux, uy, uz);
        if (tangent && a.bc && a.bc[id]) { ux = 0; uy = 0; uz = 0; }
        double *r = rec + (size_t)k * NC;
        r[0] = q.x;
        r[1] = q.y;
        if (DIM == 3) { r[2] = q.z; r[IV] = q.w; } else { r[IV] = q.z; }
        r[IU] = ux;
        r[IU + 1] = uy;
        if (DIM == 3) r[IU + 2] = uz;
    }
    for (uint32_t k = threadIdx.x; k < bn; k += blockDim.x) sbw[k] = a.bw[b0 + k];
    __syncthreads();

    const uint32_t so = a.self_off[t];
    const uint32_t groups = blockDim.x / L;
    const uint32_t g = threadIdx.x / L;
    const int lane = threadIdx.x & (L - 1);
    for (uint32_t q = g; q < tn; q += groups) {
        const uint32_t i = t0 + q;
        const double *ri = rec + (size_t)(so + q) * NC;
        const double xix = ri[0], xiy = ri[1], xiz = DIM == 3 ? ri[2] : 0.0, Vi = ri[IV];
        const double uix = ri[IU], uiy = ri[IU + 1], uiz = DIM == 3 ? ri[IU + 2] : 0.0;
        const bool fixed_i = tangent && a.bc && a.bc[i];
        Acc64 s64;
        Acc32 s32;
        const uint32_t rs = a.row_ptr[i] - b0, re = a.row_ptr[i + 1] - b0;
        // each lane takes bonds rs+lane, rs+lane+L, ... in this order, two at a time
        uint32_t p = rs + lane;
        for (; p + L < re; p += 2 * L) {
            const uint16_t w0 = sbw[p], w1 = sbw[p + L];
            const double *r0 = rec + (size_t)(w0 & BW_IDX) * NC;
            const double *r1 = rec + (size_t)(w1 & BW_IDX) * NC;
            double A[NC], B[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) { A[c] = r0[c]; B[c] = r1[c]; }
            if (!(w0 & BW_DEAD) &&
                bond<DIM, MIXED, WANT_E>(a, A[0] - xix, A[1] - xiy, DIM == 3 ? A[2] - xiz : 0.0,
                                         A[IU] - uix, A[IU + 1] - uiy,
                                         DIM == 3 ? A[IU + 2] - uiz : 0.0, A[IV], s64, s32))
                a.bw[b0 + p] = w0 | BW_DEAD;
            if (!(w1 & BW_DEAD) &&
                bond<DIM, MIXED, WANT_E>(a, B[0] - xix, B[1] - xiy, DIM == 3 ? B[2] - xiz : 0.0,
                                         B[IU] - uix, B[IU + 1] - uiy,
                                         DIM == 3 ? B[IU + 2] - uiz : 0.0, B[IV], s64, s32))
                a.bw[b0 + p + L] = w1 | BW_DEAD;
        }
        if (p < re) {
            const uint16_t w0 = sbw[p];
            const double *r0 = rec + (size_t)(w0 & BW_IDX) * NC;
            if (!(w0 & BW_DEAD) &&
                bond<DIM, MIXED, WANT_E>(a, r0[0] - xix, r0[1] - xiy, DIM == 3 ? r0[2] - xiz : 0.0,
                                         r0[IU] - uix, r0[IU + 1] - uiy,
                                         DIM == 3 ? r0[IU + 2] - uiz : 0.0, r0[IV], s64, s32))
                a.bw[b0 + p] = w0 | BW_DEAD;
        }
        double fx, fy, fz, Ue;
        group_reduce<DIM, L, MIXED, WANT_E>(s64, s32, fx, fy, fz, Ue);
        if (lane == 0) {
            // a fixed node's own w is zero in LDS; node_update re-reads it
            node_update<DIM>(a, i, fx, fy, fz, Ue, Vi, uix, uiy, uiz, fixed_i);
        }
    }
}

__global__ void bw_compose_k(uint64_t nnz, const uint16_t *lcol, const uint8_t *alive,
                             uint16_t *bw) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) bw[p] = lcol[p] | ((alive && !alive[p]) ? BW_DEAD : (uint16_t)0);
}

__global__ void bw_alive_k(uint64_t nnz, const uint16_t *bw, uint8_t *alive) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) alive[p] = (bw[p] & BW_DEAD) ? 0 : 1;
}


template <int DIM, int L>
int launch_t(pd_ctx ctx, const NodeArgs &a, bool mixed, int block) {
    const unsigned grid = (a.n + a.tile - 1) / a.tile;
    if (grid == 0) return PD_OK;
    const size_t lds = tile_lds_bytes(DIM, a.hcap, a.bcap);
    void (*k)(NodeArgs);
    const bool e = mode_wants_energy(a);
    if (mixed) k = e ? tile_kernel<DIM, L, true, true> : tile_kernel<DIM, L, true, false>;
    else k = e ? tile_kernel<DIM, L, false, true> : tile_kernel<DIM, L, false, false>;
    (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    k<<<grid, block, lds, ctx->stream>>>(a);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

template <int DIM>
int launch_d(pd_ctx ctx, const NodeArgs &a, int lanes, bool mixed, int block) {
    switch (lanes) {
    case 1: return launch_t<DIM, 1>(ctx, a, mixed, block);
    case 2: return launch_t<DIM, 2>(ctx, a, mixed, block);
    case 4: return launch_t<DIM, 4>(ctx, a, mixed, block);
    case 8: return launch_t<DIM, 8>(ctx, a, mixed, block);
    case 16: return launch_t<DIM, 16>(ctx, a, mixed, block);
    case 32: return launch_t<DIM, 32>(ctx, a, mixed, block);
    case 64: return launch_t<DIM, 64>(ctx, a, mixed, block);
    default: return pd_set_error(ctx, PD_EINVAL, "unsupported lane count %d", lanes);
    }
}

}  // namespace

size_t tile_lds_bytes(int dim, uint32_t hcap, uint32_t bcap) {
    const int nc = dim == 3 ? 7 : 5;
    return (size_t)hcap * nc * sizeof(double) + (size_t)bcap * sizeof(uint16_t);
}

int pd_launch_tile(pd_ctx ctx, int dim, const NodeArgs &a, int lanes, bool mixed, int block) {
    return dim == 3 ? launch_d<3>(ctx, a, lanes, mixed, block)
                    : launch_d<2>(ctx, a, lanes, mixed, block);
}

int pd_bw_compose(pd_ctx ctx, const pd_nbr nbr, const uint8_t *alive_sfc, uint16_t *bw) {
    bw_compose_k<<<pd_blocks(nbr->nnz), PD_BLOCK, 0, ctx->stream>>>(nbr->nnz, nbr->lcol,
                                                                     alive_sfc, bw);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_bw_to_alive(pd_ctx ctx, const pd_nbr nbr, const uint16_t *bw, uint8_t *alive_sfc) {
    bw_alive_k<<<pd_blocks(nbr->nnz), PD_BLOCK, 0, ctx->stream>>>(nbr->nnz, bw, alive_sfc);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

// Builds (or rebuilds for another T) the tile structure of a neighbour list.
// Returns PD_ECAPACITY if some tile's halo exceeds HALO_MAX records.
int pd_nbr_build_tiles(pd_ctx ctx, pd_nbr nbr, uint32_t T) {
    if (nbr->tile_T == T && nbr->lcol) return PD_OK;
    pd_free(nbr->halo_ptr);
    pd_free(nbr->halo);
    pd_free(nbr->self_off);
    pd_free(nbr->lcol);
    nbr->tile_T = 0;
    const uint32_t n = nbr->n;
    const uint32_t ntiles = (n + T - 1) / T;
    hipStream_t st = ctx->stream;
    uint32_t *count = nullptr, *bonds = nullptr;
    uint64_t *scan = nullptr;
    int status = PD_OK;
    auto cleanup = [&]() {
        pd_free(count);
        pd_free(bonds);
        pd_free(scan);
    };
    if ((status = pd_alloc(ctx, &count, ntiles)) != PD_OK) return status;
    if ((status = pd_alloc(ctx, &bonds, ntiles)) != PD_OK) return cleanup(), status;
    if ((status = pd_alloc(ctx, &scan, (size_t)ntiles + 1)) != PD_OK) return cleanup(), status;
    if ((status = pd_flag_clear(ctx)) != PD_OK) return cleanup(), status;
    tile_count_k<<<ntiles, TB_BUILD, 0, st>>>(n, T, nbr->row_ptr, nbr->col, count, bonds,
                                              ctx->flag);
    if (hipGetLastError() != hipSuccess) return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile_count_k");
    int overflow = 0;
    if ((status = pd_flag_read(ctx, &overflow)) != PD_OK) return cleanup(), status;
    if (overflow) return cleanup(), PD_ECAPACITY;
    if ((status = pd_scan_u32(ctx, count, scan, ntiles)) != PD_OK) return cleanup(), status;
    uint64_t total = 0;
    if (hipMemcpy(&total, scan + ntiles, sizeof total, hipMemcpyDeviceToHost) != hipSuccess)
        return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile scan copy");
    // largest halo
    std::vector<uint32_t> hc(ntiles);
    if (hipMemcpy(hc.data(), count, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess)
        return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile count copy");
    uint32_t hmax = 0;
    for (uint32_t c : hc) hmax = c > hmax ? c : hmax;
    if (hipMemcpy(hc.data(), bonds, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost) != hipSuccess)
        return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile bond count copy");
    uint32_t bmax = 0;
    for (uint32_t c : hc) bmax = c > bmax ? c : bmax;
    if ((status = pd_alloc(ctx, &nbr->halo_ptr, (size_t)ntiles + 1)) != PD_OK) return cleanup(), status;
    if ((status = pd_narrow_u64(ctx, scan, nbr->halo_ptr, ntiles)) != PD_OK) return cleanup(), status;
    if ((status = pd_alloc(ctx, &nbr->halo, total)) != PD_OK) return cleanup(), status;
    if ((status = pd_alloc(ctx, &nbr->self_off, ntiles)) != PD_OK) return cleanup(), status;
    if ((status = pd_alloc(ctx, &nbr->lcol, nbr->nnz)) != PD_OK) return cleanup(), status;
    tile_fill_k<<<ntiles, TB_BUILD, 0, st>>>(n, T, nbr->row_ptr, nbr->col, nbr->halo_ptr,
                                             nbr->halo, nbr->self_off, nbr->lcol);
    if (hipGetLastError() != hipSuccess) return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile_fill_k");
    if (hipStreamSynchronize(st) != hipSuccess) return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile sync");
    cleanup();
    nbr->tile_T = T;
    nbr->ntiles = ntiles;
    nbr->halo_max = hmax;
    nbr->bonds_max = bmax;
    nbr->halo_total = total;
    return PD_OK;
}
