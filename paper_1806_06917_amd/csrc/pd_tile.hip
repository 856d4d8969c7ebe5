// LDS-staged tiles for the bond-force gather.
//
// A tile is T consecutive nodes in sfc order.  Its halo H_t is the sorted set
// of all nodes its bonds touch (its own nodes included).  Per launch, one
// workgroup per tile copies the records {X, V, u} of H_t from HBM/L2 into LDS
// (sorted ids come in long contiguous runs, so these loads coalesce), then
// every bond reads its neighbour from LDS through a 16-bit tile-local index
// (lcol), which also halves the per-bond index stream.  The per-node
// summation order is the gather kernel's (same lanes, same reduction), so
// both kernels give bit-identical results.
//
// Build (once per neighbour list and tile size), one workgroup per tile:
// insert the ids into an LDS hash set, compact, bitonic-sort, then find each
// bond's local index by binary search.
#include <climits>
#include <type_traits>
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
// tile kernel
//
// Persistent: workgroup b works through the tiles tbeg + l, tbeg + l + gx, ...
// of the contiguous tile range its XCD owns (x = b mod 8, l = b / 8, gx
// workgroups on that XCD), so neighbouring tiles share an L2.  Three-stage
// software pipeline over those tiles:
//   ids(k+2)  halo ids of the tile after next          -> registers
//   recs(k+1) halo records, bond words, row offsets     -> registers
//   tile k    from LDS: bond sums, then the node updates
// so the HBM/L2 latency of staging a tile hides behind the previous tile's
// arithmetic.  Per-tile metadata for all of the workgroup's tiles is read
// into LDS once at the start, so no prefetch waits on a dependent load.
// LDS holds each halo record as {x y z ux uy uz} (2-d: {x y ux uy} padded):
// a 48-byte stride puts the 16-byte reads of eight consecutive records in
// eight disjoint bank windows (rows are sorted by sfc id, so a node's lanes
// mostly read consecutive records).  c V_j lives in its own array and is not
// read at all when every node has the same volume.  A broken bond keeps its
// index with bit 15 set and contributes exact zeros (c V_j taken as 0), so
// the per-node sum is the same, bit for bit, as the gather kernel's.
// ---------------------------------------------------------------------------
template <int DIM>
struct Rec {
    static constexpr int NC = 6;                  // doubles per record (48 bytes)
    static constexpr int U = DIM;                 // index of ux
};

constexpr int TILE_WPT = 8;          // 32-bit bond-word pairs staged per thread
constexpr int TILE_META = 5;         // h0, hn, b0 (even), b1, self offset
constexpr uint16_t BW_DEAD = 0x8000;

// record j as 16-byte LDS reads (the 48-byte stride keeps every record
// 16-byte aligned)
// Workgroup barrier that orders LDS only: global loads and stores in flight
// stay in flight (a plain __syncthreads would wait for all of them).  Global
// data is never passed between threads of one launch here.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int DIM>
__device__ __forceinline__ void read_rec(const double *rec, uint32_t j, double *A) {
    const double2 *q = reinterpret_cast<const double2 *>(rec + (size_t)j * Rec<DIM>::NC);
    const double2 a0 = q[0], a1 = q[1];
    A[0] = a0.x; A[1] = a0.y; A[2] = a1.x; A[3] = a1.y;
    if (DIM == 3) {
        const double2 a2 = q[2];
        A[4] = a2.x; A[5] = a2.y;
    }
}

template <int DIM, int L, bool MIXED, bool WANT_E, int RPT>
__global__ __launch_bounds__(1024) void tile_kernel(NodeArgs a) {
    if (a.done && *a.done) return;
    extern __shared__ __attribute__((aligned(16))) double lds[];
    constexpr int NC = Rec<DIM>::NC, IU = Rec<DIM>::U;
    constexpr int WPT = TILE_WPT;
    const uint32_t B = blockDim.x, tid = threadIdx.x;
    const uint32_t H = a.hcap, T = a.tile;
    const bool cv_uniform = a.cv_uniform != 0.0;
    double *rec = lds;                                                   // H * NC
    double *cv = rec + (size_t)H * NC;                                   // H
    double *fres = cv + H;                                               // T * 4
    uint32_t *meta = reinterpret_cast<uint32_t *>(fres + (size_t)T * 4);  // mmax * TILE_META
    uint32_t *sflag = meta + (size_t)a.mmax * TILE_META;                  // 4: break flag
    uint32_t *srp = sflag + 4;                                            // T + 1
    uint32_t *sbw = srp + (T + 1);                                        // bond-word pairs
    const uint16_t *sbw16 = reinterpret_cast<const uint16_t *>(sbw);
    uint16_t *sbw16w = reinterpret_cast<uint16_t *>(sbw);
    const uint32_t *bw32 = reinterpret_cast<const uint32_t *>(a.bw);
    const bool tangent = a.mode == M_TANGENT;
    const bool wants_v = mode_reads_v(a.mode);

    const uint32_t nb = gridDim.x, x = blockIdx.x % 8, l = blockIdx.x / 8;
    const uint32_t gx = nb / 8 + (x < nb % 8 ? 1u : 0u);
    const uint32_t tq = a.ntiles / 8, tr = a.ntiles % 8;
    const uint32_t tbeg = x * tq + (x < tr ? x : tr), tcnt = tq + (x < tr ? 1u : 0u);
    const uint32_t K = l < tcnt ? (tcnt - l + gx - 1) / gx : 0u;
    if (K == 0) return;

    for (uint32_t k = tid; k < K; k += B) {
        const uint32_t t = tbeg + l + k * gx, t0 = t * T, tn = min(T, a.n - t0);
        const uint32_t h0 = a.halo_ptr[t];
        uint32_t *m = meta + (size_t)k * TILE_META;
        m[0] = h0;
        m[1] = a.halo_ptr[t + 1] - h0;
        m[2] = a.row_ptr[t0] & ~1u;
        m[3] = a.row_ptr[t0 + tn];
        m[4] = a.self_off[t];
    }
    __syncthreads();

    // pipeline registers
    int32_t pid[RPT], pid_next[RPT];
    double4 pxv[RPT];
    double pux[RPT], puy[RPT], puz[RPT];
    uint8_t pfix[RPT];
    uint32_t pw[WPT];
    uint32_t prp = 0;

    auto fetch_ids = [&](uint32_t k, int32_t *ids) {
        const uint32_t h0 = meta[k * TILE_META], hn = meta[k * TILE_META + 1];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const uint32_t q = tid + r * B;
            ids[r] = q < hn ? a.halo[h0 + q] : 0;
        }
    };
    // every load below is unconditional, from a clamped (valid) index: a load
    // under a branch makes the compiler copy its result at the branch merge,
    // which waits for the load and so defeats the prefetch
    auto fetch_tile = [&](uint32_t k) {
        const uint32_t t = tbeg + l + k * gx, t0 = t * T, tn = min(T, a.n - t0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const uint32_t id = (uint32_t)pid[r];      // 0 past the halo's end
            pxv[r] = reinterpret_cast<const double4 *>(a.xv)[id];
            load_vec<DIM>(a.u, id, pux[r], puy[r], puz[r]);
            pfix[r] = (tangent && a.bc) ? a.bc[id] : (uint8_t)0;
        }
        const uint32_t b0 = meta[k * TILE_META + 2], b1 = meta[k * TILE_META + 3];
        const uint32_t nw = (b1 - b0 + 1) / 2;
#pragma unroll
        for (int w = 0; w < WPT; ++w) {
            const uint32_t q = tid + w * B;
            pw[w] = bw32[b0 / 2 + (q < nw ? q : 0u)];
        }
        prp = a.row_ptr[t0 + min(tid, tn)];
    };

    fetch_ids(0, pid);
    fetch_tile(0);
    if (K > 1) fetch_ids(1, pid_next);

    for (uint32_t k = 0; k < K; ++k) {
        const uint32_t t = tbeg + l + k * gx, t0 = t * T, tn = min(T, a.n - t0);
        const uint32_t hn = meta[k * TILE_META + 1], b0 = meta[k * TILE_META + 2];
        const uint32_t b1 = meta[k * TILE_META + 3], so = meta[k * TILE_META + 4];
        const uint32_t nw = (b1 - b0 + 1) / 2;
        lds_barrier();                         // LDS free: tile k-1 is complete
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const uint32_t q = tid + r * B;
            if (q < hn) {
                double *rr = rec + (size_t)q * NC;
                const bool fz = pfix[r] != 0;
                rr[0] = pxv[r].x;
                rr[1] = pxv[r].y;
                if (DIM == 3) rr[2] = pxv[r].z;
                rr[IU] = fz ? 0.0 : pux[r];
                rr[IU + 1] = fz ? 0.0 : puy[r];
                if (DIM == 3) rr[IU + 2] = fz ? 0.0 : puz[r];
                if (!cv_uniform) cv[q] = a.c * (DIM == 3 ? pxv[r].w : pxv[r].z);
            }
        }
#pragma unroll
        for (int w = 0; w < WPT; ++w) {
            const uint32_t q = tid + w * B;
            if (q < nw) sbw[q] = pw[w];
        }
        if (tid <= tn) srp[tid] = prp - b0;
        if (tid == 0) sflag[0] = 0;
        lds_barrier();

        // boundary kind of the node this thread updates after the bond sums
        const int kind = (a.bc && tid < tn) ? a.bc[t0 + tid] : PD_BC_FREE;

        // prefetch: records of tile k+1 (ids already here), ids of tile k+2
        if (k + 1 < K) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) pid[r] = pid_next[r];
            fetch_tile(k + 1);
            if (k + 2 < K) fetch_ids(k + 2, pid_next);
        }

        // bond sums of tile k.  A bond that breaks gets its dead bit in the
        // LDS copy of the bond words; tiles with a break write their words
        // back afterwards (a store inside the bond loop would make every
        // node wait for the prefetch loads still in flight).
        const uint32_t groups = B / L, g = tid / L;
        const int lane = tid & (L - 1);
        // one copy of the loop per volume layout, so the uniform case keeps c V
        // in scalar registers
        auto bond_sums = [&](auto uniform_volume) {
            constexpr bool UV = decltype(uniform_volume)::value;
            for (uint32_t q = g; q < tn; q += groups) {
                const double *ri = rec + (size_t)(so + q) * NC;
                const double xix = ri[0], xiy = ri[1], xiz = DIM == 3 ? ri[2] : 0.0;
                const double uix = ri[IU], uiy = ri[IU + 1], uiz = DIM == 3 ? ri[IU + 2] : 0.0;
                Acc64 acc;
                const uint32_t rs = srp[q], re = srp[q + 1];
                uint32_t p = rs + lane;
                for (; p + L < re; p += 2 * L) {
                    const uint32_t w0 = sbw16[p], w1 = sbw16[p + L];
                    const uint32_t j0 = __builtin_amdgcn_ubfe(w0, 0, 15);
                    const uint32_t j1 = __builtin_amdgcn_ubfe(w1, 0, 15);
                    double A[NC], C[NC];
                    read_rec<DIM>(rec, j0, A);
                    read_rec<DIM>(rec, j1, C);
                    const double cv0 = UV ? a.cv_uniform : cv[j0];
                    const double cv1 = UV ? a.cv_uniform : cv[j1];
                    if (bond<DIM, MIXED, WANT_E>(a.damage, a.s_c, A[0] - xix, A[1] - xiy,
                                                 DIM == 3 ? A[2] - xiz : 0.0, A[IU] - uix,
                                                 A[IU + 1] - uiy, DIM == 3 ? A[IU + 2] - uiz : 0.0,
                                                 cv0, (w0 & BW_DEAD) != 0, acc)) {
                        sbw16w[p] = (uint16_t)(w0 | BW_DEAD);
                        sflag[0] = 1;
                    }
                    if (bond<DIM, MIXED, WANT_E>(a.damage, a.s_c, C[0] - xix, C[1] - xiy,
                                                 DIM == 3 ? C[2] - xiz : 0.0, C[IU] - uix,
                                                 C[IU + 1] - uiy, DIM == 3 ? C[IU + 2] - uiz : 0.0,
                                                 cv1, (w1 & BW_DEAD) != 0, acc)) {
                        sbw16w[p + L] = (uint16_t)(w1 | BW_DEAD);
                        sflag[0] = 1;
                    }
                }
                if (p < re) {
                    const uint32_t w0 = sbw16[p], j0 = __builtin_amdgcn_ubfe(w0, 0, 15);
                    double A[NC];
                    read_rec<DIM>(rec, j0, A);
                    const double cv0 = UV ? a.cv_uniform : cv[j0];
                    if (bond<DIM, MIXED, WANT_E>(a.damage, a.s_c, A[0] - xix, A[1] - xiy,
                                                 DIM == 3 ? A[2] - xiz : 0.0, A[IU] - uix,
                                                 A[IU + 1] - uiy, DIM == 3 ? A[IU + 2] - uiz : 0.0,
                                                 cv0, (w0 & BW_DEAD) != 0, acc)) {
                        sbw16w[p] = (uint16_t)(w0 | BW_DEAD);
                        sflag[0] = 1;
                    }
                }
                double fx, fy, fz, Ue;
                group_reduce<DIM, L, WANT_E>(acc, fx, fy, fz, Ue);
                if (lane == 0) {
                    double *fr = fres + (size_t)q * 4;
                    fr[0] = fx;
                    fr[1] = fy;
                    fr[2] = fz;
                    fr[3] = Ue;
                }
            }
        };
        if (cv_uniform) bond_sums(std::true_type{});
        else bond_sums(std::false_type{});
        lds_barrier();
        if (sflag[0]) {
            // exactly this tile's bonds [row_ptr[t0], row_ptr[t0 + tn]) go back
            const uint32_t rs = srp[0], re = srp[tn];
            for (uint32_t q = rs + tid; q < re; q += B) a.bw[b0 + q] = sbw16[q];
        }

        // node updates of tile k (T <= B: thread q updates node q)
        if (tid < tn) {
            const uint32_t q = tid, i = t0 + q;
            const double *ri = rec + (size_t)(so + q) * NC;
            const double *fr = fres + (size_t)q * 4;
            const bool fixed_i = tangent && a.bc && kind != 0;
            const double Vi = (a.mode == M_TANGENT || a.mode == M_ENERGY)
                                  ? a.xv[4 * (size_t)i + (DIM == 3 ? 3 : 2)]
                                  : 0.0;
            double vx = 0, vy = 0, vz = 0;
            if (wants_v) load_vec<DIM>(a.v, i, vx, vy, vz);
            node_update<DIM>(a, i, fr[0], fr[1], fr[2], fr[3], Vi, ri[IU], ri[IU + 1],
                             DIM == 3 ? ri[IU + 2] : 0.0, fixed_i, vx, vy, vz, kind);
        }
    }
}

__global__ void bw_compose_k(uint64_t nnz, const uint16_t *lcol, const uint8_t *alive,
                             uint16_t *bw) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz + PD_BW_PAD)
        bw[p] = p >= nnz ? BW_DEAD : (uint16_t)(lcol[p] | ((alive && !alive[p]) ? BW_DEAD : 0));
}

__global__ void bw_alive_k(uint64_t nnz, const uint16_t *bw, uint8_t *alive) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) alive[p] = (bw[p] & BW_DEAD) ? 0 : 1;
}

template <int DIM, int L, bool MIXED, bool WANT_E>
void *pick_rpt(int rpt) {
    return rpt == 1 ? (void *)tile_kernel<DIM, L, MIXED, WANT_E, 1>
                    : (void *)tile_kernel<DIM, L, MIXED, WANT_E, 2>;
}

template <int DIM, int L>
void *pick_kernel(bool mixed, bool e, int rpt) {
    if (mixed) return e ? pick_rpt<DIM, L, true, true>(rpt) : pick_rpt<DIM, L, true, false>(rpt);
    return e ? pick_rpt<DIM, L, false, true>(rpt) : pick_rpt<DIM, L, false, false>(rpt);
}

template <int DIM>
void *pick_lanes(int lanes, bool mixed, bool e, int rpt) {
    switch (lanes) {
    case 2: return pick_kernel<DIM, 2>(mixed, e, rpt);
    case 4: return pick_kernel<DIM, 4>(mixed, e, rpt);
    case 8: return pick_kernel<DIM, 8>(mixed, e, rpt);
    case 16: return pick_kernel<DIM, 16>(mixed, e, rpt);
    case 32: return pick_kernel<DIM, 32>(mixed, e, rpt);
    default: return nullptr;
    }
}

}  // namespace

size_t tile_lds_bytes(int dim, uint32_t hcap, uint32_t bcap, uint32_t tile, uint32_t mmax) {
    (void)dim;
    return (size_t)hcap * 7 * sizeof(double) + (size_t)tile * 4 * sizeof(double) +
           (size_t)(mmax * TILE_META + 4) * sizeof(uint32_t) +
           (size_t)(tile + 1) * sizeof(uint32_t) + (size_t)(bcap / 2 + 2) * sizeof(uint32_t);
}

// Launch geometry of the persistent tile kernel: threads per workgroup,
// records staged per thread (RPT), workgroups, and the per-workgroup tile
// bound mmax.  Returns false if the layout does not fit.
bool pd_tile_geometry(int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap, uint32_t bcap,
                      int block, int num_cu, int *rpt, unsigned *grid, uint32_t *mmax,
                      size_t *lds, int max_per_cu) {
    const size_t lds_max = 160 * 1024;
    if ((uint32_t)block < tile) return false;   // one thread per tile node in the updates
    *rpt = (hcap + (uint32_t)block - 1) / (uint32_t)block;
    if (*rpt < 1) *rpt = 1;
    if (*rpt > 2) return false;
    if (bcap / 2 + 2 > (uint32_t)(TILE_WPT * block)) return false;
    for (int per_cu = max_per_cu > 0 && max_per_cu < 2 ? max_per_cu : 2; per_cu >= 1; --per_cu) {
        unsigned g = (unsigned)(num_cu * per_cu);
        if (g > ntiles) g = ntiles;
        if (g < 1) g = 1;
        // largest tile count of one workgroup
        uint32_t m = 0;
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t gx = g / 8 + (x < g % 8 ? 1u : 0u);
            const uint32_t tc = ntiles / 8 + (x < ntiles % 8 ? 1u : 0u);
            if (gx == 0) {
                if (tc) m = 0xffffffffu;
                continue;
            }
            const uint32_t kk = (tc + gx - 1) / gx;
            if (kk > m) m = kk;
        }
        if (m == 0xffffffffu) continue;
        const size_t bytes = tile_lds_bytes(dim, hcap, bcap, tile, m);
        if (bytes * (size_t)per_cu <= lds_max || (per_cu == 1 && bytes <= lds_max)) {
            *grid = g;
            *mmax = m;
            *lds = bytes;
            return true;
        }
    }
    return false;
}

// the layout fits and every form of the kernel a simulation may launch on it
// (both precisions, with and without energies) can be resident at `block`
// threads: some forms need more registers than others
bool pd_tile_resident(int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap, uint32_t bcap,
                      int lanes, int block, int num_cu) {
    int rpt = 0;
    unsigned grid = 0;
    uint32_t mmax = 0;
    size_t lds = 0;
    if (!pd_tile_geometry(dim, ntiles, tile, hcap, bcap, block, num_cu, &rpt, &grid, &mmax, &lds,
                          0))
        return false;
    for (int mixed = 0; mixed < 2; ++mixed)
        for (int e = 0; e < 2; ++e) {
            void *k = dim == 3 ? pick_lanes<3>(lanes, mixed != 0, e != 0, rpt)
                               : pick_lanes<2>(lanes, mixed != 0, e != 0, rpt);
            if (!k) return false;
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k, block, lds) !=
                    hipSuccess ||
                occ < 1)
                return false;
        }
    return true;
}

int pd_launch_tile(pd_ctx ctx, int dim, const NodeArgs &a0, int lanes, bool mixed, int block) {
    NodeArgs a = a0;
    int rpt = 0;
    unsigned grid = 0;
    size_t lds = 0;
    if (!pd_tile_geometry(dim, a.ntiles, a.tile, a.hcap, a.bcap, block, ctx->num_cu, &rpt, &grid,
                          &a.mmax, &lds, 0))
        return pd_set_error(ctx, PD_ECAPACITY, "tile layout does not fit this launch");
    const bool e = mode_wants_energy(a);
    void *k = dim == 3 ? pick_lanes<3>(lanes, mixed, e, rpt) : pick_lanes<2>(lanes, mixed, e, rpt);
    if (!k) return pd_set_error(ctx, PD_EINVAL, "tile kernel needs 2..32 lanes, got %d", lanes);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // every workgroup of the persistent grid must be resident at once: cap the
    // workgroups per CU by what registers and LDS allow for this kernel
    int occ = 0;
    PD_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k, block, lds));
    if (occ < 1) return pd_set_error(ctx, PD_ECAPACITY, "tile kernel cannot be resident");
    if (grid > (unsigned)(ctx->num_cu * occ)) {
        int rpt2 = 0;
        if (!pd_tile_geometry(dim, a.ntiles, a.tile, a.hcap, a.bcap, block, ctx->num_cu, &rpt2,
                              &grid, &a.mmax, &lds, occ) ||
            rpt2 != rpt)
            return pd_set_error(ctx, PD_ECAPACITY, "tile layout does not fit this launch");
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    void *args[] = {&a};
    PD_HIP(ctx, hipLaunchKernel(k, dim3(grid), dim3(block), args, lds, ctx->stream));
    return PD_OK;
}

int pd_bw_compose(pd_ctx ctx, const pd_nbr nbr, const uint8_t *alive_sfc, uint16_t *bw) {
    bw_compose_k<<<pd_blocks(nbr->nnz + PD_BW_PAD), PD_BLOCK, 0, ctx->stream>>>(nbr->nnz, nbr->lcol,
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
    pd_free(nbr->s_bw);
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
    if (hipMemcpyAsync(&total, scan + ntiles, sizeof total, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile scan copy");
    // largest halo
    std::vector<uint32_t> hc(ntiles);
    if (hipMemcpyAsync(hc.data(), count, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return cleanup(), pd_set_error(ctx, PD_EDEVICE, "tile count copy");
    uint32_t hmax = 0;
    for (uint32_t c : hc) hmax = c > hmax ? c : hmax;
    if (hipMemcpyAsync(hc.data(), bonds, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
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
