// Neighbour lists B_delta(X_i) = {X_j : |X_j - X_i| <= delta, j != i} in the
// reference configuration (Section "Discretization of peridynamics
// equations"; built once, as the bond-based algorithm prescribes).
//
// Pipeline, all on the GPU:
//   1. bounding box + finiteness check (block partials, host finish)
//   2. bins of edge >= delta; a 64-bit key per node = Morton code of its bin
//      followed by the Morton code of its position inside the bin
//   3. counting sort by bin (histogram, scan, scatter), then each bin sorted
//      by (key, original id): a deterministic space-filling-curve order
//   4. per node: count candidates from the 3^d surrounding bins that pass the
//      distance predicate, scan to row offsets, fill, sort each row by the
//      neighbour's original id (segments sorted in LDS by a bitonic network)
// The predicate is evaluated with FP contraction disabled so that it rounds
// exactly like the plain definition d2 = (dx*dx + dy*dy) + dz*dz.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pd_internal.hpp"

namespace {

constexpr int FLAG_COINCIDENT = 1;

__device__ __forceinline__ uint64_t spread2(uint64_t x) {  // 32 bits -> even bits
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __forceinline__ uint64_t spread3(uint64_t x) {  // 21 bits -> every third bit
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton(int dim, uint64_t a, uint64_t b, uint64_t c) {
    if (dim == 2) return spread2(a) | (spread2(b) << 1);
    return spread3(a) | (spread3(b) << 1) | (spread3(c) << 2);
}

struct Grid {
    int dim;
    double lo[3];
    double edge;
    int64_t nc[3];
    int bits;       // Morton bits per axis of the bin index
    int fbits;      // Morton bits per axis inside a bin
};

__device__ __forceinline__ int64_t bin_of(const Grid &g, int k, double x) {
    int64_t q = (int64_t)floor((x - g.lo[k]) / g.edge);
    if (q < 0) q = 0;
    if (q >= g.nc[k]) q = g.nc[k] - 1;
    return q;
}

// squared distance with every product and sum separately rounded
__device__ __forceinline__ double dist2(int dim, double4 a, double4 b) {
#pragma clang fp contract(off)
    const double dx = b.x - a.x;
    const double dy = b.y - a.y;
    double d2 = dx * dx + dy * dy;
    if (dim == 3) {
        const double dz = b.z - a.z;
        d2 = d2 + dz * dz;
    }
    return d2;
}

__global__ void bbox_k(int dim, uint32_t n, const double *X, double *part, int *bad) {
    __shared__ double smin[3][PD_BLOCK], smax[3][PD_BLOCK];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nonfinite = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < dim; ++k) {
            const double x = X[i * dim + k];
            if (!isfinite(x)) nonfinite = 1;
            mn[k] = fmin(mn[k], x);
            mx[k] = fmax(mx[k], x);
        }
    for (int k = 0; k < 3; ++k) {
        smin[k][threadIdx.x] = mn[k];
        smax[k][threadIdx.x] = mx[k];
    }
    if (nonfinite) atomicOr(bad, 2);
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 3; ++k) {
                smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + off]);
                smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) {
            part[(2 * k) * gridDim.x + blockIdx.x] = smin[k][0];
            part[(2 * k + 1) * gridDim.x + blockIdx.x] = smax[k][0];
        }
}

__global__ void keys_k(Grid g, uint32_t n, const double *X, uint64_t *key, uint32_t *binm,
                       uint32_t *hist) {
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    int64_t cc[3] = {0, 0, 0};
    uint64_t fc[3] = {0, 0, 0};
    const double fq = (double)(1ull << g.fbits);
    for (int k = 0; k < g.dim; ++k) {
        const double x = X[(uint64_t)o * g.dim + k];
        cc[k] = bin_of(g, k, x);
        double t = ((x - g.lo[k]) / g.edge - (double)cc[k]) * fq;
        int64_t q = (int64_t)floor(t);
        if (q < 0) q = 0;
        if (q >= (int64_t)(1ull << g.fbits)) q = (int64_t)(1ull << g.fbits) - 1;
        fc[k] = (uint64_t)q;
    }
    const uint64_t cm = morton(g.dim, cc[0], cc[1], cc[2]);
    const uint64_t fm = morton(g.dim, fc[0], fc[1], fc[2]);
    key[o] = (cm << (g.dim * g.fbits)) | fm;
    binm[o] = (uint32_t)cm;
    atomicAdd(&hist[cm], 1u);
}

__global__ void bin_scatter_k(uint32_t n, const uint32_t *binm, const uint64_t *bstart,
                              uint32_t *cursor, int32_t *perm) {
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const uint32_t m = binm[o];
    const uint32_t pos = (uint32_t)bstart[m] + atomicAdd(&cursor[m], 1u);
    perm[pos] = (int32_t)o;
}

// Segments (a bin's nodes, a row's neighbours) are sorted one workgroup per
// segment: the segment is read into LDS, padded to the next power of two
// with elements above every real one, put in order by a bitonic sorting
// network and written back.  A segment longer than the LDS capacity is
// sorted by one thread (insertion sort) in a second kernel that skips every
// other segment.  The order is a total order on distinct elements (node ids
// are unique), so both kernels give the same result.
constexpr int SEG_BLOCK = 256;
constexpr uint32_t ROW_CAP = 4096;   // int32 ids: 16 KB of LDS
constexpr uint32_t BIN_CAP = 2048;   // (key, id) pairs: 24 KB of LDS
constexpr unsigned SEG_GRID = 16384; // workgroups; each strides over segments

__device__ __forceinline__ uint32_t pow2_ceil(uint32_t x) {
    return x <= 1u ? 1u : 1u << (32 - __builtin_clz(x - 1u));
}

// the bitonic network over P (a power of two) elements of LDS: stage k
// merges runs of length k, pass j compares elements j apart; a pair sits in
// ascending order when its lower index has bit k clear.  gt(i, l) says
// whether element i belongs after element l; swap(i, l) exchanges them.
template <class Gt, class Swap>
__device__ __forceinline__ void bitonic_lds(uint32_t P, Gt gt, Swap swap) {
    for (uint32_t k = 2; k <= P; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += SEG_BLOCK) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                if (gt(i, i + j) == ((i & k) == 0)) swap(i, i + j);
            }
            __syncthreads();
        }
}

// each bin's nodes by (key, original id)
__global__ __launch_bounds__(SEG_BLOCK) void bin_sort_lds_k(uint64_t nbins, const uint64_t *bstart,
                                                            const uint64_t *key, int32_t *perm) {
    __shared__ uint64_t sk[BIN_CAP];
    __shared__ int32_t si[BIN_CAP];
    for (uint64_t m = blockIdx.x; m < nbins; m += gridDim.x) {
        const uint64_t a = bstart[m], len = bstart[m + 1] - a;
        if (len < 2 || len > BIN_CAP) continue;     // the same for the whole workgroup
        const uint32_t P = pow2_ceil((uint32_t)len);
        for (uint32_t x = threadIdx.x; x < P; x += SEG_BLOCK) {
            int32_t id = INT32_MAX;
            uint64_t kk = UINT64_MAX;
            if (x < len) {
                id = perm[a + x];
                kk = key[id];
            }
            sk[x] = kk;
            si[x] = id;
        }
        __syncthreads();
        bitonic_lds(
            P,
            [&](uint32_t i, uint32_t l) {
                return sk[i] > sk[l] || (sk[i] == sk[l] && si[i] > si[l]);
            },
            [&](uint32_t i, uint32_t l) {
                const uint64_t tk = sk[i];
                const int32_t ti = si[i];
                sk[i] = sk[l];
                si[i] = si[l];
                sk[l] = tk;
                si[l] = ti;
            });
        for (uint32_t x = threadIdx.x; x < len; x += SEG_BLOCK) perm[a + x] = si[x];
        __syncthreads();                            // LDS is reused by the next bin
    }
}

// the bins too long for LDS: one thread per bin, insertion sort by (key, id)
__global__ void bin_sort_long_k(uint64_t nbins, const uint64_t *bstart, const uint64_t *key,
                                int32_t *perm) {
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nbins) return;
    const uint64_t a = bstart[m], e = bstart[m + 1];
    if (e - a <= BIN_CAP) return;
    for (uint64_t p = a + 1; p < e; ++p) {
        const int32_t id = perm[p];
        const uint64_t kk = key[id];
        uint64_t q = p;
        while (q > a) {
            const int32_t other = perm[q - 1];
            const uint64_t ko = key[other];
            if (ko < kk || (ko == kk && other < id)) break;
            perm[q] = other;
            --q;
        }
        perm[q] = id;
    }
}

__global__ void invert_k(uint32_t n, const int32_t *perm, int32_t *iperm, int dim, const double *X,
                         double4 *xs) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = perm[s];
    iperm[o] = (int32_t)s;
    xs[s] = dim == 3 ? make_double4(X[3 * o], X[3 * o + 1], X[3 * o + 2], 0.0)
                     : make_double4(X[2 * o], X[2 * o + 1], 0.0, 0.0);
}

// Candidate loop shared by the count and fill passes.
template <bool FILL>
__global__ void candidates_k(Grid g, double thr, uint32_t n, const double4 *xs,
                             const uint64_t *bstart, uint32_t *cnt, const uint32_t *row_ptr,
                             int32_t *col, int *flag) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 xi = xs[s];
    const double xc[3] = {xi.x, xi.y, xi.z};
    int64_t cc[3] = {0, 0, 0};
    for (int k = 0; k < g.dim; ++k) cc[k] = bin_of(g, k, xc[k]);
    uint32_t m = 0;
    const uint32_t base = FILL ? row_ptr[s] : 0;
    const int zr = g.dim == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t x = cc[0] + dx, y = cc[1] + dy, z = cc[2] + dz;
                if (x < 0 || y < 0 || z < 0 || x >= g.nc[0] || y >= g.nc[1] ||
                    (g.dim == 3 && z >= g.nc[2]))
                    continue;
                const uint64_t bm = morton(g.dim, (uint64_t)x, (uint64_t)y, (uint64_t)z);
                const uint64_t a = bstart[bm], e = bstart[bm + 1];
                for (uint64_t t = a; t < e; ++t) {
                    if (t == s) continue;
                    const double d2 = dist2(g.dim, xi, xs[t]);
                    if (d2 == 0.0) atomicOr(flag, FLAG_COINCIDENT);
                    if (d2 <= thr) {
                        if (FILL) col[base + m] = (int32_t)t;
                        ++m;
                    }
                }
            }
    if (!FILL) cnt[s] = m;
}

// each CSR row ascending (internal rows by curve position, exported rows by
// original id)
__global__ __launch_bounds__(SEG_BLOCK) void row_sort_lds_k(uint32_t n, const uint32_t *row_ptr,
                                                            int32_t *col) {
    __shared__ int32_t sc[ROW_CAP];
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const uint32_t a = row_ptr[r], len = row_ptr[r + 1] - a;
        if (len < 2 || len > ROW_CAP) continue;     // the same for the whole workgroup
        const uint32_t P = pow2_ceil(len);
        for (uint32_t x = threadIdx.x; x < P; x += SEG_BLOCK)
            sc[x] = x < len ? col[a + x] : INT32_MAX;
        __syncthreads();
        bitonic_lds(
            P, [&](uint32_t i, uint32_t l) { return sc[i] > sc[l]; },
            [&](uint32_t i, uint32_t l) {
                const int32_t t = sc[i];
                sc[i] = sc[l];
                sc[l] = t;
            });
        for (uint32_t x = threadIdx.x; x < len; x += SEG_BLOCK) col[a + x] = sc[x];
        __syncthreads();                            // LDS is reused by the next row
    }
}

// the rows too long for LDS: one thread per row, insertion sort
__global__ void row_sort_long_k(uint32_t n, const uint32_t *row_ptr, int32_t *col) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t a = row_ptr[s], e = row_ptr[s + 1];
    if (e - a <= ROW_CAP) return;
    for (uint32_t p = a + 1; p < e; ++p) {
        const int32_t c = col[p];
        uint32_t q = p;
        while (q > a && col[q - 1] > c) {
            col[q] = col[q - 1];
            --q;
        }
        col[q] = c;
    }
}

// both row sorts of the build
void sort_rows(hipStream_t st, uint32_t n, const uint32_t *row_ptr, int32_t *col) {
    row_sort_lds_k<<<std::min<unsigned>(n, SEG_GRID), SEG_BLOCK, 0, st>>>(n, row_ptr, col);
    row_sort_long_k<<<pd_blocks(n), PD_BLOCK, 0, st>>>(n, row_ptr, col);
}

// exported rows (original numbering) filled unsorted, one wave per row, then
// sorted by original id
__global__ void excol_fill_k(uint32_t n, const int32_t *perm, const uint32_t *row_ptr,
                             const uint32_t *ex_row_ptr, const int32_t *col, int32_t *ex_col) {
    const uint32_t s = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const uint32_t lane = threadIdx.x % 64;
    if (s >= n) return;
    const uint32_t a = row_ptr[s], e = row_ptr[s + 1], x = ex_row_ptr[perm[s]];
    for (uint32_t k = lane; k < e - a; k += 64) ex_col[x + k] = perm[col[a + k]];
}

// exported position of every internal bond: binary search of the
// neighbour's original id in its exported row (one wave per row)
__global__ void ex_pos_k(uint32_t n, const int32_t *perm, const uint32_t *row_ptr,
                         const uint32_t *ex_row_ptr, const int32_t *col, const int32_t *ex_col,
                         uint32_t *ex_pos) {
    const uint32_t s = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const uint32_t lane = threadIdx.x % 64;
    if (s >= n) return;
    const uint32_t a = row_ptr[s], e = row_ptr[s + 1];
    const uint32_t xa = ex_row_ptr[perm[s]], xe = ex_row_ptr[perm[s] + 1];
    for (uint32_t p = a + lane; p < e; p += 64) {
        const int32_t key = perm[col[p]];
        uint32_t lo = xa, hi = xe;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ex_col[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        ex_pos[p] = lo;
    }
}

__global__ void orig_counts_k(uint32_t n, const int32_t *perm, const uint32_t *cnt,
                              uint32_t *cnt_orig, int32_t *max_row) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    cnt_orig[perm[s]] = cnt[s];
    atomicMax(max_row, (int32_t)cnt[s]);
}

__global__ void export_cols_k(uint64_t nnz, const int32_t *perm, const int32_t *col,
                              const uint32_t *ex_pos, int32_t *out) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) out[ex_pos[p]] = perm[col[p]];
}

}  // namespace

static void nbr_release(pd_nbr b) {
    if (!b) return;
    pd_free(b->perm);
    pd_free(b->iperm);
    pd_free(b->row_ptr);
    pd_free(b->col);
    pd_free(b->ex_row_ptr);
    pd_free(b->ex_pos);
    pd_free(b->halo_ptr);
    pd_free(b->halo);
    pd_free(b->self_off);
    pd_free(b->lcol);
    pd_free(b->s_xv);
    pd_free(b->s_u);
    pd_free(b->s_f);
    pd_free(b->s_U);
    pd_free(b->s_ulin);
    pd_free(b->s_lps);
    pd_free(b->s_alive);
    pd_free(b->s_fixed);
    pd_ctx ctx = b->ctx;
    delete b;
    pd_ctx_unref(ctx);
}

namespace {
// RAII holder for the build's temporaries
struct Tmp {
    uint64_t *key = nullptr, *bstart = nullptr, *scan = nullptr;
    uint32_t *binm = nullptr, *hist = nullptr, *cursor = nullptr, *cnt = nullptr,
             *cnt_orig = nullptr;
    double4 *xs = nullptr;
    double *part = nullptr;
    int32_t *maxrow = nullptr;
    int32_t *ex_col = nullptr;
    ~Tmp() {
        pd_free(ex_col);
        pd_free(key); pd_free(bstart); pd_free(scan); pd_free(binm); pd_free(hist);
        pd_free(cursor); pd_free(cnt); pd_free(cnt_orig); pd_free(xs); pd_free(part);
        pd_free(maxrow);
    }
};

int build(pd_ctx ctx, int dim, uint32_t n, const double *X, double delta, pd_nbr b) {
    hipStream_t st = ctx->stream;
    Tmp t;
    b->thr = (delta * delta) * (1.0 + 1e-10);

    // 1. bounding box
    const unsigned bb_blocks = std::min<unsigned>(pd_blocks(n), 1024);
    PD_TRY(pd_alloc(ctx, &t.part, 6 * (size_t)bb_blocks));
    PD_TRY(pd_flag_clear(ctx));
    bbox_k<<<bb_blocks, PD_BLOCK, 0, st>>>(dim, n, X, t.part, ctx->flag);
    PD_LAUNCH_CHECK(ctx);
    std::vector<double> part(6 * (size_t)bb_blocks);
    PD_HIP(ctx, hipMemcpyAsync(part.data(), t.part, sizeof(double) * part.size(),
                               hipMemcpyDeviceToHost, st));
    int flag = 0;
    PD_TRY(pd_flag_read(ctx, &flag));
    if (flag & 2) return pd_set_error(ctx, PD_EINVAL, "X contains non-finite coordinates");
    Grid g{};
    g.dim = dim;
    double hi[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        for (unsigned q = 0; q < bb_blocks; ++q) {
            mn = std::min(mn, part[(2 * k) * bb_blocks + q]);
            mx = std::max(mx, part[(2 * k + 1) * bb_blocks + q]);
        }
        g.lo[k] = k < dim ? mn : 0.0;
        hi[k] = k < dim ? mx : 0.0;
    }

    // 2. bins
    g.edge = std::sqrt(b->thr) * (1.0 + 1e-12);
    int64_t ncmax = 1;
    for (int k = 0; k < 3; ++k) {
        g.nc[k] = k < dim ? (int64_t)std::floor((hi[k] - g.lo[k]) / g.edge) + 1 : 1;
        if (g.nc[k] > (int64_t)1 << 20)
            return pd_set_error(ctx, PD_ECAPACITY, "bounding box spans more than 2^20 bins");
        ncmax = std::max(ncmax, g.nc[k]);
    }
    g.bits = 0;
    while (((int64_t)1 << g.bits) < ncmax) ++g.bits;
    if (dim * g.bits > 27)
        return pd_set_error(ctx, PD_ECAPACITY, "bounding box needs more than 2^27 bins");
    g.fbits = (dim == 3 ? 21 : 31) - g.bits;
    if (g.fbits > 10) g.fbits = 10;
    const uint64_t nbins = 1ull << (dim * g.bits);

    PD_TRY(pd_alloc(ctx, &t.key, n));
    PD_TRY(pd_alloc(ctx, &t.binm, n));
    PD_TRY(pd_alloc(ctx, &t.hist, nbins));
    PD_TRY(pd_alloc(ctx, &t.cursor, nbins));
    PD_TRY(pd_alloc(ctx, &t.bstart, nbins + 1));
    PD_HIP(ctx, hipMemsetAsync(t.hist, 0, sizeof(uint32_t) * nbins, st));
    PD_HIP(ctx, hipMemsetAsync(t.cursor, 0, sizeof(uint32_t) * nbins, st));
    keys_k<<<pd_blocks(n), PD_BLOCK, 0, st>>>(g, n, X, t.key, t.binm, t.hist);
    PD_LAUNCH_CHECK(ctx);
    if (nbins > 0xffffffffull) return pd_set_error(ctx, PD_ECAPACITY, "too many bins");
    PD_TRY(pd_scan_u32(ctx, t.hist, t.bstart, (uint32_t)nbins));

    // 3. counting sort by bin, then (key, id) inside each bin
    PD_TRY(pd_alloc(ctx, &b->perm, n));
    PD_TRY(pd_alloc(ctx, &b->iperm, n));
    bin_scatter_k<<<pd_blocks(n), PD_BLOCK, 0, st>>>(n, t.binm, t.bstart, t.cursor, b->perm);
    PD_LAUNCH_CHECK(ctx);
    bin_sort_lds_k<<<(unsigned)std::min<uint64_t>(nbins, SEG_GRID), SEG_BLOCK, 0, st>>>(
        nbins, t.bstart, t.key, b->perm);
    bin_sort_long_k<<<pd_blocks(nbins), PD_BLOCK, 0, st>>>(nbins, t.bstart, t.key, b->perm);
    PD_LAUNCH_CHECK(ctx);
    PD_TRY(pd_alloc(ctx, &t.xs, n));
    invert_k<<<pd_blocks(n), PD_BLOCK, 0, st>>>(n, b->perm, b->iperm, dim, X, t.xs);
    PD_LAUNCH_CHECK(ctx);

    // 4. count, scan, fill, sort rows
    PD_TRY(pd_alloc(ctx, &t.cnt, n));
    PD_TRY(pd_flag_clear(ctx));
    candidates_k<false><<<pd_blocks(n), PD_BLOCK, 0, st>>>(g, b->thr, n, t.xs, t.bstart, t.cnt,
                                                          nullptr, nullptr, ctx->flag);
    PD_LAUNCH_CHECK(ctx);
    PD_TRY(pd_alloc(ctx, &t.scan, (size_t)n + 1));
    PD_TRY(pd_scan_u32(ctx, t.cnt, t.scan, n));
    PD_TRY(pd_flag_read(ctx, &flag));
    if (flag & FLAG_COINCIDENT) return pd_set_error(ctx, PD_EINVAL, "two nodes coincide");
    uint64_t nnz = 0;
    PD_HIP(ctx, hipMemcpyAsync(&nnz, t.scan + n, sizeof(uint64_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nnz > 0xffffffffull)
        return pd_set_error(ctx, PD_ECAPACITY, "%llu bonds exceed the 2^32-1 limit",
                            (unsigned long long)nnz);
    b->nnz = nnz;
    PD_TRY(pd_alloc(ctx, &b->row_ptr, (size_t)n + 1));
    PD_TRY(pd_narrow_u64(ctx, t.scan, b->row_ptr, n));
    PD_TRY(pd_alloc(ctx, &b->col, nnz));
    candidates_k<true><<<pd_blocks(n), PD_BLOCK, 0, st>>>(g, b->thr, n, t.xs, t.bstart, nullptr,
                                                         b->row_ptr, b->col, ctx->flag);
    PD_LAUNCH_CHECK(ctx);
    sort_rows(st, n, b->row_ptr, b->col);
    PD_LAUNCH_CHECK(ctx);

    // exported (original-order) row offsets and the longest row
    PD_TRY(pd_alloc(ctx, &t.cnt_orig, n));
    PD_TRY(pd_alloc(ctx, &t.maxrow, 1));
    PD_HIP(ctx, hipMemsetAsync(t.maxrow, 0, sizeof(int32_t), st));
    orig_counts_k<<<pd_blocks(n), PD_BLOCK, 0, st>>>(n, b->perm, t.cnt, t.cnt_orig, t.maxrow);
    PD_LAUNCH_CHECK(ctx);
    PD_TRY(pd_scan_u32(ctx, t.cnt_orig, t.scan, n));
    PD_TRY(pd_alloc(ctx, &b->ex_row_ptr, (size_t)n + 1));
    PD_TRY(pd_narrow_u64(ctx, t.scan, b->ex_row_ptr, n));
    // exported position of each internal bond (rows in original numbering,
    // neighbours ascending by original id)
    PD_TRY(pd_alloc(ctx, &t.ex_col, nnz));
    PD_TRY(pd_alloc(ctx, &b->ex_pos, nnz));
    excol_fill_k<<<pd_blocks((uint64_t)n * 64), PD_BLOCK, 0, st>>>(n, b->perm, b->row_ptr,
                                                                    b->ex_row_ptr, b->col, t.ex_col);
    PD_LAUNCH_CHECK(ctx);
    sort_rows(st, n, b->ex_row_ptr, t.ex_col);
    PD_LAUNCH_CHECK(ctx);
    ex_pos_k<<<pd_blocks((uint64_t)n * 64), PD_BLOCK, 0, st>>>(n, b->perm, b->row_ptr,
                                                                b->ex_row_ptr, b->col, t.ex_col,
                                                                b->ex_pos);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(&b->max_row, t.maxrow, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PD_HIP(ctx, hipStreamSynchronize(st));
    return PD_OK;
}
}  // namespace

extern "C" int pd_build_neighbors(pd_ctx ctx, int dim, int64_t n, const double *X, double delta,
                                  pd_nbr *out) {
    if (!out) return pd_set_error(ctx, PD_EINVAL, "out must not be NULL");
    *out = nullptr;
    PD_TRY(pd_check_ctx(ctx));
    if (dim != 2 && dim != 3) return pd_set_error(ctx, PD_EINVAL, "dim must be 2 or 3");
    if (n <= 0) return pd_set_error(ctx, PD_EINVAL, "n must be positive");
    if (n >= ((int64_t)1 << 31)) return pd_set_error(ctx, PD_ECAPACITY, "n must be below 2^31");
    if (!(delta > 0.0) || !std::isfinite(delta))
        return pd_set_error(ctx, PD_EINVAL, "delta must be finite and positive");
    PD_TRY(pd_check_dev_ptr(ctx, X, "X"));
    pd_nbr b = new (std::nothrow) pd_nbr_s();
    if (!b) return PD_ENOMEM;
    b->ctx = ctx;
    ctx->refs += 1;
    b->dim = dim;
    b->n = (uint32_t)n;
    b->delta = delta;
    int st = build(ctx, dim, (uint32_t)n, X, delta, b);
    if (st != PD_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        nbr_release(b);
        return st;
    }
    *out = b;
    return PD_OK;
}

extern "C" int pd_nbr_info(pd_nbr nbr, int64_t *nnz, int32_t *max_row) {
    if (!nbr) return PD_EINVAL;
    if (nnz) *nnz = (int64_t)nbr->nnz;
    if (max_row) *max_row = nbr->max_row;
    return PD_OK;
}

extern "C" int pd_nbr_export(pd_nbr nbr, int64_t *row_ptr, int32_t *col) {
    if (!nbr || nbr->closing) return PD_EINVAL;
    pd_ctx ctx = nbr->ctx;
    PD_TRY(pd_check_ctx(ctx));
    const uint32_t n = nbr->n;
    if (row_ptr) {
        std::vector<uint32_t> tmp((size_t)n + 1);
        PD_HIP(ctx, hipMemcpyAsync(tmp.data(), nbr->ex_row_ptr, sizeof(uint32_t) * (n + 1),
                                   hipMemcpyDeviceToHost, ctx->stream));
        PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (size_t k = 0; k <= n; ++k) row_ptr[k] = tmp[k];
    }
    if (col && nbr->nnz) {
        int32_t *d = nullptr;
        PD_TRY(pd_alloc(ctx, &d, nbr->nnz));
        export_cols_k<<<pd_blocks(nbr->nnz), PD_BLOCK, 0, ctx->stream>>>(
            nbr->nnz, nbr->perm, nbr->col, nbr->ex_pos, d);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(col, d, sizeof(int32_t) * nbr->nnz, hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        pd_free(d);
        if (e != hipSuccess) return pd_hip_error(ctx, e, "export", __FILE__, __LINE__);
    }
    return PD_OK;
}

extern "C" int pd_nbr_permutation(pd_nbr nbr, int32_t *perm) {
    if (!nbr || nbr->closing || !perm) return PD_EINVAL;
    pd_ctx ctx = nbr->ctx;
    PD_TRY(pd_check_ctx(ctx));
    PD_HIP(ctx, hipMemcpyAsync(perm, nbr->perm, sizeof(int32_t) * nbr->n, hipMemcpyDeviceToHost,
                               ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

void pd_nbr_unref(pd_nbr nbr) {
    if (!nbr) return;
    nbr->refs -= 1;
    if (nbr->closing && nbr->refs <= 0) nbr_release(nbr);
}

extern "C" int pd_nbr_destroy(pd_nbr nbr) {
    if (!nbr || nbr->closing) return PD_EINVAL;
    (void)hipSetDevice(nbr->ctx->device);
    (void)hipStreamSynchronize(nbr->ctx->stream);
    if (nbr->refs > 0) {
        nbr->closing = true;
        return PD_OK;
    }
    nbr_release(nbr);
    return PD_OK;
}
