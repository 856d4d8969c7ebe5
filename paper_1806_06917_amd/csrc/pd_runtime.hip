// Context, error reporting and the small data-movement kernels shared by the
// entry points: scans, sfc <-> original order permutations, bond-flag
// reordering and deterministic reductions.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>

#include "pd_internal.hpp"

// ---------------------------------------------------------------------------
// device memory cache
// ---------------------------------------------------------------------------
// hipMalloc and hipFree cost tens of microseconds each and hipFree waits for
// the whole device, while a serving loop builds and drops simulations (a
// dozen buffers each) all the time.  So a freed block is kept per device and
// handed out again.  A block is freed on the stream of the context that
// allocated it: an event recorded there at the free marks the end of its
// last use, and the block is handed out again only after that event has
// completed (blocks still in use are passed over), so no later work on any
// stream can overlap an earlier user.  Sizes round up to 256 bytes (64 KiB
// from 1 MiB on); a request takes the smallest cached block of at least its
// size and at most an eighth more.  At most PD_CACHE_MAX bytes stay cached;
// when hipMalloc fails the device's cache is released and the call retried.
namespace {

constexpr size_t PD_CACHE_MAX = size_t(16) << 30;

struct CachedBlock {
    void *p;
    hipEvent_t done;   // recorded at the free on the owner's stream
};
struct LiveBlock {
    size_t bytes;
    int device;
    hipStream_t stream;
};
struct DeviceCache {
    std::multimap<size_t, CachedBlock> free;
    size_t bytes = 0;
    std::vector<hipEvent_t> events;   // idle events for reuse
};

// never destroyed: frees may still arrive while the process exits
std::mutex &g_mem_mu = *new std::mutex;
std::unordered_map<void *, LiveBlock> &g_live = *new std::unordered_map<void *, LiveBlock>;
std::map<int, DeviceCache> &g_cache = *new std::map<int, DeviceCache>;

size_t round_bytes(size_t b) {
    const size_t q = b < (size_t(1) << 20) ? 256 : (size_t(64) << 10);
    return (b + q - 1) / q * q;
}

// every cached block of a device back to the driver (device current)
void release_cache(DeviceCache &c) {
    for (auto &kv : c.free) {
        (void)hipEventSynchronize(kv.second.done);
        (void)hipEventDestroy(kv.second.done);
        (void)hipFree(kv.second.p);
    }
    c.free.clear();
    c.bytes = 0;
}

}  // namespace

int pd_alloc_bytes(pd_ctx ctx, void **p, size_t bytes) {
    *p = nullptr;
    bytes = round_bytes(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_mem_mu);
    DeviceCache &c = g_cache[dev];
    // the smallest fitting block whose last use has completed (a block still
    // in use on its stream is passed over rather than waited for)
    for (auto it = c.free.lower_bound(bytes);
         it != c.free.end() && it->first <= bytes + bytes / 8; ++it) {
        if (hipEventQuery(it->second.done) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        CachedBlock b = it->second;
        const size_t have = it->first;
        c.free.erase(it);
        c.bytes -= have;
        c.events.push_back(b.done);
        *p = b.p;
        g_live[b.p] = LiveBlock{have, dev, ctx ? ctx->stream : nullptr};
        return PD_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess && !c.free.empty()) {
        (void)hipGetLastError();
        release_cache(c);
        e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return pd_set_error(ctx, PD_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes,
                            hipGetErrorString(e));
    }
    g_live[*p] = LiveBlock{bytes, dev, ctx ? ctx->stream : nullptr};
    return PD_OK;
}

void pd_mem_restream(hipStream_t from, hipStream_t to, const void *keep1, const void *keep2) {
    std::lock_guard<std::mutex> lock(g_mem_mu);
    for (auto &kv : g_live)
        if (kv.second.stream == from && kv.first != keep1 && kv.first != keep2)
            kv.second.stream = to;
}

void pd_free_bytes(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {
        (void)hipFree(p);
        return;
    }
    const LiveBlock lb = it->second;
    g_live.erase(it);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != lb.device) (void)hipSetDevice(lb.device);
    DeviceCache &c = g_cache[lb.device];
    hipEvent_t ev = nullptr;
    if (!c.events.empty()) {
        ev = c.events.back();
        c.events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    if (ev && hipEventRecord(ev, lb.stream) == hipSuccess) {
        c.free.emplace(lb.bytes, CachedBlock{p, ev});
        c.bytes += lb.bytes;
        // over the cap: the largest cached blocks go back to the driver
        while (c.bytes > PD_CACHE_MAX && !c.free.empty()) {
            auto last = std::prev(c.free.end());
            (void)hipEventSynchronize(last->second.done);
            c.events.push_back(last->second.done);
            (void)hipFree(last->second.p);
            c.bytes -= last->first;
            c.free.erase(last);
        }
    } else {
        // no event (or the owner's stream is gone): give it back at once
        (void)hipGetLastError();
        if (ev) c.events.push_back(ev);
        (void)hipFree(p);
    }
    if (cur != lb.device) (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int pd_set_error(pd_ctx ctx, int status, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
        if (status == PD_EDEVICE) ctx->failed = 1;
    }
    return status;
}

int pd_hip_error(pd_ctx ctx, hipError_t e, const char *what, const char *file, int line) {
    (void)hipGetLastError();
    return pd_set_error(ctx, PD_EDEVICE, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file,
                        line);
}

int pd_check_ctx(pd_ctx ctx) {
    if (!ctx) return PD_EINVAL;
    if (ctx->closing) return pd_set_error(ctx, PD_EINVAL, "the context has been destroyed");
    if (ctx->failed) return PD_EDEVICE;
    PD_HIP(ctx, hipSetDevice(ctx->device));
    return PD_OK;
}

int pd_check_dev_ptr(pd_ctx ctx, const void *p, const char *name) {
    if (!p) return pd_set_error(ctx, PD_EINVAL, "%s must not be NULL", name);
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return pd_set_error(ctx, PD_EINVAL, "%s is not device memory", name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return pd_set_error(ctx, PD_EINVAL, "%s is not device memory", name);
    if (attr.device != ctx->device)
        return pd_set_error(ctx, PD_EINVAL, "%s lives on device %d, context on %d", name,
                            attr.device, ctx->device);
    return PD_OK;
}

int pd_auto_lanes(pd_ctx ctx, uint64_t nnz, uint32_t n) {
    if (ctx && ctx->lanes > 0) return ctx->lanes;
    // about 16 bonds per lane: enough work per lane to amortise the lane
    // reduction; with the automatic 128-node tiles that gives 1024-thread
    // (3-d, delta = 3h) or 512-thread (2-d, delta = 4h) workgroups
    const double k = n ? (double)nnz / (double)n : 0.0;
    int L = 1;
    while (L < 32 && L * 16 < k) L *= 2;
    return L;
}

// ---------------------------------------------------------------------------
// public: version, status strings, micromodulus, context
// ---------------------------------------------------------------------------
extern "C" int pd_version(void) { return PD_VERSION_NUMBER; }

extern "C" const char *pd_status_string(int s) {
    switch (s) {
    case PD_OK: return "ok";
    case PD_EINVAL: return "invalid argument";
    case PD_ENOMEM: return "out of device memory";
    case PD_EDEVICE: return "device error";
    case PD_ENOCONV: return "no convergence";
    case PD_ENONFINITE: return "non-finite state";
    case PD_ECAPACITY: return "size limit exceeded";
    default: return "unknown status";
    }
}

extern "C" double pd_micromodulus(int dim, double E, double delta) {
    const double pi = 3.14159265358979323846;
    if (dim == 2) return 9.0 * E / (pi * delta * delta * delta);
    if (dim == 3) return 12.0 * E / (pi * delta * delta * delta * delta);
    return NAN;
}

extern "C" int pd_ctx_create(int device, void *hip_stream, pd_ctx *out) {
    if (!out) return PD_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return PD_EDEVICE;
    }
    if (device < 0 || device >= count) return PD_EINVAL;
    pd_ctx c = new (std::nothrow) pd_ctx_s();
    if (!c) return PD_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return PD_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        c->num_cu = ncu;
    (void)hipGetLastError();
    int st = pd_alloc(c, &c->red, (size_t)PD_RED_BLOCKS * PD_RED_SLOTS);
    if (st == PD_OK) st = pd_alloc(c, &c->flag, 1);
    if (st == PD_OK &&
        hipHostMalloc((void **)&c->red_host, sizeof(double) * PD_RED_BLOCKS * PD_RED_SLOTS) !=
            hipSuccess)
        st = PD_ENOMEM;
    if (st == PD_OK && hipHostMalloc((void **)&c->flag_host, sizeof(int)) != hipSuccess)
        st = PD_ENOMEM;
    if (st == PD_OK) st = pd_noalloc_setup(c);   // with the device current
    if (st != PD_OK) {
        (void)hipGetLastError();
        pd_ctx_destroy(c);
        return st;
    }
    *out = c;
    return PD_OK;
}

static void ctx_free(pd_ctx ctx) {
    pd_free(ctx->red);
    pd_free(ctx->flag);
    if (ctx->red_host) (void)hipHostFree(ctx->red_host);
    if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
    delete ctx;
}

void pd_ctx_unref(pd_ctx ctx) {
    if (!ctx) return;
    ctx->refs -= 1;
    if (ctx->closing && ctx->refs <= 0) ctx_free(ctx);
}

extern "C" int pd_ctx_destroy(pd_ctx ctx) {
    if (!ctx || ctx->closing) return PD_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->refs > 0) {
        ctx->closing = true;
        return PD_OK;
    }
    ctx_free(ctx);
    return PD_OK;
}

extern "C" const char *pd_last_error(pd_ctx ctx) {
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

int pd_check_law(pd_ctx ctx, const pd_material *m) {
    if (!(m->pv_h >= 0.0) || !std::isfinite(m->pv_h))
        return pd_set_error(ctx, PD_EINVAL, "pv_h must be finite and >= 0");
    if (!(m->j_c2 >= 0.0) || !std::isfinite(m->j_c2) || !std::isfinite(m->j_c1))
        return pd_set_error(ctx, PD_EINVAL, "j_c1 must be finite and j_c2 finite and >= 0");
    if (m->law != PD_LAW_LINEAR && m->law != PD_LAW_NP && m->law != PD_LAW_LPS)
        return pd_set_error(ctx, PD_EINVAL, "law must be PD_LAW_LINEAR, PD_LAW_NP or PD_LAW_LPS");
    if (m->law == PD_LAW_LPS) {
        if (m->dim != 3) return pd_set_error(ctx, PD_EINVAL, "PD_LAW_LPS is the 3-d solid");
        if (!(m->bulk > 0.0) || !std::isfinite(m->bulk) || !(m->shear >= 0.0) ||
            !std::isfinite(m->shear))
            return pd_set_error(ctx, PD_EINVAL, "PD_LAW_LPS needs bulk > 0 and shear >= 0");
        if (m->s_c > 0.0) return pd_set_error(ctx, PD_EINVAL, "PD_LAW_LPS takes no damage");
        if (m->j_c2 > 0.0)
            return pd_set_error(ctx, PD_EINVAL, "PD_LAW_LPS takes no influence function");
        return PD_OK;
    }
    if (m->stretch != PD_STRETCH_LINEARISED && m->stretch != PD_STRETCH_EXACT)
        return pd_set_error(ctx, PD_EINVAL,
                            "stretch must be PD_STRETCH_LINEARISED or PD_STRETCH_EXACT");
    if (m->law == PD_LAW_NP && (!(m->beta > 0.0) || !std::isfinite(m->beta)))
        return pd_set_error(ctx, PD_EINVAL, "PD_LAW_NP needs a finite beta > 0");
    return PD_OK;
}

extern "C" int pd_ctx_set_lanes(pd_ctx ctx, int lanes) {
    if (!ctx) return PD_EINVAL;
    if (lanes != 0 && (lanes < 1 || lanes > 64 || (lanes & (lanes - 1))))
        return pd_set_error(ctx, PD_EINVAL, "lanes must be 0 or a power of two in [1, 64]");
    ctx->lanes = lanes;
    return PD_OK;
}

extern "C" int pd_ctx_set_tuning(pd_ctx ctx, int kernel, int tile, int block) {
    if (!ctx) return PD_EINVAL;
    if (kernel < 0 || kernel > 3)
        return pd_set_error(ctx, PD_EINVAL, "kernel must be 0, 1, 2 or 3");
    if (tile != 0 && (tile < 16 || tile > 4096 || (tile % 16)))
        return pd_set_error(ctx, PD_EINVAL, "tile must be 0 or a multiple of 16 in [16, 4096]");
    if (block != 0 && (block < 64 || block > 1024 || (block % 64)))
        return pd_set_error(ctx, PD_EINVAL, "block must be 0 or a multiple of 64 in [64, 1024]");
    ctx->kernel = kernel;
    ctx->tile = tile;
    ctx->block = block;
    return PD_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan (three passes, 1024 items per block)
// ---------------------------------------------------------------------------
namespace {
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = PD_BLOCK * SCAN_ITEMS;

__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t *total) {
    __shared__ uint64_t s[PD_BLOCK];
    const int t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (int off = 1; off < PD_BLOCK; off <<= 1) {
        uint64_t y = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const uint64_t incl = s[t];
    *total = s[PD_BLOCK - 1];
    __syncthreads();
    return incl - x;
}

__global__ void scan_tile_sums(const uint32_t *in, uint32_t n, uint64_t *sums) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t acc = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) acc += in[base + k];
    uint64_t total;
    block_exclusive_scan(acc, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void scan_sums_serial(uint64_t *sums, uint32_t count) {
    // single block: running exclusive scan over `count` tile sums
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < count; base += PD_BLOCK) {
        const uint32_t k = base + threadIdx.x;
        uint64_t x = k < count ? sums[k] : 0;
        uint64_t total;
        uint64_t ex = block_exclusive_scan(x, &total);
        if (k < count) sums[k] = ex + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
}

__global__ void scan_apply(const uint32_t *in, uint32_t n, const uint64_t *sums, uint64_t *out) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t v[SCAN_ITEMS];
    uint64_t acc = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        acc += v[k];
    }
    uint64_t total;
    uint64_t ex = block_exclusive_scan(acc, &total) + sums[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == PD_BLOCK - 1) out[n] = ex;
}

__global__ void narrow_u64(const uint64_t *in, uint32_t *out, uint32_t n) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= n) out[k] = (uint32_t)in[k];
}
}  // namespace

int pd_scan_u32(pd_ctx ctx, const uint32_t *in, uint64_t *out, uint32_t n) {
    const uint32_t tiles = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE) + (n == 0);
    uint64_t *sums = nullptr;
    PD_TRY(pd_alloc(ctx, &sums, tiles));
    scan_tile_sums<<<tiles, PD_BLOCK, 0, ctx->stream>>>(in, n, sums);
    scan_sums_serial<<<1, PD_BLOCK, 0, ctx->stream>>>(sums, tiles);
    scan_apply<<<tiles, PD_BLOCK, 0, ctx->stream>>>(in, n, sums, out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    pd_free(sums);
    if (e != hipSuccess) return pd_hip_error(ctx, e, "scan", __FILE__, __LINE__);
    return PD_OK;
}

int pd_narrow_u64(pd_ctx ctx, const uint64_t *in, uint32_t *out, uint32_t n) {
    narrow_u64<<<pd_blocks((uint64_t)n + 1), PD_BLOCK, 0, ctx->stream>>>(in, out, n);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

// ---------------------------------------------------------------------------
// permutations between the caller's order and the internal sfc order
// ---------------------------------------------------------------------------
namespace {
__global__ void gather_xv_k(const int32_t *perm, uint32_t n, int dim, const double *X,
                            const double *V, double *xv) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = perm[s];
    double4 r;
    if (dim == 3) r = make_double4(X[3 * o], X[3 * o + 1], X[3 * o + 2], V ? V[o] : 0.0);
    else r = make_double4(X[2 * o], X[2 * o + 1], V ? V[o] : 0.0, 0.0);
    reinterpret_cast<double4 *>(xv)[s] = r;
}

// internal vectors use a padded stride: 4 doubles in 3-d, 2 in 2-d
__global__ void gather_vec_k(const int32_t *perm, uint32_t n, int dim, const double *src,
                             double *dst) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = perm[s];
    if (dim == 3) {
        double4 r = src ? make_double4(src[3 * o], src[3 * o + 1], src[3 * o + 2], 0.0)
                        : make_double4(0, 0, 0, 0);
        reinterpret_cast<double4 *>(dst)[s] = r;
    } else {
        double2 r = src ? make_double2(src[2 * o], src[2 * o + 1]) : make_double2(0, 0);
        reinterpret_cast<double2 *>(dst)[s] = r;
    }
}

__global__ void scatter_vec_k(const int32_t *perm, uint32_t n, int dim, const double *src,
                              double *dst) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = perm[s];
    if (dim == 3) {
        const double4 r = reinterpret_cast<const double4 *>(src)[s];
        dst[3 * o] = r.x;
        dst[3 * o + 1] = r.y;
        dst[3 * o + 2] = r.z;
    } else {
        const double2 r = reinterpret_cast<const double2 *>(src)[s];
        dst[2 * o] = r.x;
        dst[2 * o + 1] = r.y;
    }
}

__global__ void scatter_scalar_k(const int32_t *perm, uint32_t n, const double *src, double *dst) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[perm[s]] = src[s];
}

__global__ void gather_u8_k(const int32_t *perm, uint32_t n, const uint8_t *src, uint8_t *dst,
                            uint8_t fill) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = src ? src[perm[s]] : fill;
}

// bond flags between exported and internal order through the exported
// position of each internal bond
template <bool IN>
__global__ void alive_move_k(const uint32_t *ex_pos, uint64_t nnz, const uint8_t *src,
                             uint8_t *dst) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    if (IN) dst[p] = src ? src[ex_pos[p]] : (uint8_t)1;
    else dst[ex_pos[p]] = src[p];
}

__global__ void sum_partials_k(const double *data, uint32_t n, int slots, double *part) {
    __shared__ double sh[PD_BLOCK];
    for (int s = 0; s < slots; ++s) {
        double acc = 0.0;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (uint64_t)gridDim.x * blockDim.x)
            acc += data[i * slots + s];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[s * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ void vol_range_k(const double *xv, uint32_t n, int vi, double *part) {
    __shared__ double smin[PD_BLOCK], smax[PD_BLOCK];
    double mn = INFINITY, mx = -INFINITY;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = xv[4 * i + vi];
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int off = PD_BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = smin[0];
        part[gridDim.x + blockIdx.x] = smax[0];
    }
}

__global__ void flag_clear_k(int *flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}
}  // namespace

int pd_gather_xv(pd_ctx ctx, const pd_nbr nbr, const double *X, const double *V, double *xv) {
    gather_xv_k<<<pd_blocks(nbr->n), PD_BLOCK, 0, ctx->stream>>>(nbr->perm, nbr->n, nbr->dim, X,
                                                                  V, xv);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_gather_vec(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst, bool) {
    gather_vec_k<<<pd_blocks(nbr->n), PD_BLOCK, 0, ctx->stream>>>(nbr->perm, nbr->n, nbr->dim,
                                                                   src, dst);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_scatter_vec(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst) {
    scatter_vec_k<<<pd_blocks(nbr->n), PD_BLOCK, 0, ctx->stream>>>(nbr->perm, nbr->n, nbr->dim,
                                                                    src, dst);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_scatter_scalar(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst) {
    scatter_scalar_k<<<pd_blocks(nbr->n), PD_BLOCK, 0, ctx->stream>>>(nbr->perm, nbr->n, src, dst);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_gather_u8(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst, uint8_t fill) {
    gather_u8_k<<<pd_blocks(nbr->n), PD_BLOCK, 0, ctx->stream>>>(nbr->perm, nbr->n, src, dst, fill);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_alive_in(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst) {
    alive_move_k<true><<<pd_blocks(nbr->nnz), PD_BLOCK, 0, ctx->stream>>>(nbr->ex_pos, nbr->nnz,
                                                                          src, dst);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_alive_out(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst) {
    alive_move_k<false><<<pd_blocks(nbr->nnz), PD_BLOCK, 0, ctx->stream>>>(nbr->ex_pos, nbr->nnz,
                                                                           src, dst);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_sum(pd_ctx ctx, const double *data, uint32_t n, int slots, double *out) {
    if (slots < 1 || slots > PD_RED_SLOTS) return pd_set_error(ctx, PD_EINVAL, "bad slot count");
    sum_partials_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, ctx->stream>>>(data, n, slots, ctx->red);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(ctx->red_host, ctx->red, sizeof(double) * PD_RED_BLOCKS * slots,
                               hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < slots; ++s) {
        double acc = 0.0;
        for (int k = 0; k < PD_RED_BLOCKS; ++k) acc += ctx->red_host[s * PD_RED_BLOCKS + k];
        out[s] = acc;
    }
    return PD_OK;
}

int pd_uniform_volume(pd_ctx ctx, const pd_nbr nbr, const double *xv, double *V) {
    vol_range_k<<<PD_RED_BLOCKS, PD_BLOCK, 0, ctx->stream>>>(xv, nbr->n, nbr->dim == 3 ? 3 : 2,
                                                              ctx->red);
    PD_LAUNCH_CHECK(ctx);
    PD_HIP(ctx, hipMemcpyAsync(ctx->red_host, ctx->red, sizeof(double) * 2 * PD_RED_BLOCKS,
                               hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double mn = INFINITY, mx = -INFINITY;
    for (int k = 0; k < PD_RED_BLOCKS; ++k) {
        mn = fmin(mn, ctx->red_host[k]);
        mx = fmax(mx, ctx->red_host[PD_RED_BLOCKS + k]);
    }
    *V = (nbr->n > 0 && mn == mx) ? mn : 0.0;
    return PD_OK;
}

int pd_flag_clear(pd_ctx ctx) {
    flag_clear_k<<<1, 64, 0, ctx->stream>>>(ctx->flag);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_flag_read(pd_ctx ctx, int *value) {
    PD_HIP(ctx, hipMemcpyAsync(ctx->flag_host, ctx->flag, sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    PD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *value = *ctx->flag_host;
    return PD_OK;
}
