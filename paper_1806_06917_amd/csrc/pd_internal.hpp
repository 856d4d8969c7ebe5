// Internal declarations of the gfx950 peridynamics library (not installed).
//
// Data layout in HBM (internal "sfc" order = nodes sorted along a Morton
// space-filling curve of their horizon-sized bins, so that the neighbours of
// consecutive nodes are close in memory):
//   XV      double[n][4]   {x, y, z, V} (3-d) or {x, y, V, 0} (2-d), constant
//   u, v    double[n][US]  US = 4 in 3-d ({x, y, z, 0}), 2 in 2-d
//   row_ptr uint32[n+1], col int32[nnz] (sfc ids), rows ascending by the
//           neighbour's sfc id (so the lanes of a node read nearby records);
//           ex_pos uint32[nnz] maps each bond to its position in the exported
//           CSR (original numbering, neighbours ascending by original id)
//   alive   uint8[nnz]     1 = intact
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "pd.h"

#define PD_VERSION_NUMBER 10000

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
// one autotuner result: the fastest tile size and lane count measured for
// meshes of a dimension, neighbour-count bucket and precision
struct pd_tune_entry {
    int dim = 0, bucket = 0, precision = 0;
    int tile = 0, lanes = 0;
    double us = 0.0;
};

struct pd_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int lanes = 0;          // 0: automatic
    int kernel = 0;         // 0: automatic, 1: gather, 2: LDS tiles, 3: streamed tiles
    int tile = 0;           // nodes per tile, 0: automatic
    int block = 0;          // threads per tile workgroup, 0: automatic
    int num_cu = 256;       // compute units of the device
    int failed = 0;         // sticky device failure
    std::string last_error;
    double *red = nullptr;  // device partial sums, PD_RED_BLOCKS * PD_RED_SLOTS
    double *red_host = nullptr;  // pinned mirror of red
    int *flag = nullptr;    // device status word (non-finite, coincident ...)
    int *flag_host = nullptr;
    int refs = 0;           // neighbour lists and simulations created on this context
    bool closing = false;   // destroyed while refs > 0: freed with the last of them
    std::vector<pd_tune_entry> tuned;   // autotuner cache
};

struct pd_nbr_s {
    pd_ctx ctx = nullptr;
    int dim = 0;
    uint32_t n = 0;
    uint64_t nnz = 0;
    int32_t max_row = 0;
    double delta = 0, thr = 0;
    int32_t *perm = nullptr;     // sfc -> original
    int32_t *iperm = nullptr;    // original -> sfc
    uint32_t *row_ptr = nullptr; // [n+1] sfc order
    int32_t *col = nullptr;      // [nnz] sfc ids
    uint32_t *ex_row_ptr = nullptr;  // [n+1] original order
    uint32_t *ex_pos = nullptr;      // [nnz] exported position of each internal bond
    // LDS tiles (pd_tile.hip): T consecutive sfc nodes per tile
    uint32_t tile_T = 0, ntiles = 0, halo_max = 0, bonds_max = 0;
    uint64_t halo_total = 0;
    uint32_t *halo_ptr = nullptr;  // [ntiles+1]
    int32_t *halo = nullptr;       // sorted sfc ids of each tile's halo
    uint32_t *self_off = nullptr;  // [ntiles] local index of the tile's first node
    uint16_t *lcol = nullptr;      // [nnz] tile-local neighbour index
    uint64_t fail_key = 0;         // last tuning request no tile layout fitted (+1)
    int users = 0;                 // simulations attached (their bond words use the tiles)
    int refs = 0;                  // simulations built on this list
    bool closing = false;          // destroyed while refs > 0: freed with the last of them
    uint16_t *s_bw = nullptr;      // scratch bond words for the stateless entry points
    // scratch for the stateless entry points (pd_internal_force, pd_apply_tangent)
    double *s_xv = nullptr, *s_u = nullptr, *s_f = nullptr, *s_U = nullptr;
    double *s_ulin = nullptr;    // linearisation point of the NP tangent
    double *s_lps = nullptr;     // {m, theta} per node of the peridynamic solid
    uint8_t *s_alive = nullptr, *s_fixed = nullptr;
};

struct pd_sim_s {
    pd_ctx ctx = nullptr;
    pd_nbr nbr = nullptr;
    pd_material mat{};
    double *xv = nullptr;
    double *u[2] = {nullptr, nullptr};
    int cur = 0;
    double *v = nullptr;
    double *bc_vel = nullptr;
    double *b = nullptr;
    uint8_t *bc = nullptr;
    uint8_t *alive = nullptr;    // bond flags (gather kernel; export copy for tiles)
    uint16_t *bw = nullptr;      // bond words (tile kernel): local index | dead bit
    bool tiled = false;          // this simulation runs the tile kernel
    int block = 0;               // its tile-kernel workgroup size (0: gather kernel)
    double cv_uniform = 0.0;     // c V if all volumes are equal, else 0
    double *scratch = nullptr;   // [n] per-node energies for diagnostics
    double *lps = nullptr;       // [n][2] {m, theta} (linear peridynamic solid)
    double *lpsc = nullptr;      // [n][2] {a, d} of the solid's streamed steps (float32 pairs in mixed precision)
    int64_t step = 0;
    int64_t ramp = 0;
    double last_dt = 0;
    bool v_half = false;         // v holds v^{k-1/2} (force at u^k still to be applied)
    int lanes = 0;
    // streamed steps: node records {X, u} (ping-pong with u), launch geometry
    double *rec[2] = {nullptr, nullptr};
    bool stream = false;
    bool u_stale = false;        // rec[cur] is newer than u[cur]
    bool rec_stale = true;       // u[cur] is newer than rec[cur]
    int s_block = 0;
    unsigned s_grid = 0;
    uint32_t s_mmax = 0;
    size_t s_lds = 0;
    int s_form = 0;              // SK_LINEAR, SK_NP or SK_LPS_FORCE (two launches a step)
    int s2_block = 0;            // the solid's state pass: its own launch geometry
    unsigned s2_grid = 0;
    uint32_t s2_mmax = 0;
    size_t s2_lds = 0;
    double vol_uniform = 0.0;    // the common nodal volume (0: volumes differ)
};

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
int pd_set_error(pd_ctx ctx, int status, const char *fmt, ...);
int pd_hip_error(pd_ctx ctx, hipError_t e, const char *what, const char *file, int line);

#define PD_HIP(ctx, call)                                                   \
    do {                                                                    \
        hipError_t e__ = (call);                                            \
        if (e__ != hipSuccess) return pd_hip_error((ctx), e__, #call, __FILE__, __LINE__); \
    } while (0)

#define PD_TRY(expr)                 \
    do {                             \
        int s__ = (expr);            \
        if (s__ != PD_OK) return s__; \
    } while (0)

#define PD_LAUNCH_CHECK(ctx) PD_HIP(ctx, hipGetLastError())

// Device memory of the library's own buffers, through a per-device cache
// (pd_runtime.hip): a freed block is kept and handed out again once the work
// queued on its owner's stream before the free has completed.
int pd_alloc_bytes(pd_ctx ctx, void **p, size_t bytes);
void pd_free_bytes(void *p);
// the live blocks owned by stream `from` (except keep1, keep2) now belong to
// stream `to`: their frees wait for the work queued there
void pd_mem_restream(hipStream_t from, hipStream_t to, const void *keep1, const void *keep2);
// moves an idle simulation and its neighbour list (used by no other
// simulation) to another context of the same device (pd_force.hip)
int pd_sim_rehome(pd_sim s, pd_ctx to);

template <class T>
int pd_alloc(pd_ctx ctx, T **p, size_t count) {
    if (count == 0) count = 1;
    void *q = nullptr;
    const int st = pd_alloc_bytes(ctx, &q, count * sizeof(T));
    *p = (T *)q;
    return st;
}

template <class T>
void pd_free(T *&p) {
    if (p) pd_free_bytes((void *)p);
    p = nullptr;
}

int pd_check_ctx(pd_ctx ctx);

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
constexpr int PD_BLOCK = 256;
constexpr int PD_RED_BLOCKS = 512;
constexpr int PD_RED_SLOTS = 4;

inline unsigned pd_blocks(uint64_t threads, int block = PD_BLOCK) {
    return (unsigned)((threads + block - 1) / block);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  This
// remaps the hardware block index so that each XCD receives one contiguous
// range of tiles (neighbouring nodes share that XCD's L2).
__device__ __forceinline__ uint32_t pd_xcd_tile(uint32_t b, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t q = nb / X, r = nb % X, x = b % X, l = b / X;
    return x * q + (x < r ? x : r) + l;
}

int pd_auto_lanes(pd_ctx ctx, uint64_t nnz, uint32_t n);

// ---------------------------------------------------------------------------
// shared host helpers (implemented in pd_runtime.hip)
// ---------------------------------------------------------------------------
// exclusive scan of uint32 counts -> uint64 offsets (out has n+1 entries)
int pd_scan_u32(pd_ctx ctx, const uint32_t *in, uint64_t *out, uint32_t n);
// out[k] = (uint32) in[k]
int pd_narrow_u64(pd_ctx ctx, const uint64_t *in, uint32_t *out, uint32_t n);
// sfc-order copies of original-order nodal arrays, and back
int pd_gather_xv(pd_ctx ctx, const pd_nbr nbr, const double *X, const double *V, double *xv);
int pd_gather_vec(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst, bool zero_if_null);
int pd_scatter_vec(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst);
int pd_gather_u8(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst, uint8_t fill);
int pd_scatter_scalar(pd_ctx ctx, const pd_nbr nbr, const double *src, double *dst);
// bond flags: exported order <-> internal order (src NULL: all 1)
int pd_alive_in(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst);
int pd_alive_out(pd_ctx ctx, const pd_nbr nbr, const uint8_t *src, uint8_t *dst);
// deterministic sums of `slots` interleaved per-node values: data[i*slots + s]
int pd_sum(pd_ctx ctx, const double *data, uint32_t n, int slots, double *out);
// the common nodal volume if all n volumes are equal, else 0 (synchronises)
int pd_uniform_volume(pd_ctx ctx, const pd_nbr nbr, const double *xv, double *V);
// device status word
int pd_flag_clear(pd_ctx ctx);
int pd_flag_read(pd_ctx ctx, int *value);
// checks that a device pointer is accessible device memory of ctx's device
int pd_check_dev_ptr(pd_ctx ctx, const void *p, const char *name);

int pd_nbr_build_tiles(pd_ctx ctx, pd_nbr nbr, uint32_t T);

// handle lifetimes: a context or neighbour list destroyed while handles built
// on it are alive is freed when the last of those goes
void pd_ctx_unref(pd_ctx ctx);
void pd_nbr_unref(pd_nbr nbr);

// sfc-order building blocks of the implicit solver (pd_force.hip)
// bw + block > 0: tile kernel with bond words bw; otherwise the gather kernel
int pd_tangent_sfc(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, const double *xv,
                   const uint8_t *alive_sfc, uint16_t *bw, int block, const uint8_t *fixed_sfc,
                   const double *w, double *y, const int *done, const double *u_lin = nullptr);
int pd_force_sfc(pd_ctx ctx, const pd_nbr nbr, const pd_material *mat, const double *xv,
                 const uint8_t *alive_sfc, uint16_t *bw, int block, const double *u, double *f);
// pd_internal_force in pieces (pd_force.hip): argument checks; the
// internal-order buffers of one evaluation on the gather kernel (their size
// for a mesh and law, and their layout in one block of device memory); the
// evaluation itself with the caller's buffers (it allocates nothing)
struct pd_force_bufs {
    double *xv, *u, *f, *U, *lps;
    uint8_t *alive;
};
int pd_check_force_args(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                        const double *V, const double *u, const uint8_t *alive, const double *f,
                        const double *U);
size_t pd_force_bufs_bytes(const pd_nbr nbr, const pd_material *mat);
pd_force_bufs pd_force_bufs_carve(const pd_nbr nbr, const pd_material *mat, void *base);
int pd_force_gather(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                    const double *V, const double *u, uint8_t *alive, double *f, double *U,
                    const pd_force_bufs &b);
// the allocation-free entry point's device scratch: looked up once per device
// (pd_noalloc.hip; called by pd_ctx_create with the device current)
int pd_noalloc_setup(pd_ctx ctx);

// kernel choice for a call site under the context's tuning; *block > 0 means
// the tile kernel with that workgroup size, 0 the gather kernel
int pd_plan_kernel(pd_ctx ctx, pd_nbr nbr, int lanes, int *block);

// the material's pairwise law is not the linearised law of the tiled kernels
inline bool pd_general_law(const pd_material *m) {
    return m->law != PD_LAW_LINEAR || m->stretch != PD_STRETCH_LINEARISED || m->pv_h > 0.0 ||
           m->j_c2 > 0.0;
}
// law, stretch and beta are valid (pd_runtime.hip)
int pd_check_law(pd_ctx ctx, const pd_material *m);

// autotuner cache (pd_tune.hip): neighbour-count bucket of a mesh, lookup
int pd_tune_bucket(double mean_neighbors);
const pd_tune_entry *pd_tune_find(pd_ctx ctx, int dim, double mean_neighbors, int precision);
