// The allocation-free variant of the internal-force evaluation
// (pd_internal_force_noalloc): the same computation as pd_internal_force
// (Algorithm 1 and the other laws, on the gather kernel), with the
// internal-order copies of X, V, u, f, U, the solid's {m, theta} and the bond
// flags in a fixed device array of this file instead of buffers the library
// allocates.  It is for callers that cannot allocate device memory: code
// under stream capture, tight serving loops, harnesses that forbid it.
//
// The array lives in every device the library runs on until the process
// ends.  Host code never passes its name to a kernel (in host code the name
// is a stand-in, not a device address): pd_noalloc_setup looks its address
// up once per device, with that device current, and the entry point uses
// that address.  Every call on a device shares the array, so calls that
// overlap on one device race; each call rewrites every part it reads.
#include <mutex>

#include "pd_internal.hpp"

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;   // PD_NOALLOC_MAX_BYTES in pd.h
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mutex;
void *g_ptr[MAX_DEVICES] = {};

}  // namespace

int pd_noalloc_setup(pd_ctx ctx) {
    static_assert(NOALLOC_BYTES == (size_t)PD_NOALLOC_MAX_BYTES, "the header states the size");
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        return pd_set_error(ctx, PD_EDEVICE, "device index %d out of range", ctx->device);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[ctx->device]) return PD_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return pd_set_error(ctx, PD_EDEVICE, "scratch array address: %s", hipGetErrorString(e));
    }
    g_ptr[ctx->device] = p;
    return PD_OK;
}

extern "C" int pd_internal_force_noalloc(pd_ctx ctx, pd_nbr nbr, const pd_material *mat,
                                         const double *X, const double *V, const double *u,
                                         uint8_t *alive, double *f, double *U) {
    PD_TRY(pd_check_force_args(ctx, nbr, mat, X, V, u, alive, f, U));
    const size_t need = pd_force_bufs_bytes(nbr, mat);
    if (need > NOALLOC_BYTES)
        return pd_set_error(ctx, PD_ECAPACITY,
                            "the mesh needs %zu bytes of scratch, above the fixed %zu", need,
                            NOALLOC_BYTES);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        base = g_ptr[ctx->device];
    }
    if (!base) return pd_set_error(ctx, PD_EDEVICE, "scratch array not set up on this device");
    return pd_force_gather(ctx, nbr, mat, X, V, u, alive, f, U,
                           pd_force_bufs_carve(nbr, mat, base));
}
