// A host program that uses the library through its C ABI alone (no Python,
// no PyTorch): it reads a mesh, builds the neighbour lists, evaluates the
// internal force once (Algorithm 1, linearised law) and writes the exported
// lists and the force back.
//
//   abi_force <in.bin> <out.bin>
//   in:  int64 n, int64 dim, float64 delta, float64 c, then float64 X[n][dim],
//        V[n], u[n][dim]
//   out: int64 nnz, int64 row_ptr[n+1], int32 col[nnz], float64 f[n][dim]
// Exit status 0 on success; otherwise the failing call and the library's
// message on stderr.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "pd.h"

static int fail(const char *what, int st, pd_ctx ctx) {
    std::fprintf(stderr, "%s: %s (%s)\n", what, pd_status_string(st),
                 ctx ? pd_last_error(ctx) : "");
    return 1;
}

template <class T>
static bool rd(std::FILE *f, T *p, size_t n) { return std::fread(p, sizeof(T), n, f) == n; }

int main(int argc, char **argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: abi_force in.bin out.bin\n");
        return 2;
    }
    std::FILE *fi = std::fopen(argv[1], "rb");
    if (!fi) return 2;
    int64_t n = 0, dim = 0;
    double delta = 0.0, c = 0.0;
    if (!rd(fi, &n, 1) || !rd(fi, &dim, 1) || !rd(fi, &delta, 1) || !rd(fi, &c, 1)) return 2;
    const size_t nd = (size_t)(n * dim);
    std::vector<double> X(nd), V((size_t)n), u(nd), f(nd);
    if (!rd(fi, X.data(), nd) || !rd(fi, V.data(), (size_t)n) || !rd(fi, u.data(), nd)) return 2;
    std::fclose(fi);

    pd_ctx ctx = nullptr;
    int st = pd_ctx_create(0, nullptr, &ctx);
    if (st != PD_OK) return fail("pd_ctx_create", st, nullptr);
    double *dX = nullptr, *dV = nullptr, *du = nullptr, *df = nullptr;
    if (hipMalloc((void **)&dX, nd * 8) != hipSuccess || hipMalloc((void **)&dV, n * 8) != hipSuccess ||
        hipMalloc((void **)&du, nd * 8) != hipSuccess || hipMalloc((void **)&df, nd * 8) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(dX, X.data(), nd * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dV, V.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(du, u.data(), nd * 8, hipMemcpyHostToDevice) != hipSuccess) {
        std::fprintf(stderr, "hipMemcpy failed\n");
        return 1;
    }
    pd_nbr nbr = nullptr;
    st = pd_build_neighbors(ctx, (int)dim, n, dX, delta, &nbr);
    if (st != PD_OK) return fail("pd_build_neighbors", st, ctx);
    int64_t nnz = 0;
    st = pd_nbr_info(nbr, &nnz, nullptr);
    if (st != PD_OK) return fail("pd_nbr_info", st, ctx);
    std::vector<int64_t> row_ptr((size_t)n + 1);
    std::vector<int32_t> col((size_t)nnz);
    st = pd_nbr_export(nbr, row_ptr.data(), col.data());
    if (st != PD_OK) return fail("pd_nbr_export", st, ctx);

    pd_material mat = {};
    mat.dim = (int)dim;
    mat.precision = PD_FP64;
    mat.c = c;
    mat.rho = 1.0;
    st = pd_internal_force(ctx, nbr, &mat, dX, dV, du, nullptr, df, nullptr);
    if (st != PD_OK) return fail("pd_internal_force", st, ctx);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(f.data(), df, nd * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        std::fprintf(stderr, "read-back failed\n");
        return 1;
    }
    pd_nbr_destroy(nbr);
    pd_ctx_destroy(ctx);
    (void)hipFree(dX);
    (void)hipFree(dV);
    (void)hipFree(du);
    (void)hipFree(df);

    std::FILE *fo = std::fopen(argv[2], "wb");
    if (!fo) return 2;
    std::fwrite(&nnz, 8, 1, fo);
    std::fwrite(row_ptr.data(), 8, row_ptr.size(), fo);
    std::fwrite(col.data(), 4, col.size(), fo);
    std::fwrite(f.data(), 8, f.size(), fo);
    std::fclose(fo);
    return 0;
}
