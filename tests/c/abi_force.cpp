// A host program that uses the library through its C ABI alone (no Python,
// no PyTorch): on one mesh it calls every entry point of the hot path --
// the neighbour lists, one internal-force evaluation (Algorithm 1,
// linearised law), the tangent applied to a vector, a velocity-Verlet
// trajectory and the quasi-static solve -- all in FP64, and writes the
// results back.
//
//   abi_force <in.bin> <out.bin>
//   in:  int64 n, dim, nsteps; float64 delta, c, dt; float64 X[n][dim], V[n],
//        u[n][dim], b[n][dim]; uint8 fixed[n]
//   out: int64 nnz, int64 row_ptr[n+1], int32 col[nnz], float64 f[n][dim]
//        (force at u), y[n][dim] (tangent applied to u, fixed rows
//        identity), uT[n][dim], vT[n][dim] (nsteps steps of dt from u, v = 0,
//        free boundary), us[n][dim] (solution of the quasi-static problem
//        with body force b and the fixed nodes clamped), float64 rel_residual
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
    int64_t n = 0, dim = 0, nsteps = 0;
    double delta = 0.0, c = 0.0, dt = 0.0;
    if (!rd(fi, &n, 1) || !rd(fi, &dim, 1) || !rd(fi, &nsteps, 1) || !rd(fi, &delta, 1) ||
        !rd(fi, &c, 1) || !rd(fi, &dt, 1))
        return 2;
    const size_t nd = (size_t)(n * dim);
    std::vector<double> X(nd), V((size_t)n), u(nd), b(nd), f(nd), y(nd), uT(nd), vT(nd), us(nd);
    std::vector<uint8_t> fixed((size_t)n);
    if (!rd(fi, X.data(), nd) || !rd(fi, V.data(), (size_t)n) || !rd(fi, u.data(), nd) ||
        !rd(fi, b.data(), nd) || !rd(fi, fixed.data(), (size_t)n))
        return 2;
    std::fclose(fi);

    pd_ctx ctx = nullptr;
    int st = pd_ctx_create(0, nullptr, &ctx);
    if (st != PD_OK) return fail("pd_ctx_create", st, nullptr);
    double *dX = nullptr, *dV = nullptr, *du = nullptr, *df = nullptr, *dy = nullptr,
           *db = nullptr, *dv = nullptr, *dus = nullptr;
    uint8_t *dfix = nullptr;
    if (hipMalloc((void **)&dX, nd * 8) != hipSuccess || hipMalloc((void **)&dV, n * 8) != hipSuccess ||
        hipMalloc((void **)&du, nd * 8) != hipSuccess || hipMalloc((void **)&df, nd * 8) != hipSuccess ||
        hipMalloc((void **)&dy, nd * 8) != hipSuccess || hipMalloc((void **)&db, nd * 8) != hipSuccess ||
        hipMalloc((void **)&dv, nd * 8) != hipSuccess || hipMalloc((void **)&dus, nd * 8) != hipSuccess ||
        hipMalloc((void **)&dfix, (size_t)n) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(dX, X.data(), nd * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dV, V.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(du, u.data(), nd * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(db, b.data(), nd * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dfix, fixed.data(), (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(dus, 0, nd * 8) != hipSuccess) {
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
    st = pd_apply_tangent(ctx, nbr, &mat, dX, dV, nullptr, dfix, du, dy);
    if (st != PD_OK) return fail("pd_apply_tangent", st, ctx);
    pd_sim sim = nullptr;
    st = pd_sim_create(ctx, nbr, &mat, dX, dV, du, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0,
                       &sim);
    if (st != PD_OK) return fail("pd_sim_create", st, ctx);
    st = pd_verlet_step(sim, nsteps, dt);
    if (st != PD_OK) return fail("pd_verlet_step", st, ctx);
    double *duT = dus;   // u after the steps (read back before dus takes the solve)
    st = pd_sim_get(sim, duT, dv, nullptr, nullptr, nullptr);
    if (st != PD_OK) return fail("pd_sim_get", st, ctx);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(f.data(), df, nd * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(y.data(), dy, nd * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(uT.data(), duT, nd * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(vT.data(), dv, nd * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(dus, 0, nd * 8) != hipSuccess) {
        std::fprintf(stderr, "read-back failed\n");
        return 1;
    }
    pd_sim_destroy(sim);
    pd_solve_info info = {};
    st = pd_solve_implicit(ctx, nbr, &mat, dX, dV, nullptr, dfix, db, dus, 1e-10, 100000, &info);
    if (st != PD_OK) return fail("pd_solve_implicit", st, ctx);
    if (hipMemcpy(us.data(), dus, nd * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        std::fprintf(stderr, "read-back failed\n");
        return 1;
    }
    pd_nbr_destroy(nbr);
    pd_ctx_destroy(ctx);
    for (void *p : {(void *)dX, (void *)dV, (void *)du, (void *)df, (void *)dy, (void *)db,
                    (void *)dv, (void *)dus, (void *)dfix})
        (void)hipFree(p);

    std::FILE *fo = std::fopen(argv[2], "wb");
    if (!fo) return 2;
    std::fwrite(&nnz, 8, 1, fo);
    std::fwrite(row_ptr.data(), 8, row_ptr.size(), fo);
    std::fwrite(col.data(), 4, col.size(), fo);
    for (const std::vector<double> *a : {&f, &y, &uT, &vT, &us}) std::fwrite(a->data(), 8, a->size(), fo);
    std::fwrite(&info.rel_residual, 8, 1, fo);
    std::fclose(fo);
    return 0;
}
