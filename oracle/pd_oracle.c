/*
 * pd_oracle.c -- plain FP64 CPU oracle for bond-based peridynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library; it is written directly from the paper
 * (Diehl et al., "An asynchronous and task-based implementation of
 * peridynamics utilizing HPX", arXiv:1806.06917) and is deliberately slow and
 * literal: one node at a time, neighbours in ascending id order, every sum
 * sequential.  OpenMP (if enabled) only distributes whole nodes over threads,
 * so results are bit-identical for any thread count.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (contraction off so
 * that every product and sum below is a separately rounded IEEE operation).
 *
 * Notation (paper, Section "Peridynamics theory" and Algorithm 1):
 *   xi  = X_j - X_i          reference bond vector
 *   eta = u_j - u_i          bond deformation
 *   S   = (eta . xi)/|xi|^2  linearised bond strain (Algorithm 1)
 *   c   = 4 psi'(0) / (delta |B_delta(0)|)  micromodulus of the linearised law
 *   NP  = the nonlinear potential psi(r) = C (1 - exp(-beta r)) of the
 *         validation section, used in Algorithm 1 by or_force_law (with the
 *         exact-stretch variant), or_tangent_law and or_solve_law
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes):
 *   - the horizon ball is closed: |xi| <= delta, with the FP test
 *     d2 <= (delta*delta)*(1+1e-10) evaluated without fused multiply-add;
 *   - a node is not its own neighbour;
 *   - influence function J = 1 on the closed ball and the linearised
 *     potential psi'(r) -> psi'(0) (the "LP" model of the 2-d validation);
 *     or_force_law_j also takes the 1-d validation's influence function
 *     J(r) = c1 r exp(-r^2/c2) of r = |xi|/delta as a factor of each bond;
 *   - no partial-volume correction (V_ij = 1);
 *   - damage: a bond breaks, irreversibly and only in tension, at the first
 *     force evaluation where S > s_c (strict), before it contributes.
 *
 * Parity status: every function below is pinned by CPU tests against closed
 * forms, invariants or brute force (see the test suite); none is "parity
 * unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BC_FREE 0
#define OR_BC_CLAMPED 1
#define OR_BC_VELOCITY 2

/* ------------------------------------------------------------------------ */
/* Horizon membership (Section "Discretization": B_delta(X_i) = {X_j :        */
/* |X_j - X_i| <= delta}).                                                   */
/* ------------------------------------------------------------------------ */

double or_threshold(double delta) { return (delta * delta) * (1.0 + 1e-10); }

/* squared distance, summed x, then y, then z; every operation rounded */
static double or_dist2(int dim, const double *a, const double *b) {
    double dx = b[0] - a[0];
    double dy = b[1] - a[1];
    double d2 = dx * dx + dy * dy;
    if (dim == 3) {
        double dz = b[2] - a[2];
        d2 = d2 + dz * dz;
    }
    return d2;
}

/*
 * Brute force over all pairs: O(n^2).  row_ptr has n+1 entries.  With
 * col == NULL only row_ptr is filled.  Rows list neighbours in ascending id.
 * Returns nnz, or -1 if two distinct nodes coincide.
 */
int64_t or_nbr_brute(int dim, int64_t n, const double *X, double thr,
                     int64_t *row_ptr, int32_t *col) {
    int bad = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d2 = or_dist2(dim, X + i * dim, X + j * dim);
            if (d2 == 0.0) bad = 1;
            if (d2 <= thr) {
                if (col) col[row_ptr[i] + cnt] = (int32_t)j;
                ++cnt;
            }
        }
        if (!col) row_ptr[i + 1] = row_ptr[i] + cnt;
    }
    return bad ? -1 : row_ptr[n];
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * The same neighbour sets, found through square/cubic bins of edge >= delta:
 * candidates come from the 3^dim bins around the node's bin, then each row is
 * sorted ascending.  Same predicate as or_nbr_brute, so the same output.
 */
int64_t or_nbr_binned(int dim, int64_t n, const double *X, double thr,
                      int64_t *row_ptr, int32_t *col) {
    if (n <= 0) { row_ptr[0] = 0; return 0; }
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { lo[k] = X[k]; hi[k] = X[k]; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            double x = X[i * dim + k];
            if (x < lo[k]) lo[k] = x;
            if (x > hi[k]) hi[k] = x;
        }
    double edge = sqrt(thr) * (1.0 + 1e-12);
    int64_t nc[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) nc[k] = (int64_t)floor((hi[k] - lo[k]) / edge) + 1;
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *cstart = (int64_t *)calloc(ncell + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t cc[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            int64_t q = (int64_t)floor((X[i * dim + k] - lo[k]) / edge);
            if (q >= nc[k]) q = nc[k] - 1;
            if (q < 0) q = 0;
            cc[k] = q;
        }
        cell_of[i] = cc[0] + nc[0] * (cc[1] + nc[1] * cc[2]);
        cstart[cell_of[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ncell);
        memcpy(fill, cstart, sizeof(int64_t) * ncell);
        for (int64_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = i;
        free(fill);
    }
    int bad = 0;
    int64_t *cnt = (int64_t *)calloc(n, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        int64_t ci = cell_of[i];
        int64_t cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
        int64_t m = 0;
        int64_t base = col ? row_ptr[i] : 0;
        for (int64_t dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    int64_t x = cx + dx, y = cy + dy, z = cz + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= nc[0] || y >= nc[1] || z >= nc[2]) continue;
                    int64_t c = x + nc[0] * (y + nc[1] * z);
                    for (int64_t q = cstart[c]; q < cstart[c + 1]; ++q) {
                        int64_t j = order[q];
                        if (j == i) continue;
                        double d2 = or_dist2(dim, X + i * dim, X + j * dim);
                        if (d2 == 0.0) bad |= 1;
                        if (d2 <= thr) {
                            if (col) col[base + m] = (int32_t)j;
                            ++m;
                        }
                    }
                }
        cnt[i] = m;
        if (col) qsort(col + base, (size_t)m, sizeof(int32_t), cmp_i32);
    }
    if (!col) {
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    }
    free(cnt); free(cell_of); free(cstart); free(order);
    return bad ? -1 : row_ptr[n];
}

/* ------------------------------------------------------------------------ */
/* Micromodulus of the linearised bond law, c = 4 psi'(0)/(delta |B_delta|) */
/* (Algorithm 1), calibrated so that the strain-energy density under a      */
/* uniform isotropic strain equals the classical one: plane stress with      */
/* nu = 1/3 in 2-d, nu = 1/4 in 3-d (the bond-based restriction stated in    */
/* Section "Peridynamics theory").                                           */
/* ------------------------------------------------------------------------ */
double or_micromodulus(int dim, double E, double delta) {
    const double pi = 3.14159265358979323846;
    if (dim == 2) return 9.0 * E / (pi * delta * delta * delta);
    return 12.0 * E / (pi * delta * delta * delta * delta);
}

/* ------------------------------------------------------------------------ */
/* Internal force density and strain energy density, Algorithm 1 with       */
/* J = 1 and psi' = psi'(0) (linearised law):                               */
/*   f_i += c * S * (xi/|xi|) * V_j                                          */
/*   U_i += (c/4) * S^2 * |xi| * V_j                                         */
/* (c/4 = psi'(0)/(delta |B_delta|), psi(r) = psi'(0) r).                    */
/* alive == NULL: every bond intact and no damage.  Otherwise a dead bond is */
/* skipped, and with s_c > 0 a live bond with S > s_c is broken before it   */
/* contributes.  U may be NULL.                                              */
/* ------------------------------------------------------------------------ */
void or_force(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
              const double *X, const double *V, const double *u, double c,
              double s_c, uint8_t *alive, double *f, double *U) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        double Ui = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            double xi[3] = {0, 0, 0}, eta[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                xi[k] = X[j * dim + k] - X[i * dim + k];
                eta[k] = u[j * dim + k] - u[i * dim + k];
            }
            double r2 = 0.0, ex = 0.0;
            for (int k = 0; k < dim; ++k) {
                r2 = r2 + xi[k] * xi[k];
                ex = ex + eta[k] * xi[k];
            }
            double S = ex / r2;
            if (alive && s_c > 0.0 && S > s_c) {
                alive[p] = 0;
                continue;
            }
            double r = sqrt(r2);
            for (int k = 0; k < dim; ++k) fi[k] = fi[k] + c * S * (xi[k] / r) * V[j];
            if (U) Ui = Ui + 0.25 * c * S * S * r * V[j];
        }
        for (int k = 0; k < dim; ++k) f[i * dim + k] = fi[k];
        if (U) U[i] = Ui;
    }
}

/* Kinetic energy sum_i rho V_i |v_i|^2 / 2 and potential energy
 * sum_i V_i U_i (each a plain sequential sum). */
double or_kinetic(int dim, int64_t n, const double *V, double rho, const double *v) {
    double ke = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s = s + v[i * dim + k] * v[i * dim + k];
        ke = ke + 0.5 * rho * V[i] * s;
    }
    return ke;
}

double or_potential(int64_t n, const double *V, const double *U) {
    double pe = 0.0;
    for (int64_t i = 0; i < n; ++i) pe = pe + V[i] * U[i];
    return pe;
}

/* ------------------------------------------------------------------------ */
/* Pre-crack: a bond is cut when the closed segment [X_i, X_j] meets a notch */
/* segment [A, B] (2-d).  Orientation tests in FP64 without contraction; the */
/* bond's end points are put in a canonical order first so that (i,j) and   */
/* (j,i) get the same answer.                                                */
/* ------------------------------------------------------------------------ */
static double or_orient(double ax, double ay, double bx, double by, double cx, double cy) {
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}
static int or_sgn(double x) { return (x > 0.0) - (x < 0.0); }
static double or_min(double a, double b) { return a < b ? a : b; }
static double or_max(double a, double b) { return a > b ? a : b; }

static int or_segments_meet(double px, double py, double qx, double qy,
                            double ax, double ay, double bx, double by) {
    if (qx < px || (qx == px && qy < py)) {
        double tx = px, ty = py;
        px = qx; py = qy; qx = tx; qy = ty;
    }
    int o1 = or_sgn(or_orient(ax, ay, bx, by, px, py));
    int o2 = or_sgn(or_orient(ax, ay, bx, by, qx, qy));
    int o3 = or_sgn(or_orient(px, py, qx, qy, ax, ay));
    int o4 = or_sgn(or_orient(px, py, qx, qy, bx, by));
    if (o1 == 0 && o2 == 0 && o3 == 0 && o4 == 0) {
        /* collinear: the projections on both axes must overlap */
        return or_max(or_min(px, qx), or_min(ax, bx)) <= or_min(or_max(px, qx), or_max(ax, bx)) &&
               or_max(or_min(py, qy), or_min(ay, by)) <= or_min(or_max(py, qy), or_max(ay, by));
    }
    return o1 * o2 <= 0 && o3 * o4 <= 0;
}

void or_notch_cut(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *X, int nseg, const double *seg, uint8_t *alive) {
    if (dim != 2) return;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col[p];
            for (int s = 0; s < nseg; ++s)
                if (or_segments_meet(X[2 * i], X[2 * i + 1], X[2 * j], X[2 * j + 1],
                                     seg[4 * s], seg[4 * s + 1], seg[4 * s + 2], seg[4 * s + 3]))
                    alive[p] = 0;
        }
}

/* ------------------------------------------------------------------------ */
/* Velocity-Verlet (the three velocity-Verlet equations of Section          */
/* "Explicit time integration", with the density rho), boundary data         */
/* applied at t^{k+1}:                                                       */
/*   v^{k+1/2} = v^k + (dt/2) (f^k + b)/rho                                  */
/*   u^{k+1}   = u^k + dt v^{k+1/2}                                          */
/*   (boundary conditions at t^{k+1})                                        */
/*   f^{k+1}   = force(u^{k+1})  (with the damage update)                    */
/*   v^{k+1}   = v^{k+1/2} + (dt/2) (f^{k+1} + b)/rho                        */
/* Clamped nodes keep u = v = 0.  Prescribed-velocity nodes skip both kicks: */
/* v^{k+1/2} = r(k+1/2) vbar, u^{k+1} = u^k + dt v^{k+1/2},                  */
/* v^{k+1} = r(k+1) vbar, with the ramp r(s) = min(1, s/ramp) (r = 1 when    */
/* ramp <= 0).  On entry f holds force(u^k) for the current step index       */
/* step0; b may be NULL (zero).                                              */
/* ------------------------------------------------------------------------ */
static double or_ramp(double s, int64_t ramp) {
    if (ramp <= 0) return 1.0;
    double r = s / (double)ramp;
    return r < 1.0 ? r : 1.0;
}

/* or_verlet_law / or_verlet_lps: the same steps with the force of the     */
/* general pairwise law (or_force_law) or of the linear peridynamic solid   */
/* (or_lps); or_verlet is the linearised law (law 0, stretch 0), for which  */
/* or_force_law and or_force agree bit for bit.                             */
void or_force_law_pv(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *X, const double *V, const double *u, double c, double s_c,
                     int law, double beta, int stretch, double pv_h, double pv_R,
                     uint8_t *alive, double *f, double *U);
void or_force_law_j(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *X, const double *V, const double *u, double c, double s_c,
                    int law, double beta, int stretch, double pv_h, double pv_R, double j_c1,
                    double j_c2, double j_delta, uint8_t *alive, double *f, double *U);
void or_lps_pv(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
               const double *V, const double *u, double K, double mu, double pv_h, double pv_R,
               const uint8_t *alive, double *m, double *theta, double *f, double *W);

typedef struct {
    int dim, law, stretch;
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *X, *V;
    double c, s_c, beta, K, mu;
    int lps;
    double pv_h, pv_R;
    double j_c1, j_c2, j_delta;   /* influence function (j_c2 = 0: J = 1) */
} or_model;

static void or_model_force(const or_model *md, const double *u, uint8_t *alive, double *f) {
    if (md->lps)
        or_lps_pv(md->n, md->row_ptr, md->col, md->X, md->V, u, md->K, md->mu, md->pv_h,
                  md->pv_R, alive, NULL, NULL, f, NULL);
    else
        or_force_law_j(md->dim, md->n, md->row_ptr, md->col, md->X, md->V, u, md->c, md->s_c,
                       md->law, md->beta, md->stretch, md->pv_h, md->pv_R, md->j_c1, md->j_c2,
                       md->j_delta, alive, f, NULL);
}

static void or_verlet_core(const or_model *md, double rho, const uint8_t *bc_kind,
                           const double *bc_vel, const double *b, int64_t ramp, double dt,
                           int64_t step0, int64_t nsteps, double *u, double *v, double *f,
                           uint8_t *alive) {
    const int dim = md->dim;
    const int64_t n = md->n;
    for (int64_t k = step0; k < step0 + nsteps; ++k) {
        double rh = or_ramp((double)k + 0.5, ramp);
        double r1 = or_ramp((double)(k + 1), ramp);
        for (int64_t i = 0; i < n; ++i) {
            int kind = bc_kind ? bc_kind[i] : OR_BC_FREE;
            for (int d = 0; d < dim; ++d) {
                int64_t q = i * dim + d;
                if (kind == OR_BC_CLAMPED) {
                    u[q] = 0.0;
                    v[q] = 0.0;
                } else if (kind == OR_BC_VELOCITY) {
                    double vh = rh * bc_vel[q];
                    u[q] = u[q] + dt * vh;
                    v[q] = vh;
                } else {
                    double bq = b ? b[q] : 0.0;
                    double vh = v[q] + (0.5 * dt) * (f[q] + bq) / rho;
                    u[q] = u[q] + dt * vh;
                    v[q] = vh;
                }
            }
        }
        or_model_force(md, u, alive, f);
        for (int64_t i = 0; i < n; ++i) {
            int kind = bc_kind ? bc_kind[i] : OR_BC_FREE;
            for (int d = 0; d < dim; ++d) {
                int64_t q = i * dim + d;
                if (kind == OR_BC_CLAMPED) {
                    v[q] = 0.0;
                } else if (kind == OR_BC_VELOCITY) {
                    v[q] = r1 * bc_vel[q];
                } else {
                    double bq = b ? b[q] : 0.0;
                    v[q] = v[q] + (0.5 * dt) * (f[q] + bq) / rho;
                }
            }
        }
    }
}

/* Central-difference scheme (the finite-difference equation of Section      */
/* "Explicit time integration"): for free nodes                             */
/*   u^{k+1} = 2 u^k - u^{k-1} + dt^2/rho (f^k + b),                         */
/* boundary nodes as in the velocity-Verlet steps.  The paper gives no      */
/* starting rule: the first step is one velocity-Verlet step from (u, v),   */
/* which is the Taylor start u^1 = u^0 + dt v^0 + dt^2/(2 rho)(f^0 + b).    */
/* On return u = u^N, f = f^N and, for free nodes, v = v^N =                */
/* (u^N - u^{N-1})/dt + dt/(2 rho)(f^N + b), the velocity-Verlet velocity.  */
static void or_central_core(const or_model *md, double rho, const uint8_t *bc_kind,
                            const double *bc_vel, const double *b, int64_t ramp, double dt,
                            int64_t step0, int64_t nsteps, double *u, double *v, double *f,
                            uint8_t *alive) {
    const int dim = md->dim;
    const int64_t n = md->n, m = n * dim;
    if (nsteps <= 0) return;
    double *up = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    for (int64_t q = 0; q < m; ++q) up[q] = u[q];
    or_verlet_core(md, rho, bc_kind, bc_vel, b, ramp, dt, step0, 1, u, v, f, alive);
    for (int64_t k = step0 + 1; k < step0 + nsteps; ++k) {
        double rh = or_ramp((double)k + 0.5, ramp);
        for (int64_t i = 0; i < n; ++i) {
            int kind = bc_kind ? bc_kind[i] : OR_BC_FREE;
            for (int d = 0; d < dim; ++d) {
                int64_t q = i * dim + d;
                double un;
                if (kind == OR_BC_CLAMPED) {
                    un = 0.0;
                } else if (kind == OR_BC_VELOCITY) {
                    un = u[q] + dt * (rh * bc_vel[q]);
                } else {
                    double bq = b ? b[q] : 0.0;
                    un = 2.0 * u[q] - up[q] + dt * dt * (f[q] + bq) / rho;
                }
                up[q] = u[q];
                u[q] = un;
            }
        }
        or_model_force(md, u, alive, f);
    }
    double r1 = or_ramp((double)(step0 + nsteps), ramp);
    for (int64_t i = 0; i < n; ++i) {
        int kind = bc_kind ? bc_kind[i] : OR_BC_FREE;
        for (int d = 0; d < dim; ++d) {
            int64_t q = i * dim + d;
            if (kind == OR_BC_CLAMPED) {
                v[q] = 0.0;
            } else if (kind == OR_BC_VELOCITY) {
                v[q] = r1 * bc_vel[q];
            } else if (nsteps > 1) {
                double bq = b ? b[q] : 0.0;
                v[q] = (u[q] - up[q]) / dt + (0.5 * dt) * (f[q] + bq) / rho;
            }
        }
    }
    free(up);
}

void or_central_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *X, const double *V, double rho, double c, double s_c,
                    int law, double beta, int stretch, const uint8_t *bc_kind,
                    const double *bc_vel, const double *b, int64_t ramp, double dt,
                    int64_t step0, int64_t nsteps, double *u, double *v, double *f,
                    uint8_t *alive) {
    or_model md = {dim, law, stretch, n, row_ptr, col, X, V, c, s_c, beta, 0.0, 0.0, 0, 0.0, 0.0,
                   0.0, 0.0, 0.0};
    or_central_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

void or_verlet_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const double *X, const double *V, double rho, double c, double s_c,
                   int law, double beta, int stretch,
                   const uint8_t *bc_kind, const double *bc_vel, const double *b,
                   int64_t ramp, double dt, int64_t step0, int64_t nsteps,
                   double *u, double *v, double *f, uint8_t *alive) {
    or_model md = {dim, law, stretch, n, row_ptr, col, X, V, c, s_c, beta, 0.0, 0.0, 0, 0.0, 0.0,
                   0.0, 0.0, 0.0};
    or_verlet_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

void or_verlet_lps(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
                   const double *V, double rho, double K, double mu, const uint8_t *bc_kind,
                   const double *bc_vel, const double *b, int64_t ramp, double dt,
                   int64_t step0, int64_t nsteps, double *u, double *v, double *f,
                   uint8_t *alive) {
    or_model md = {3, 0, 0, n, row_ptr, col, X, V, 0.0, 0.0, 0.0, K, mu, 1, 0.0, 0.0,
                   0.0, 0.0, 0.0};
    or_verlet_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

/* Velocity-Verlet steps with partial volumes (or_pv) under a pairwise law   */
/* (lps = 0: c, s_c, law, beta, stretch) or the peridynamic solid (lps = 1:  */
/* K, mu, dim 3).                                                            */
void or_verlet_pv(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *X, const double *V, double rho, int lps, double c, double s_c,
                  int law, double beta, int stretch, double K, double mu, double pv_h,
                  double pv_R, const uint8_t *bc_kind, const double *bc_vel, const double *b,
                  int64_t ramp, double dt, int64_t step0, int64_t nsteps, double *u, double *v,
                  double *f, uint8_t *alive) {
    or_model md = {dim, law, stretch, n, row_ptr, col, X, V, c, s_c, beta, K, mu, lps, pv_h, pv_R,
                   0.0, 0.0, 0.0};
    or_verlet_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

/* Velocity-Verlet and central-difference steps of a pairwise law with the  */
/* influence function J (or_force_law_j; j_c2 = 0: J = 1) and, optionally,  */
/* partial volumes.                                                          */
void or_verlet_j(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                 const double *X, const double *V, double rho, double c, double s_c, int law,
                 double beta, int stretch, double pv_h, double pv_R, double j_c1, double j_c2,
                 double j_delta, const uint8_t *bc_kind, const double *bc_vel, const double *b,
                 int64_t ramp, double dt, int64_t step0, int64_t nsteps, double *u, double *v,
                 double *f, uint8_t *alive) {
    or_model md = {dim, law, stretch, n, row_ptr, col, X, V, c, s_c, beta, 0.0, 0.0, 0, pv_h, pv_R,
                   j_c1, j_c2, j_delta};
    or_verlet_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

void or_central_j(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *X, const double *V, double rho, double c, double s_c, int law,
                  double beta, int stretch, double pv_h, double pv_R, double j_c1, double j_c2,
                  double j_delta, const uint8_t *bc_kind, const double *bc_vel, const double *b,
                  int64_t ramp, double dt, int64_t step0, int64_t nsteps, double *u, double *v,
                  double *f, uint8_t *alive) {
    or_model md = {dim, law, stretch, n, row_ptr, col, X, V, c, s_c, beta, 0.0, 0.0, 0, pv_h, pv_R,
                   j_c1, j_c2, j_delta};
    or_central_core(&md, rho, bc_kind, bc_vel, b, ramp, dt, step0, nsteps, u, v, f, alive);
}

void or_verlet(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
               const double *X, const double *V, double rho, double c, double s_c,
               const uint8_t *bc_kind, const double *bc_vel, const double *b,
               int64_t ramp, double dt, int64_t step0, int64_t nsteps,
               double *u, double *v, double *f, uint8_t *alive) {
    or_verlet_law(dim, n, row_ptr, col, X, V, rho, c, s_c, 0, 0.0, 0, bc_kind, bc_vel, b, ramp,
                  dt, step0, nsteps, u, v, f, alive);
}

/* ------------------------------------------------------------------------ */
/* Tangent operator.  For the linearised law f is linear in u, so the       */
/* central difference of the paper's tangent equation is exact and the     */
/* operator is H = -V (x) df/du:                                             */
/*   y_i = -V_i sum_j c ((w_j - w_i) . xi / |xi|^2) (xi/|xi|) V_j  (free i)  */
/*   y_i = w_i                                                  (fixed i)   */
/* with w_j read as 0 at fixed nodes.  H is symmetric, and positive definite */
/* when the fixed set removes the rigid motions.                             */
/* ------------------------------------------------------------------------ */
void or_apply_tangent(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const double *X, const double *V, double c, const uint8_t *alive,
                      const uint8_t *fixed, const double *w, double *y) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (fixed && fixed[i]) {
            for (int k = 0; k < dim; ++k) y[i * dim + k] = w[i * dim + k];
            continue;
        }
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            int jfix = fixed ? fixed[j] : 0;
            double xi[3] = {0, 0, 0}, dw[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                xi[k] = X[j * dim + k] - X[i * dim + k];
                dw[k] = (jfix ? 0.0 : w[j * dim + k]) - w[i * dim + k];
            }
            double r2 = 0.0, ex = 0.0;
            for (int k = 0; k < dim; ++k) {
                r2 = r2 + xi[k] * xi[k];
                ex = ex + dw[k] * xi[k];
            }
            double S = ex / r2;
            double r = sqrt(r2);
            for (int k = 0; k < dim; ++k) acc[k] = acc[k] + c * S * (xi[k] / r) * V[j];
        }
        for (int k = 0; k < dim; ++k) y[i * dim + k] = -V[i] * acc[k];
    }
}

static double or_dot(int64_t m, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t q = 0; q < m; ++q) s = s + a[q] * b[q];
    return s;
}

/*
 * Conjugate gradients (Hestenes-Stiefel) on H x = rhs, from the x given.
 * Stops when ||rhs - H x|| <= rtol ||rhs||.  Returns 0 on convergence, 1 if
 * maxit was reached.
 */
int or_cg(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
          const double *V, double c, const uint8_t *alive, const uint8_t *fixed,
          const double *rhs, double *x, double rtol, int maxit, int *iters, double *relres) {
    int64_t m = n * dim;
    double *r = (double *)malloc(sizeof(double) * m);
    double *p = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    or_apply_tangent(dim, n, row_ptr, col, X, V, c, alive, fixed, x, q);
    for (int64_t k = 0; k < m; ++k) { r[k] = rhs[k] - q[k]; p[k] = r[k]; }
    double bnorm = sqrt(or_dot(m, rhs, rhs));
    if (bnorm == 0.0) bnorm = 1.0;
    double rr = or_dot(m, r, r);
    int it = 0, status = 1;
    while (1) {
        if (sqrt(rr) <= rtol * bnorm) { status = 0; break; }
        if (it >= maxit) break;
        or_apply_tangent(dim, n, row_ptr, col, X, V, c, alive, fixed, p, q);
        double alpha = rr / or_dot(m, p, q);
        for (int64_t k = 0; k < m; ++k) { x[k] = x[k] + alpha * p[k]; r[k] = r[k] - alpha * q[k]; }
        double rr_new = or_dot(m, r, r);
        double beta = rr_new / rr;
        rr = rr_new;
        for (int64_t k = 0; k < m; ++k) p[k] = r[k] + beta * p[k];
        ++it;
    }
    if (iters) *iters = it;
    if (relres) *relres = sqrt(rr) / bnorm;
    free(r); free(p); free(q);
    return status;
}

/*
 * Residual of the quasi-static problem (the paper's residual equation, read
 * per node and scaled by the nodal volume): r_i = V_i (f_i(u) + b_i) on free
 * nodes, 0 on fixed nodes.  Returns ||r||_2.
 */
double or_residual(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const double *X, const double *V, double c, const uint8_t *alive,
                   const uint8_t *fixed, const double *b, const double *u, double *r) {
    or_force(dim, n, row_ptr, col, X, V, u, c, 0.0, (uint8_t *)alive, r, NULL);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            int64_t q = i * dim + k;
            if (fixed && fixed[i]) r[q] = 0.0;
            else r[q] = V[i] * (r[q] + (b ? b[q] : 0.0));
            s = s + r[q] * r[q];
        }
    return sqrt(s);
}

/*
 * Newton iteration of the paper's implicit scheme (flow chart of Section
 * "Implicit time integration"): while ||r|| > rtol ||V b|| solve
 * H du = r and set u <- u + du.  For the linearised law one step suffices up
 * to the inner tolerance.  u holds the fixed values on entry.  Returns 0 on
 * convergence, 1 otherwise.
 */
int or_solve_implicit(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const double *X, const double *V, double c, const uint8_t *alive,
                      const uint8_t *fixed, const double *b, double *u, double rtol,
                      double inner_rtol, int maxit, int max_outer, int *outer,
                      int *inner, double *relres) {
    int64_t m = n * dim;
    double *r = (double *)malloc(sizeof(double) * m);
    double *du = (double *)malloc(sizeof(double) * m);
    double bn = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            double t = (fixed && fixed[i]) ? 0.0 : V[i] * (b ? b[i * dim + k] : 0.0);
            bn = bn + t * t;
        }
    bn = sqrt(bn);
    if (bn == 0.0) bn = 1.0;
    int it_out = 0, it_in = 0, status = 1;
    double rel = 0.0;
    while (1) {
        rel = or_residual(dim, n, row_ptr, col, X, V, c, alive, fixed, b, u, r) / bn;
        if (rel <= rtol) { status = 0; break; }
        if (it_out >= max_outer) break;
        memset(du, 0, sizeof(double) * m);
        int k = 0;
        double rr = 0.0;
        or_cg(dim, n, row_ptr, col, X, V, c, alive, fixed, r, du, inner_rtol, maxit, &k, &rr);
        it_in += k;
        for (int64_t q = 0; q < m; ++q) u[q] = u[q] + du[q];
        ++it_out;
    }
    if (outer) *outer = it_out;
    if (inner) *inner = it_in;
    if (relres) *relres = rel;
    free(r); free(du);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Classical continuum mechanics comparisons of the implicit validation      */
/* (Section "Validation", implicit).  One dimension: a bar of cross section */
/* A and Young's modulus E under an end force F carries the uniform stress  */
/* F/A, the strain F/(A E) and the strain-energy density stress*strain/2.   */
/* out = {stress, strain, energy density}.                                   */
/* ------------------------------------------------------------------------ */
void or_ccm_bar_1d(double F, double A, double E, double *out) {
    const double stress = F / A;
    const double strain = stress / E;
    out[0] = stress;
    out[1] = strain;
    out[2] = 0.5 * stress * strain;
}

/* Two dimensions, plane stress: a plate under a uniform traction t along x, */
/* held at x = x0 in x and symmetric about y = yc, has the uniform strains   */
/* eps_xx = t/E, eps_yy = -nu t/E, no shear, hence the displacement          */
/*   u_x = (t/E)(x - x0),  u_y = -nu (t/E)(y - yc)                           */
/* at the nodes X (n x 2); u is n x 2.                                       */
void or_ccm_plane_stress(int64_t n, const double *X, double t, double E, double nu, double x0,
                         double yc, double *u) {
    const double e = t / E;
    for (int64_t i = 0; i < n; ++i) {
        u[2 * i] = e * (X[2 * i] - x0);
        u[2 * i + 1] = -nu * e * (X[2 * i + 1] - yc);
    }
}

/* ------------------------------------------------------------------------ */
/* General pairwise law of Algorithm 1 (the NP model of the validation       */
/* section): with J = 1 on the ball,                                         */
/*   f_i += 4/(delta |B_delta(0)|) psi'(|xi| S^2) S e V_j                    */
/*   U_i += 1/(delta |B_delta(0)|) psi(|xi| S^2) V_j                         */
/* and the NP potential psi(r) = C (1 - exp(-beta r)), psi'(0) = C beta.     */
/* Written with the micromodulus c = 4 psi'(0)/(delta |B_delta(0)|):         */
/*   f_i += c exp(-beta r) S e V_j,  U_i += c/(4 beta) (1 - exp(-beta r)) V_j */
/* (1 - exp(-beta r) evaluated as -expm1(-beta r), free of cancellation).   */
/* with r = |xi| S^2.  law 0 is the linearised law (psi' = psi'(0), the      */
/* exponential factor 1 and the energy (c/4) r V_j); law 1 is NP.            */
/* stretch 0: S = eta.xi/|xi|^2 and e = xi/|xi| (Algorithm 1); stretch 1:    */
/* the exact stretch S = (|xi+eta| - |xi|)/|xi| acting along the deformed    */
/* bond, e = (xi+eta)/|xi+eta| (the PMB form the paper names).               */
/* Damage as in or_force: with alive given and s_c > 0 a live bond with      */
/* S > s_c breaks before it contributes.                                     */
/* ------------------------------------------------------------------------ */
/* Partial volume of a bond (the correction the paper names without a       */
/* formula; read here as the partial-area rule): with the neighbour list     */
/* built at radius R = delta + h/2, V_j is scaled by                          */
/* min(1, max(0, (R - |xi|)/h)) -- 1 inside delta - h/2, falling linearly to  */
/* 0 at delta + h/2.  h <= 0: no correction (factor exactly 1).               */
static double or_pv(double len, double R, double h) {
    if (!(h > 0.0)) return 1.0;
    double w = (R - len) / h;
    return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}

void or_force_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *X, const double *V, const double *u, double c, double s_c,
                  int law, double beta, int stretch, uint8_t *alive, double *f, double *U) {
    or_force_law_pv(dim, n, row_ptr, col, X, V, u, c, s_c, law, beta, stretch, 0.0, 0.0, alive,
                    f, U);
}

void or_force_law_pv(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *X, const double *V, const double *u, double c, double s_c,
                     int law, double beta, int stretch, double pv_h, double pv_R,
                     uint8_t *alive, double *f, double *U) {
    or_force_law_j(dim, n, row_ptr, col, X, V, u, c, s_c, law, beta, stretch, pv_h, pv_R, 0.0,
                   0.0, 0.0, alive, f, U);
}

/* Influence function of the 1-d validation (Section "One dimensional" of   */
/* the explicit-scheme validation): J(r) = c1 r exp(-r^2 / c2) at           */
/* r = |xi|/delta, multiplying the bond's force and energy; c2 <= 0: J = 1  */
/* (the 2-d validation's choice on the ball).                               */
static double or_influence(double len, double delta, double c1, double c2) {
    if (!(c2 > 0.0)) return 1.0;
    double r = len / delta;
    return c1 * r * exp(-(r * r) / c2);
}

void or_force_law_j(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *X, const double *V, const double *u, double c, double s_c,
                    int law, double beta, int stretch, double pv_h, double pv_R, double j_c1,
                    double j_c2, double j_delta, uint8_t *alive, double *f, double *U) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        double Ui = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            double xi[3] = {0, 0, 0}, eta[3] = {0, 0, 0}, y[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                xi[k] = X[j * dim + k] - X[i * dim + k];
                eta[k] = u[j * dim + k] - u[i * dim + k];
                y[k] = xi[k] + eta[k];
            }
            double r2 = 0.0, ex = 0.0, y2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                r2 = r2 + xi[k] * xi[k];
                ex = ex + eta[k] * xi[k];
                y2 = y2 + y[k] * y[k];
            }
            double len = sqrt(r2);
            double S, e[3] = {0, 0, 0};
            if (stretch == 0) {
                S = ex / r2;
                for (int k = 0; k < dim; ++k) e[k] = xi[k] / len;
            } else {
                double ylen = sqrt(y2);
                S = (ylen - len) / len;
                for (int k = 0; k < dim; ++k) e[k] = y[k] / ylen;
            }
            if (alive && s_c > 0.0 && S > s_c) {
                alive[p] = 0;
                continue;
            }
            double r = len * S * S;
            double phi = law == 1 ? exp(-beta * r) : 1.0;
            double Vj = V[j] * or_pv(len, pv_R, pv_h) * or_influence(len, j_delta, j_c1, j_c2);
            for (int k = 0; k < dim; ++k) fi[k] = fi[k] + c * phi * S * e[k] * Vj;
            if (U) {
                double psi = law == 1 ? -expm1(-beta * r) / beta : r;
                Ui = Ui + 0.25 * c * psi * Vj;
            }
        }
        for (int k = 0; k < dim; ++k) f[i * dim + k] = fi[k];
        if (U) U[i] = Ui;
    }
}

/* Tangent of the linearised-stretch law at the displacement ulin:          */
/* d/d eta [psi'(|xi| S^2) S] = (psi'(r) + 2 r psi''(r)) dS/d eta with      */
/* dS/d eta = xi/|xi|^2, so each bond acts with the stiffness               */
/*   k = c exp(-beta r) (1 - 2 beta r)   (NP),   k = c   (linear),          */
/* r = |xi| S(ulin)^2, and H = -V (x) df/du applies as                      */
/*   y_i = -V_i sum_j k ((w_j - w_i).xi/|xi|^2) (xi/|xi|) V_j   (free i)    */
/*   y_i = w_i   (fixed i), w_j read as 0 at fixed j.                       */
void or_tangent_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *X, const double *V, double c, int law, double beta,
                    const double *ulin, const uint8_t *alive, const uint8_t *fixed,
                    const double *w, double *y) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (fixed && fixed[i]) {
            for (int k = 0; k < dim; ++k) y[i * dim + k] = w[i * dim + k];
            continue;
        }
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            int jfix = fixed ? fixed[j] : 0;
            double xi[3] = {0, 0, 0}, dw[3] = {0, 0, 0}, eta[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                xi[k] = X[j * dim + k] - X[i * dim + k];
                dw[k] = (jfix ? 0.0 : w[j * dim + k]) - w[i * dim + k];
                eta[k] = ulin ? ulin[j * dim + k] - ulin[i * dim + k] : 0.0;
            }
            double r2 = 0.0, ew = 0.0, eu = 0.0;
            for (int k = 0; k < dim; ++k) {
                r2 = r2 + xi[k] * xi[k];
                ew = ew + dw[k] * xi[k];
                eu = eu + eta[k] * xi[k];
            }
            double len = sqrt(r2);
            double Su = eu / r2;
            double r = len * Su * Su;
            double kb = law == 1 ? c * exp(-beta * r) * (1.0 - 2.0 * beta * r) : c;
            double Sw = ew / r2;
            for (int k = 0; k < dim; ++k) acc[k] = acc[k] + kb * Sw * (xi[k] / len) * V[j];
        }
        for (int k = 0; k < dim; ++k) y[i * dim + k] = -V[i] * acc[k];
    }
}

/* Residual r_i = V_i (f_i(u) + b_i) on free nodes (0 on fixed), for a law. */
double or_residual_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                       const double *X, const double *V, double c, int law, double beta,
                       const uint8_t *alive, const uint8_t *fixed, const double *b,
                       const double *u, double *r) {
    or_force_law(dim, n, row_ptr, col, X, V, u, c, 0.0, law, beta, 0, (uint8_t *)alive, r,
                 NULL);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            int64_t q = i * dim + k;
            if (fixed && fixed[i]) r[q] = 0.0;
            else r[q] = V[i] * (r[q] + (b ? b[q] : 0.0));
            s = s + r[q] * r[q];
        }
    return sqrt(s);
}

/* Newton's method of the implicit flow chart for a law: while              */
/* ||r(u)|| > rtol ||V b||, solve H(u) du = r(u) by conjugate gradients      */
/* (to inner_rtol relative) and set u <- u + du.  H(u) is the tangent at the */
/* current iterate (symmetric; positive definite on the free DOFs while     */
/* every bond has 2 beta r < 1).  Returns 0 on convergence, 1 otherwise.     */
int or_solve_law(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                 const double *X, const double *V, double c, int law, double beta,
                 const uint8_t *alive, const uint8_t *fixed, const double *b, double *u,
                 double rtol, double inner_rtol, int maxit, int max_outer, int *outer,
                 int *inner, double *relres) {
    int64_t m = n * dim;
    double *r = (double *)malloc(sizeof(double) * m);
    double *du = (double *)malloc(sizeof(double) * m);
    double *res = (double *)malloc(sizeof(double) * m);
    double *p = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    double bn = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            double t = (fixed && fixed[i]) ? 0.0 : V[i] * (b ? b[i * dim + k] : 0.0);
            bn = bn + t * t;
        }
    bn = sqrt(bn);
    if (bn == 0.0) bn = 1.0;
    int it_out = 0, it_in = 0, status = 1;
    double rel = 0.0;
    while (1) {
        rel = or_residual_law(dim, n, row_ptr, col, X, V, c, law, beta, alive, fixed, b, u, r) / bn;
        if (rel <= rtol) { status = 0; break; }
        if (it_out >= max_outer) break;
        /* conjugate gradients on H(u) du = r from du = 0 */
        double rn = sqrt(or_dot(m, r, r));
        for (int64_t k = 0; k < m; ++k) { du[k] = 0.0; res[k] = r[k]; p[k] = r[k]; }
        double rr = or_dot(m, res, res);
        int it = 0;
        while (sqrt(rr) > inner_rtol * rn && it < maxit) {
            or_tangent_law(dim, n, row_ptr, col, X, V, c, law, beta, u, alive, fixed, p, q);
            double alpha = rr / or_dot(m, p, q);
            for (int64_t k = 0; k < m; ++k) { du[k] = du[k] + alpha * p[k]; res[k] = res[k] - alpha * q[k]; }
            double rr_new = or_dot(m, res, res);
            double beta_cg = rr_new / rr;
            rr = rr_new;
            for (int64_t k = 0; k < m; ++k) p[k] = res[k] + beta_cg * p[k];
            ++it;
        }
        it_in += it;
        for (int64_t k = 0; k < m; ++k) u[k] = u[k] + du[k];
        ++it_out;
    }
    if (outer) *outer = it_out;
    if (inner) *inner = it_in;
    if (relres) *relres = rel;
    free(r); free(du); free(res); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Linear peridynamic solid, Algorithm 2 (3-d, influence function 1), with  */
/* the bulk and shear moduli K and mu:                                       */
/*   m_i     = sum_j |xi|^2 V_j                       (weighted volume)     */
/*   e       = |xi + eta| - |xi|                      (extension)           */
/*   theta_i = (3/m_i) sum_j |xi| e V_j               (dilatation)          */
/*   e^d     = e - theta_i |xi|/3                                           */
/*   t       = (3/m_i) K theta_i |xi| + (15 mu/m_i) e^d                     */
/*   M       = (xi + eta)/|xi + eta|                                        */
/*   f_i += t M V_j  and  f_j -= t M V_i   over every bond (i, j) of i      */
/* The force loop is the paper's scatter, run sequentially.  The strain     */
/* energy density (the paper's energy line is garbled; this is the LPS      */
/* energy of the cited state-based theory, of which t is the derivative):   */
/*   W_i = (K/2) theta_i^2 + (15 mu/(2 m_i)) sum_j (e^d)^2 V_j              */
/* Bonds with alive[p] == 0 are left out of every sum.  A node without      */
/* bonds has m = theta = 0 and no force.  Any output may be NULL.           */
/* ------------------------------------------------------------------------ */
void or_lps(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
            const double *V, const double *u, double K, double mu, const uint8_t *alive,
            double *m_out, double *theta_out, double *f, double *W) {
    or_lps_pv(n, row_ptr, col, X, V, u, K, mu, 0.0, 0.0, alive, m_out, theta_out, f, W);
}

/* or_lps with partial volumes: every V_j (and the V_i of the scatter to j) */
/* of a bond is scaled by or_pv(|xi|).                                      */
void or_lps_pv(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
               const double *V, const double *u, double K, double mu, double pv_h, double pv_R,
               const uint8_t *alive, double *m_out, double *theta_out, double *f, double *W) {
    double *m = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *th = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double mi = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x = X[j * 3 + k] - X[i * 3 + k];
                r2 = r2 + x * x;
            }
            mi = mi + r2 * (V[j] * or_pv(sqrt(r2), pv_R, pv_h));
        }
        m[i] = mi;
    }
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (alive && !alive[p]) continue;
            int64_t j = col[p];
            double r2 = 0.0, y2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x = X[j * 3 + k] - X[i * 3 + k];
                double y = x + (u[j * 3 + k] - u[i * 3 + k]);
                r2 = r2 + x * x;
                y2 = y2 + y * y;
            }
            double len = sqrt(r2);
            double e = sqrt(y2) - len;
            s = s + len * e * (V[j] * or_pv(len, pv_R, pv_h));
        }
        th[i] = m[i] > 0.0 ? 3.0 / m[i] * s : 0.0;
    }
    if (f) {
        for (int64_t q = 0; q < 3 * n; ++q) f[q] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!(m[i] > 0.0)) continue;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                if (alive && !alive[p]) continue;
                int64_t j = col[p];
                double xi[3], y[3], r2 = 0.0, y2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    xi[k] = X[j * 3 + k] - X[i * 3 + k];
                    y[k] = xi[k] + (u[j * 3 + k] - u[i * 3 + k]);
                    r2 = r2 + xi[k] * xi[k];
                    y2 = y2 + y[k] * y[k];
                }
                double len = sqrt(r2), ylen = sqrt(y2);
                double e = ylen - len;
                double ed = e - th[i] * len / 3.0;
                double t = 3.0 / m[i] * K * th[i] * len + 15.0 * mu / m[i] * ed;
                double w = or_pv(len, pv_R, pv_h);
                for (int k = 0; k < 3; ++k) {
                    double Mk = y[k] / ylen;
                    f[i * 3 + k] = f[i * 3 + k] + t * Mk * (V[j] * w);
                    f[j * 3 + k] = f[j * 3 + k] - t * Mk * (V[i] * w);
                }
            }
        }
    }
    if (W) {
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                if (alive && !alive[p]) continue;
                int64_t j = col[p];
                double r2 = 0.0, y2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double x = X[j * 3 + k] - X[i * 3 + k];
                    double y = x + (u[j * 3 + k] - u[i * 3 + k]);
                    r2 = r2 + x * x;
                    y2 = y2 + y * y;
                }
                double len = sqrt(r2);
                double ed = (sqrt(y2) - len) - th[i] * len / 3.0;
                s = s + ed * ed * (V[j] * or_pv(len, pv_R, pv_h));
            }
            W[i] = m[i] > 0.0 ? 0.5 * K * th[i] * th[i] + 15.0 * mu / (2.0 * m[i]) * s : 0.0;
        }
    }
    if (m_out) for (int64_t i = 0; i < n; ++i) m_out[i] = m[i];
    if (theta_out) for (int64_t i = 0; i < n; ++i) theta_out[i] = th[i];
    free(m);
    free(th);
}

/* ------------------------------------------------------------------------ */
/* Test bookkeeping for the damage comparison: band[p] |= 1 where bond p's   */
/* linearised strain S = (eta . xi)/|xi|^2 (Algorithm 1) lies within a       */
/* relative distance tol of the critical stretch, |S/s_c - 1| <= tol.  Bonds  */
/* in this band may break on one side and not on the other when the two     */
/* sides round S differently; every other flag must agree.                   */
/* ------------------------------------------------------------------------ */
void or_band_update(int dim, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *X, const double *u, double s_c, double tol, double tol_eta,
                    uint8_t *band) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col[p];
            double r2 = 0.0, ex = 0.0, e2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                double x = X[j * dim + k] - X[i * dim + k];
                double e = u[j * dim + k] - u[i * dim + k];
                r2 = r2 + x * x;
                ex = ex + e * x;
                e2 = e2 + e * e;
            }
            double S = ex / r2;
            if (fabs(S / s_c - 1.0) <= tol || fabs(S - s_c) <= tol_eta * sqrt(e2 / r2))
                band[p] = 1;
        }
    }
}

/* threads of the OpenMP loops (timing only: results do not depend on it) */
void or_set_threads(int k) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
