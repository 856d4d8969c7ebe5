/*
 * pd.h -- C ABI of the MI355X (gfx950) peridynamics hot-path library.
 *
 * The library computes the bond-based peridynamic model of Diehl, Jha,
 * Kaiser, Lipton and Levesque (arXiv:1806.06917):
 *   - discrete horizon B_delta(X_i) = {X_j : |X_j - X_i| <= delta}
 *     (Section "Discretization of peridynamics equations");
 *   - internal force density of the linearised bond law (Algorithm 1 with
 *     influence function J = 1 and psi' = psi'(0), the "LP" model of the
 *     2-d explicit validation): f_i = sum_j mu_ij c S_ij (xi/|xi|) V_j,
 *     S_ij = (u_j - u_i).xi/|xi|^2, xi = X_j - X_i,
 *     c = 4 psi'(0)/(delta |B_delta(0)|);
 *   - critical-stretch bond damage (the PMB model named with Algorithm 1):
 *     mu_ij drops to 0, irreversibly, at the first force evaluation with
 *     S_ij > s_c;
 *   - velocity-Verlet time stepping (Section "Explicit time integration");
 *   - the tangent operator of the quasi-static problem applied matrix-free,
 *     and its solution by conjugate gradients (Section "Implicit time
 *     integration").
 *
 * Conventions for every entry point:
 *   - Return value: PD_OK (0) or a negative PD_E* status.  Nothing throws
 *     across the ABI.  A message for the last failure on a context is
 *     available from pd_last_error(ctx) (per context; not thread-safe for
 *     concurrent callers on one context).
 *   - Arguments are validated before any launch; on a validation error no
 *     output is touched.
 *   - "device" pointers are GPU memory of the context's device (for example
 *     the data_ptr() of torch tensors), "host" pointers are CPU memory.
 *     The caller owns every pointer it passes; the library owns its handles
 *     and everything inside them and frees them in the *_destroy calls.
 *   - Nodal arrays are dense row-major [n][dim] float64 (x, y[, z]) in the
 *     caller's node numbering ("original order").  Bond arrays (alive flags)
 *     are in the "exported bond order": rows by ascending node id, within a
 *     row by ascending neighbour id, exactly the CSR that pd_nbr_export
 *     returns.  The library's internal space-filling-curve order is never
 *     exposed.
 *   - All work is enqueued on the context's stream in order.  Calls return
 *     before the GPU finishes except pd_build_neighbors, pd_nbr_info,
 *     pd_nbr_export, pd_sim_get and pd_solve_implicit, which synchronise the
 *     stream.  Handles built on one context must only be used with it.
 *   - A pd_nbr must outlive every pd_sim created from it.
 *   - Device memory the library frees is kept in a per-device cache (at most
 *     16 GiB) and handed out again to later allocations of the library once
 *     the work queued before the free has completed; it goes back to the
 *     driver when an allocation fails, or at process exit.
 */
#ifndef PD_H
#define PD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PD_OK = 0,
    PD_EINVAL = -1,      /* invalid argument (shape, value, null pointer, coincident nodes) */
    PD_ENOMEM = -2,      /* device allocation failed */
    PD_EDEVICE = -3,     /* HIP runtime or kernel error; the context stays failed */
    PD_ENOCONV = -4,     /* iterative solve reached its limit; info and u hold the last iterate */
    PD_ENONFINITE = -5,  /* a non-finite displacement or velocity was produced */
    PD_ECAPACITY = -6    /* problem exceeds a documented size limit */
};

enum { PD_FP64 = 0, PD_MIXED = 1, PD_FP32 = 2 };

enum { PD_BC_FREE = 0, PD_BC_CLAMPED = 1, PD_BC_VELOCITY = 2 };

typedef struct pd_ctx_s *pd_ctx;
typedef struct pd_nbr_s *pd_nbr;
typedef struct pd_sim_s *pd_sim;
typedef struct pd_batch_s *pd_batch;
typedef struct pd_server_s *pd_server;

/*
 * Material and arithmetic of one model.
 *   dim        2 or 3
 *   precision  PD_FP64: every bond computed in float64, 1/|xi| to full
 *              double precision.
 *              PD_MIXED: the same float64 arithmetic, except that 1/|xi| is
 *              the hardware reciprocal-square-root estimate without
 *              refinement (relative error below 2^-22).  Positions,
 *              velocities, sums and the time integration are float64 in
 *              both modes.
 *              PD_FP32 (PD_LAW_LINEAR with the linearised stretch only;
 *              other laws return PD_EINVAL): the differences xi and eta are
 *              taken in float64 and rounded to float32; |xi|^-1 (hardware
 *              float32 estimate), S, the damage test against s_c rounded to
 *              float32, and the bond force are float32; the force terms
 *              of a lane's bonds are added two at a time in float32 and
 *              each pair sum goes into a compensated float32 pair
 *              (TwoSum), converted to float64 at the end.  Positions, velocities and the time integration
 *              stay float64.  Force relative error about 1e-6 of the
 *              largest bond force.  pd_apply_tangent rejects it;
 *              pd_solve_implicit treats it as PD_MIXED.
 *   c          micromodulus c = 4 psi'(0)/(delta |B_delta(0)|) (Algorithm 1);
 *              see pd_micromodulus.
 *   rho        mass density (velocity-Verlet equations), > 0
 *   s_c        critical stretch; <= 0 disables damage
 *   law        pairwise potential psi of Algorithm 1 (J = 1 on the ball):
 *              PD_LAW_LINEAR  psi'(|xi| S^2) taken as psi'(0): bond force
 *                             c S e V_j, energy (c/4) |xi| S^2 V_j;
 *              PD_LAW_NP      psi(r) = C (1 - exp(-beta r)) (the nonlinear
 *                             model of the paper's validation section):
 *                             bond force c exp(-beta r) S e V_j, energy
 *                             c/(4 beta) (1 - exp(-beta r)) V_j, r = |xi| S^2
 *                             (C enters through c = 4 C beta/(delta|B|)).
 *   stretch    PD_STRETCH_LINEARISED  S = eta.xi/|xi|^2, e = xi/|xi|
 *                             (Algorithm 1);
 *              PD_STRETCH_EXACT  S = (|xi+eta| - |xi|)/|xi| along the
 *                             deformed bond, e = (xi+eta)/|xi+eta|.
 *   beta       PD_LAW_NP only: beta > 0.
 *   law = PD_LAW_LPS  the linear peridynamic solid of Algorithm 2 (dim 3,
 *              influence function 1, bulk modulus `bulk` > 0 and shear
 *              modulus `shear` >= 0; c, beta and stretch are not used).  Per
 *              node m_i = sum |xi|^2 V_j and theta_i = (3/m_i) sum |xi| e V_j
 *              with the extension e = |xi+eta| - |xi|; the bond force state
 *              t = (3/m_i) K theta_i |xi| + (15 mu/m_i)(e - theta_i |xi|/3)
 *              along M = (xi+eta)/|xi+eta|, summed as the gather
 *              f_i = sum_j (t_ij + t_ji) M V_j (the paper's scatter read from
 *              node i; it needs symmetric bond flags, as cut and damage
 *              flags are); energy W_i = (K/2) theta_i^2 +
 *              (15 mu/(2 m_i)) sum (e - theta_i |xi|/3)^2 V_j.  No damage
 *              (s_c must be <= 0), no tangent or implicit solve.  Both
 *              kernels evaluate t through the per-node coefficients
 *              3 K theta/m, 15 mu/m and theta/3.
 *   pv_h       partial volumes (the correction the paper names without a
 *              formula; read as the partial-area rule): with pv_h = h > 0 and
 *              the neighbour list built at radius R = delta + h/2, each
 *              bond's V_j (and in the solid also m, theta and the energy) is
 *              scaled by min(1, max(0, (R - |xi|)/h)).  0 = off.  Gather
 *              kernel only; not for the tangent or the implicit solve.
 *   j_c1, j_c2 influence function of a pairwise law (the 1-d validation
 *              of the explicit scheme): with j_c2 > 0 each bond's force and
 *              energy carry J = j_c1 r exp(-r^2/j_c2) at r = |xi|/delta,
 *              delta being the neighbour list's radius minus pv_h/2.
 *              j_c2 = 0: J = 1 (j_c1 unused).  Not for the solid; gather
 *              kernel only; not for the tangent or the implicit solve.
 * A zero-filled law/stretch/beta is the linearised law of Algorithm 1.  The
 * tiled kernels run that law, and the streamed step kernel also the NP law
 * with the linearised stretch and no damage, and the solid's explicit steps
 * without partial volumes (a state pass and a force pass per step, single
 * simulations only: pd_batch_step rejects them); the other calls of such
 * simulations, and every other combination, run on the gather kernel
 * (pd_sim_info kernel 1).  The tangent and the implicit solve take the
 * linearised stretch of a pairwise law only (PD_EINVAL otherwise).
 */
enum { PD_LAW_LINEAR = 0, PD_LAW_NP = 1, PD_LAW_LPS = 2 };
enum { PD_STRETCH_LINEARISED = 0, PD_STRETCH_EXACT = 1 };

typedef struct {
    int dim;
    int precision;
    double c;
    double rho;
    double s_c;
    int law;
    int stretch;
    double beta;
    double bulk;
    double shear;
    double pv_h;
    double j_c1;
    double j_c2;
} pd_material;

typedef struct {
    int outer_iters;      /* Newton / iterative-refinement steps taken */
    int inner_iters;      /* total conjugate-gradient iterations */
    double rel_residual;  /* ||V (f(u) + b)||_2 / ||V b||_2 over free nodes, in float64 */
} pd_solve_info;

/* Library version (major*10000 + minor*100 + patch). */
int pd_version(void);

/* Static text for a status code. */
const char *pd_status_string(int status);

/*
 * Micromodulus of the linearised bond law, c = 4 psi'(0)/(delta |B_delta|)
 * (Algorithm 1), calibrated so that under a uniform isotropic strain the
 * peridynamic strain-energy density equals the classical one with the
 * Poisson ratio fixed by the bond-based model (Section "Peridynamics
 * theory"): 2-d plane stress nu = 1/3 gives c = 9E/(pi delta^3); 3-d
 * nu = 1/4 gives c = 12E/(pi delta^4).  Host only; returns NaN for
 * dim not in {2, 3}.
 */
double pd_micromodulus(int dim, double E, double delta);

/*
 * Create a context on HIP device `device`.  `hip_stream` is a borrowed
 * hipStream_t (NULL = the null stream); it must outlive the context.
 * Returns PD_EDEVICE when no such device exists.
 */
int pd_ctx_create(int device, void *hip_stream, pd_ctx *out);
/*
 * Synchronises the stream and releases the context.  If neighbour lists or
 * simulations created on it are still alive, its memory is kept until the
 * last of them is destroyed, and every later call that takes this context
 * (directly or through those handles) fails with PD_EINVAL; destroying
 * them stays valid.  A second destroy returns PD_EINVAL.
 */
int pd_ctx_destroy(pd_ctx ctx);
const char *pd_last_error(pd_ctx ctx);

/*
 * Tuning: lanes of a wavefront that share one node's bond sum (1, 2, 4, 8,
 * 16, 32 or 64); 0 restores the automatic choice from the mean row length.
 * The per-node summation order, and hence the float rounding, depends on
 * this value only.
 */
int pd_ctx_set_lanes(pd_ctx ctx, int lanes);

/*
 * Tuning of the node kernels (results do not depend on it):
 *   kernel  0 automatic, 1 plain gather from global memory, 2 LDS-staged
 *           tiles (T consecutive nodes in the internal order share one
 *           workgroup, which copies the records of every node their bonds
 *           touch into LDS once per launch), 3 streamed tiles for the
 *           explicit steps (the same tiles, staged by asynchronous
 *           global-to-LDS copies that overlap the bond sums; needs equal
 *           nodal volumes, other calls of such a simulation use kind 2, or
 *           kind 1 where the tile kernel cannot be resident at that shape);
 *           automatic uses streamed tiles for the steps where they apply,
 *           LDS tiles elsewhere whenever the largest halo fits in LDS.
 *   tile    nodes per tile, a multiple of 16 in [16, 4096]; 0 automatic.
 *   block   threads per tile workgroup, a multiple of 64 in [64, 1024];
 *           0 automatic.
 * Takes effect for neighbour lists and simulations set up afterwards.
 */
int pd_ctx_set_tuning(pd_ctx ctx, int kernel, int tile, int block);

/*
 * Autotuner for the explicit step (launch-shape search; the method's
 * arithmetic is unchanged, only the order of each node's bond sum).
 *
 * pd_autotune builds the neighbour list of (X, V, delta) -- device arrays as
 * in pd_build_neighbors -- and, for each candidate tile size x lanes per node
 * (T * lanes in [256, 1024]: 32x8, 32x16, 64x4, 64x8, 64x16, 128x2, 128x4,
 * 128x8, 192x4, 240x4, 256x2, 256x4), creates a simulation at rest with damage on, runs 2
 * warm-up steps and times `steps` explicit steps (pd_verlet_step) with HIP
 * events on the context's stream.  The fastest is cached in the context
 * under (dim, mean-neighbour-count bucket, precision), the buckets split
 * at 8, 20, 36, 64, 96, 176, 384 and 768 neighbours per node;
 * from then on pd_sim_create uses it for meshes of that bucket whenever the
 * context's lanes and tuning are automatic (0).  The search synchronises and
 * restores the context's tuning.
 *   table, table_cap, ntable  optional: every candidate in the order above
 *     (us_per_step < 0: the tile size does not fit this mesh);
 *   best  the winner.
 * PD_ECAPACITY if no candidate fits; argument errors as in
 * pd_build_neighbors.
 * pd_tune_lookup: the cached choice for a (dim, mean neighbour count,
 *   precision); tile = lanes = 0 if there is none.
 * pd_tune_set installs a choice (e.g. one saved from an earlier search);
 *   (tile, lanes) must be a candidate above.  pd_tune_clear empties the cache.
 */
typedef struct {
    int tile;            /* nodes per tile */
    int lanes;           /* lanes per node */
    int kernel;          /* what ran: 3 streamed tiles, 2 LDS tiles, 1 none (did not fit) */
    double us_per_step;  /* measured microseconds per step, < 0 if not run */
} pd_tune_result;

int pd_autotune(pd_ctx ctx, int dim, int64_t n, const double *X, const double *V, double delta,
                int precision, int steps, pd_tune_result *table, int table_cap, int *ntable,
                pd_tune_result *best);
int pd_tune_lookup(pd_ctx ctx, int dim, double mean_neighbors, int precision,
                   pd_tune_result *out);
int pd_tune_set(pd_ctx ctx, int dim, double mean_neighbors, int precision, int tile, int lanes);
int pd_tune_clear(pd_ctx ctx);

/*
 * Build the neighbour lists B_delta(X_i) (Section "Discretization of
 * peridynamics equations") in the reference configuration, once.
 *   X      device, [n][dim] float64 reference coordinates
 *   delta  horizon, finite and > 0
 * Membership: j != i and d2 <= (delta*delta)*(1 + 1e-10), where
 * d2 = (dx*dx + dy*dy) + dz*dz with dx = X_j.x - X_i.x etc., each operation
 * separately rounded (no fused multiply-add), so the closed ball keeps the
 * lattice neighbours that sit exactly at distance delta.
 * Errors: PD_EINVAL for dim not in {2,3}, n <= 0, bad delta, non-finite X or
 * two coincident nodes; PD_ECAPACITY for more than 2^32 - 1 bonds, n >= 2^31
 * or a bounding box needing more than 2^27 bins of edge delta.
 * A mesh in which no two nodes lie within delta builds (nnz = 0), but the
 * calls that compute on it (pd_internal_force, pd_apply_tangent[_at],
 * pd_solve_implicit, pd_sim_create) reject it with PD_EINVAL: it has no
 * force, tangent or bond to evaluate.
 * Synchronises the stream.
 */
int pd_build_neighbors(pd_ctx ctx, int dim, int64_t n, const double *X, double delta,
                       pd_nbr *out);

/* nnz = number of directed bonds; max_row = longest row.  Either may be NULL. */
int pd_nbr_info(pd_nbr nbr, int64_t *nnz, int32_t *max_row);

/*
 * Copy the neighbour lists to the host in original numbering: row_ptr
 * (host, int64[n+1]) and col (host, int32[nnz]), rows ascending by node id,
 * neighbours ascending by id.  Either pointer may be NULL.
 */
int pd_nbr_export(pd_nbr nbr, int64_t *row_ptr, int32_t *col);

/* Host int32[n]: perm[k] = original id of the k-th node in the library's
 * internal space-filling-curve order (for diagnostics). */
int pd_nbr_permutation(pd_nbr nbr, int32_t *perm);

/* Synchronises the stream and releases the list; with simulations built on
 * it still alive, its memory goes with the last of them (which keep working).
 * A second destroy returns PD_EINVAL. */
int pd_nbr_destroy(pd_nbr nbr);

/*
 * One evaluation of the internal force density (Algorithm 1, linearised law)
 * at displacement u:
 *   X, V, u  device float64, [n][dim], [n], [n][dim]; X must be the array the
 *            neighbour lists were built from.
 *   alive    device uint8[nnz] in exported bond order, in/out, or NULL.
 *            NULL: every bond intact and no damage test.  Otherwise dead
 *            bonds (0) are skipped and, if mat->s_c > 0, every live bond with
 *            S > s_c is set to 0 before it contributes.
 *   f        device float64 [n][dim] output
 *   U        device float64 [n] output strain-energy density
 *            U_i = sum_j mu_ij (c/4) S_ij^2 |xi| V_j (Algorithm 1 with the
 *            linearised potential), or NULL.
 * Asynchronous.
 */
int pd_internal_force(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                      const double *V, const double *u, uint8_t *alive, double *f, double *U);

/*
 * pd_internal_force for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, results and errors, always on the
 * gather kernel, with its internal-order working copies (X, V, u, f, U, the
 * solid's per-node state, the bond flags) in a fixed device array of
 * PD_NOALLOC_MAX_BYTES bytes that the library holds on every device it runs
 * on until the process ends.  It calls no allocator.  A mesh whose working
 * copies exceed the array returns PD_ECAPACITY before any launch (the size
 * is about 8 (5 + 2 s) n + nnz bytes with s = 2 in 2-d and 4 in 3-d, plus
 * 16 n for the solid).
 * Every call on one device shares the array: calls that overlap on a device
 * (other streams, other contexts, other threads) race and must be ordered
 * by the caller.  Asynchronous on the context's stream.
 */
#define PD_NOALLOC_MAX_BYTES (64ll << 20)
int pd_internal_force_noalloc(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                              const double *V, const double *u, uint8_t *alive, double *f,
                              double *U);

/*
 * Create a resident explicit simulation (state kept on the GPU in internal
 * order).  Arrays are copied; the caller may free them afterwards.
 *   X, V        device reference coordinates and volumes (as for the nbr)
 *   u0, v0      device [n][dim] initial displacement and velocity (NULL = 0)
 *   bc_kind     device uint8[n]: PD_BC_FREE, PD_BC_CLAMPED (u = v = 0) or
 *               PD_BC_VELOCITY (prescribed velocity), NULL = all free
 *   bc_vel      device [n][dim] prescribed velocity of PD_BC_VELOCITY nodes
 *               (required when any such node exists)
 *   b           device [n][dim] body force density (constant in time), NULL = 0
 *   notch       host float64 [nseg][4] segments (ax, ay, bx, by), dim 2 only:
 *               a bond whose closed segment [X_i, X_j] meets a notch segment
 *               starts broken (orientation tests in float64 without fused
 *               multiply-add, end points taken in lexicographic order).
 *   ramp_steps  prescribed velocities are scaled by min(1, t/(ramp_steps dt));
 *               0 = no ramp.
 * The first force evaluation (and damage test) happens at the first step.
 */
int pd_sim_create(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                  const double *V, const double *u0, const double *v0, const uint8_t *bc_kind,
                  const double *bc_vel, const double *b, const double *notch, int nseg,
                  int64_t ramp_steps, pd_sim *out);

/*
 * Advance a simulation by nsteps velocity-Verlet steps of size dt (velocity
 * Verlet equations, boundary data at t^{k+1}):
 *   v^{k+1/2} = v^k + (dt/2) (f^k + b)/rho,  u^{k+1} = u^k + dt v^{k+1/2},
 *   v^{k+1} = v^{k+1/2} + (dt/2) (f^{k+1} + b)/rho,
 * with the damage test at every force evaluation.  Clamped nodes keep
 * u = v = 0; prescribed-velocity nodes take v^{k+1/2} = r(k+1/2) vbar,
 * u^{k+1} = u^k + dt v^{k+1/2}, v^{k+1} = r(k+1) vbar, r(s) =
 * min(1, s/ramp_steps).  One fused kernel per step (force + damage +
 * half-kicks + drift + boundary data); the force at the final state is
 * evaluated lazily by pd_sim_get.  Asynchronous.
 */
int pd_verlet_step(pd_sim sim, int64_t nsteps, double dt);

/*
 * Advance a simulation by nsteps steps of the central-difference scheme
 * (the finite-difference equation of Section "Explicit time integration"):
 *   u^{k+1} = 2 u^k - u^{k-1} + dt^2 (f^k + b)/rho   (free nodes),
 * boundary data as in pd_verlet_step.  The paper gives no starting rule: the
 * first step of each call is one velocity-Verlet step from the current
 * (u, v), the Taylor start u^{k+1} = u^k + dt v^k + dt^2 (f^k + b)/(2 rho).
 * pd_sim_get then reports v^N = (u^N - u^{N-1})/dt + (dt/2)(f^N + b)/rho.
 * The scheme equals velocity Verlet in exact arithmetic and differs in
 * rounding.  Runs on the simulation's step kernel (streamed, tile or
 * gather).  Asynchronous; the same dt rule as pd_verlet_step.
 */
int pd_central_step(pd_sim sim, int64_t nsteps, double dt);

/*
 * Read the state back (each output may be NULL): u, v device [n][dim],
 * alive device uint8[nnz] (exported order), ke_pe host double[2] =
 * {sum_i rho V_i |v_i|^2 / 2, sum_i V_i U_i}, step host int64.
 * Returns PD_ENONFINITE (outputs still written) if u or v is not finite.
 * Synchronises the stream.
 */
int pd_sim_get(pd_sim sim, double *u, double *v, uint8_t *alive, double *ke_pe, int64_t *step);

/* Overwrite the state (checkpoint restore); NULL leaves that part as is. */
int pd_sim_set(pd_sim sim, const double *u, const double *v, const uint8_t *alive, int64_t step);

int pd_sim_destroy(pd_sim sim);

/*
 * Batched explicit steps (serving several independent simulations at once).
 * One launch per step covers the tiles of every simulation in the batch, so
 * small meshes do not each pay a launch; with use_graph != 0 the chunk of
 * nsteps launches is captured once in a hipGraph and replayed on later calls
 * with the same batch shape.
 *
 * sims[k] takes steps[k] (0 <= steps[k] <= nsteps) velocity-Verlet steps of
 * dt[k] (host arrays of length nsims); it then stands exactly where
 * pd_verlet_step(sims[k], steps[k], dt[k]) would have left it, bit for bit.
 * Every simulation must run the streamed step kernel (pd_sim_info kernel 3)
 * on b's context, with one dim, precision, law, lane count and tile size.  The
 * call is asynchronous on the context's stream.  A batch handle holds the
 * descriptor buffer (each simulation's state at the start of the chunk,
 * uploaded by every call) and the captured graph (whose k-th launch carries
 * its step index k); it must outlive its pending work and is freed by
 * pd_batch_destroy (which synchronises).
 */
int pd_batch_create(pd_ctx ctx, pd_batch *out);
int pd_batch_step(pd_batch b, pd_sim *sims, int nsims, const int64_t *steps, const double *dt,
                  int64_t nsteps, int use_graph);
int pd_batch_destroy(pd_batch b);

/*
 * Serving: independent explicit simulations submitted as requests.
 *
 * pd_server_create(ctx, hbm_budget, chunk_steps, lanes, &srv)
 *   hbm_budget   device bytes the running simulations may hold together;
 *   chunk_steps  steps per scheduling round;
 *   lanes        lane count for every simulation (0: automatic per mesh; a
 *                fixed value lets meshes of different horizons share one
 *                batched launch).
 * pd_server_submit copies the request's host arrays and queues it (arrival
 *   order).  A request's state: PD_REQ_QUEUED -> PD_REQ_RUNNING ->
 *   PD_REQ_DONE, or PD_REQ_FAILED with info.status (PD_ECAPACITY if its
 *   device memory exceeds the whole budget).  The request's arrays are not
 *   referenced after the call returns.
 * pd_server_pump runs one scheduling round and returns when it is done
 *   (synchronises): admits queued requests in arrival order while the head's
 *   device-memory estimate fits the free budget (while simulations run, this
 *   happens during their chunk, on a stream of the server's own, and the
 *   requests admitted then join at the next round); a request whose built size
 *   (known after its neighbour list is built) does not fit after all is freed
 *   and waits at the head with that size, so the charged bytes never exceed
 *   hbm_budget (continuous batching:
 *   requests join the running set as memory frees up), advances every running
 *   simulation by up to chunk_steps steps in batched launches (one per group
 *   of simulations with the same dimension, lane count, tile size,
 *   precision and law; a chunk whose
 *   set of simulations did not change since the last round replays a
 *   captured hipGraph), and retires those that reached their step count,
 *   freeing their memory.  A result is bit for bit the same as the request
 *   run alone with pd_verlet_step at the same lane count.
 * pd_server_info: timestamps (pd_server_clock seconds, a monotonic clock)
 *   of submission (or the request's t_arrival if > 0), admission and
 *   completion; device bytes charged; directed bonds.
 * pd_server_result: the final u and v (host [n][dim], original node order)
 *   of a finished request submitted with keep_state != 0.
 * pd_server_usage: device bytes charged now and at most so far.
 * pd_server_get_stats: where the pump's time went (cumulative).
 * pd_server_destroy frees every request (queued, running or done).
 * Errors: PD_EINVAL for a malformed request or unknown id; a device error
 *   while building or stepping is returned by pd_server_pump; an error
 *   building one request fails only that request.
 */
enum { PD_REQ_QUEUED = 0, PD_REQ_RUNNING = 1, PD_REQ_DONE = 2, PD_REQ_FAILED = 3 };

typedef struct {
    int dim;                /* 2 or 3 */
    int64_t n;              /* nodes */
    const double *X;        /* host [n][dim] reference positions */
    const double *V;        /* host [n] nodal volumes */
    const double *u0, *v0;  /* host [n][dim] or NULL (zero) */
    const uint8_t *bc_kind; /* host [n] PD_BC_* or NULL (all free) */
    const double *bc_vel;   /* host [n][dim], required with bc_kind */
    const double *notch;    /* host [nseg][4] pre-crack segments (2-d) or NULL */
    int nseg;
    double delta;           /* horizon */
    pd_material mat;
    double dt;
    int64_t nsteps;         /* velocity-Verlet steps to run */
    int64_t ramp_steps;     /* boundary-velocity ramp (0: none) */
    int keep_state;         /* keep the final u, v for pd_server_result */
    double t_arrival;       /* > 0: arrival time on pd_server_clock */
} pd_request;

typedef struct {
    int64_t id;
    int state;              /* PD_REQ_* */
    int status;             /* PD_OK, or why the request failed */
    int64_t bytes;          /* device bytes charged against the budget */
    int64_t bonds;          /* directed bonds of its mesh */
    double t_submit, t_admit, t_done;
} pd_request_info;

typedef struct {
    double admit_s;     /* host wall time building admitted requests */
    double step_s;      /* launching chunks and waiting for them */
    double retire_s;    /* reading back and freeing finished requests */
    int64_t rounds;     /* pd_server_pump calls */
    int64_t admitted;
    int64_t launches;   /* batched chunks */
    int64_t replays;    /* of them, replays of a captured graph */
    double admit_overlap_s; /* of admit_s, the part spent while a chunk ran */
} pd_server_stats;

double pd_server_clock(void);
int pd_server_create(pd_ctx ctx, int64_t hbm_budget, int64_t chunk_steps, int lanes,
                     pd_server *out);
int pd_server_submit(pd_server srv, const pd_request *req, int64_t *id);
int pd_server_pump(pd_server srv, int *n_running, int *n_queued);
int pd_server_info(pd_server srv, int64_t id, pd_request_info *info);
int pd_server_result(pd_server srv, int64_t id, double *u, double *v);
int pd_server_usage(pd_server srv, int64_t *used, int64_t *peak);
int pd_server_get_stats(pd_server srv, pd_server_stats *out);
int pd_server_destroy(pd_server srv);

/*
 * Launch configuration a simulation runs with (each output may be NULL):
 * kernel 1 = gather, 2 = LDS tiles, 3 = streamed tiles for the steps;
 * tile = nodes per tile (0 for gather);
 * block = threads per workgroup; lanes = lanes per node.
 */
int pd_sim_info(pd_sim sim, int *kernel, int *tile, int *block, int *lanes);

/*
 * Matrix-free tangent operator of the quasi-static problem, y = H w with
 * H = -V (x) df/du (the paper's tangent equation, evaluated analytically):
 *   y_i = -V_i sum_j mu_ij k_ij ((w_j - w_i).xi/|xi|^2) (xi/|xi|) V_j  (free i)
 *   y_i = w_i                                                          (fixed i)
 * with w_j read as 0 at fixed nodes and the bond stiffness k_ij = c for the
 * linearised law.  fixed: device uint8[n] (NULL = none), alive: device
 * uint8[nnz] exported order (NULL = all intact).  w, y device [n][dim]
 * float64.  Asynchronous.
 * pd_apply_tangent_at linearises at the displacement u (device [n][dim]):
 * for PD_LAW_NP k_ij = c exp(-beta r)(1 - 2 beta r), r = |xi| S(u)^2 (from
 * psi'(r) + 2 r psi''(r)); for the linear law it equals pd_apply_tangent.
 */
int pd_apply_tangent(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                     const double *V, const uint8_t *alive, const uint8_t *fixed,
                     const double *w, double *y);
int pd_apply_tangent_at(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                        const double *V, const double *u, const uint8_t *alive,
                        const uint8_t *fixed, const double *w, double *y);

/*
 * Quasi-static solve (implicit scheme of the paper, one load step): find u
 * with u = given values on fixed nodes and f(u) + b = 0 on free nodes, by
 * Newton steps H(u) du = V (f(u) + b) solved with conjugate gradients,
 * H(u) the tangent at the current iterate (one step for the linearised law;
 * for PD_LAW_NP a Newton-Krylov iteration, which needs a positive definite
 * tangent: 2 beta r < 1 on the bonds that carry load).
 *   precision PD_FP64: float64 CG solving each Newton system to the target.
 *   PD_MIXED (and PD_FP32): each correction solved to 1e-2 relative (each Newton
 *   system of PD_LAW_NP to 1e-4) by a CG with float32
 *   vectors and float32 bond arithmetic in the tangent but float64 dot
 *   products, inside iterative refinement on float64 residuals (the force
 *   in float64) until rtol is met.
 *   u      device [n][dim], in: initial guess holding the fixed values,
 *          out: solution (or last iterate)
 *   b      device [n][dim] body force density
 *   rtol   target ||V (f(u)+b)|| / ||V b|| over free nodes (e.g. 1e-10)
 *   maxit  limit on the total number of CG iterations
 * Returns PD_ENOCONV with info filled when the target is not reached.
 * Synchronises the stream.
 */
int pd_solve_implicit(pd_ctx ctx, pd_nbr nbr, const pd_material *mat, const double *X,
                      const double *V, const uint8_t *alive, const uint8_t *fixed,
                      const double *b, double *u, double rtol, int maxit, pd_solve_info *info);

#ifdef __cplusplus
}
#endif

#endif /* PD_H */
