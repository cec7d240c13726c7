/*
 * hweno.h -- C ABI of the MI355X (gfx950) implementation of the fifth-order
 * finite-difference interpolation-based Hermite WENO scheme HWENO-I
 * (Xie, Tao, Jiao, Zhang, arXiv 2411.11229).
 *
 * The library computes, on the GPU:
 *   - the semi-discrete operator L = (L^1, L^2[, L^3]) of (odeH) / (ode2H) and
 *     the modified derivatives v~ [, w~] of (limiter), for one stage state;
 *   - one SSP-RK3 time step of (fully-hweno) / (2Dfully-hweno);
 *   - the transpose of the Jacobian of that time step (discrete adjoint) at
 *     the step's recorded Lax-Friedrichs alphas and time step.
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked "host".
 *   - Arrays are structure-of-arrays: [ncomp][ny][nx], x fastest, contiguous,
 *     element type given by hweno_problem.precision (double or float).
 *     ncomp = 1 (scalar laws), 3 (1D Euler: rho, rho*u, E),
 *     4 (2D Euler: rho, rho*u, rho*v, E). In 1D, ny = 1 and every w / W
 *     argument must be NULL.
 *   - u is the solution, v = u_x and w = u_y its derivatives (EQ1)/(EQ3); the
 *     caller supplies all of them.
 *   - The caller owns every buffer, including the workspace ws, whose size
 *     comes from hweno_workspace_bytes and which must be passed through
 *     hweno_workspace_init once before first use. The library allocates no
 *     device memory and keeps no device state, except the static scratch
 *     array of hweno_step_noalloc (for callers that cannot allocate); its
 *     other global state is host-side: a cache of occupancy queries and the
 *     strip-height setting of hweno_set_strip_rows. Calls on different streams
 *     with different workspaces are independent; calls sharing a workspace
 *     must be ordered on one stream.
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream);
 *     nothing blocks the host except hweno_health.
 *   - Errors are reported by status code only. Argument errors return
 *     HWENO_EINVAL before anything is enqueued. Non-finite or non-physical
 *     states found while reducing wave speeds set sticky flags in the
 *     workspace, read by hweno_health.
 */
#ifndef HWENO_H
#define HWENO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HWENO_OK = 0,
  HWENO_EINVAL = -1,         /* bad argument: null pointer, size, enum, aliasing */
  HWENO_EUNSUPPORTED = -2,   /* valid but not implemented combination           */
  HWENO_EDEVICE = -3,        /* a HIP runtime call failed                        */
  HWENO_ENONFINITE = -4,     /* a NaN / Inf was seen in a state                  */
  HWENO_ENONPHYSICAL = -5,   /* density or pressure <= 0 was seen (Euler)        */
  HWENO_ESCRATCH = -6        /* too large for hweno_step_noalloc's scratch       */
} hweno_status;

typedef enum { HWENO_ADVECTION = 0, HWENO_BURGERS = 1, HWENO_EULER = 2 } hweno_system;
/* Boundary conditions, by ghost cells (2 per side):
 *   periodic      wraps; must be set on both ends of an axis;
 *   transmissive  copies the nearest interior u, v, w (zero-order
 *                 extrapolation; the paper states no rule, this is a reading);
 *   reflective    a wall (remarks on boundary conditions in sections 2 and 3,
 *                 (RBC-1d), (RBC-2d-x), (RBC-2d-y)): ghost -1-k holds the
 *                 mirror image of cell k (ghost n+k of cell n-1-k) with the
 *                 normal momentum negated; the derivative along the wall
 *                 normal has every other component negated, the derivative
 *                 along the wall follows the state. HWENO_EULER only;
 *   dirichlet     a fixed state (the top and bottom boundaries of Example
 *                 4.11): both ghost cells hold bc_state[side] (conserved
 *                 variables), the derivatives v, w are 0 there;
 *   split         (y sides of 2D Euler only) a rule that changes along x and
 *                 in time, as on the bottom and top of Example 4.7: see
 *                 hweno_split. Only hweno_rhs (at t = 0) and the time
 *                 steps (hweno_step, hweno_steps, hweno_step_noalloc) accept
 *                 it; hweno_step_frozen and hweno_adjoint_step return
 *                 HWENO_EUNSUPPORTED.
 * The two ends of an axis are independent except for periodic. */
typedef enum {
  HWENO_PERIODIC = 0, HWENO_TRANSMISSIVE = 1, HWENO_REFLECTIVE = 2, HWENO_DIRICHLET = 3,
  HWENO_SPLIT = 4
} hweno_bc;

/* A split y side: a ghost cell at (x, y) (cell centres, the domain's
 * lower-left corner at the origin, so x = (i + 1/2) dx) follows kind[0] if
 * x < x0 + slope * y + speed * t, else kind[1]; each kind is
 * HWENO_TRANSMISSIVE, HWENO_REFLECTIVE or HWENO_DIRICHLET (with state[k],
 * conserved variables). t is the stage time: t^n, t^n + dt, t^n + dt/2 for
 * the three SSP-RK3 stages of hweno_step. */
typedef struct {
  double x0, slope, speed;
  int32_t kind[2];
  double state[2][4];
} hweno_split;
typedef enum { HWENO_F64 = 0, HWENO_F32 = 1 } hweno_precision;
/* Characteristic basis of the HWENO interpolation for the Euler systems
 * (remark on systems in section 2, local characteristic decomposition):
 *   cell       the eigenvectors of A(U_i) serve both faces and the modified
 *              derivative of cell i: one interpolation per cell and direction
 *              (the reading the paper's efficiency argument needs);
 *   interface  Jiang and Shu's form: u^-_{i+1/2}, u^+_{i+1/2} in the
 *              eigenvectors of Roe's matrix of U_i and U_{i+1}, the modified
 *              derivative in the cell basis (three interpolations per cell).
 * Ignored for the scalar laws. hweno_adjoint_step differentiates either
 * basis. */
typedef enum { HWENO_BASIS_CELL = 0, HWENO_BASIS_INTERFACE = 1 } hweno_char_basis;
typedef enum {
  HWENO_DT_PRODUCTION = 0,   /* dt = cfl / (ax/dx + ay/dy)                    */
  HWENO_DT_ACCURACY = 1,     /* dt = cfl / (ax/dx^(5/3) + ay/dy^(5/3))        */
  HWENO_DT_FIXED = 2         /* dt = dt_fixed                                  */
} hweno_dt_rule;

/*
 * The problem, following the paper's statement: a uniform cell-centred mesh
 * (section 2: x_i, dx; section 3: y_j, dy), the flux (scalar advection
 * f = a u, g = b u; Burgers f = g = u^2/2; Euler (euler1d)/(euler2d) with
 * E = P/(gas_gamma - 1) + rho |vel|^2 / 2), the linear weights of (interp)
 * (gamma0; gamma1 = gamma2 = (1 - gamma0)/2) and of (limiter) (d0;
 * d1 = d2 = (1 - d0)/2), and epsilon of (nonlinear). The paper uses
 * gamma0 = 0.95 (1D) / 0.99 (2D), d0 = 0.9, eps = 1e-10. `gravity` is g of
 * the source term of (euler2d-s), S(U) = g (0, 0, rho, rho v) (2D Euler
 * only; 0 = no source); S is linear, so the derivative equations carry
 * S(v) and S(w).
 */
typedef struct {
  int32_t dim;          /* 1 or 2                                                */
  int32_t nx, ny;       /* cells; nx >= 5; ny >= 5 in 2D, ny == 1 in 1D; one      */
                        /* state array (ncomp * nx * ny elements) under 4 GiB     */
  double dx, dy;        /* > 0; dy ignored in 1D                                  */
  int32_t system;       /* hweno_system                                           */
  double adv_a, adv_b;  /* advection speeds (HWENO_ADVECTION only)                */
  double gas_gamma;     /* ratio of specific heats, > 1 (HWENO_EULER only)        */
  double gamma0;        /* in (0, 1)                                              */
  double d0;            /* in (0, 1)                                              */
  double eps;           /* > 0                                                    */
  int32_t bc[4];        /* hweno_bc at x_lo, x_hi, y_lo, y_hi (see hweno_bc)      */
  int32_t precision;    /* hweno_precision of every array argument                */
  int32_t char_basis;   /* hweno_char_basis                                       */
  double bc_state[4][4];/* conserved state of each HWENO_DIRICHLET side (x_lo,     */
                        /* x_hi, y_lo, y_hi), first ncomp entries; finite, and    */
                        /* rho, P > 0 for Euler                                   */
  double gravity;       /* g of (euler2d-s); 0 unless system == EULER, dim == 2   */
  hweno_split split[2]; /* y_lo, y_hi rules where bc[2] / bc[3] == HWENO_SPLIT    */
} hweno_problem;

/* Human-readable name of a status code (static string). */
const char* hweno_status_string(hweno_status s);

/* Validates `prob` (host) and stores the workspace size in bytes (host). */
hweno_status hweno_workspace_bytes(const hweno_problem* prob, size_t* bytes);

/* Clears the workspace's flag word and scalars. Call once per workspace
 * before its first use (enqueued on `stream`). */
hweno_status hweno_workspace_init(const hweno_problem* prob, void* ws, hipStream_t stream);

/*
 * Lax-Friedrichs alphas of (flux-LF): alpha[0] = max over interior cells of
 * |f'(u)| (Euler: |u| + c), alpha[1] the same for g (0 in 1D).
 * u: [ncomp][ny][nx]; alpha: device double[2], written.
 */
hweno_status hweno_max_wavespeed(const hweno_problem* prob, const void* u, double* alpha,
                                 void* ws, hipStream_t stream);

/*
 * One evaluation of the spatial operator, Steps 1-4 of sections 2 and 3:
 * Lu, Lv, Lw <- L^1, L^2, L^3 of (odeH)/(ode2H) at the state (u, v, w) with
 * the given alphas (device double[2]); vtilde, wtilde <- the modified
 * derivatives of (limiter) in x and y. For systems the interpolation and
 * the limiter run in local characteristic variables of the cell centre (or
 * of the faces, see hweno_char_basis). Split sides are taken at t = 0. With
 * `gravity` the source S of (euler2d-s) is included. Outputs must not alias
 * inputs. In 1D, w, Lw and wtilde are NULL.
 */
hweno_status hweno_rhs(const hweno_problem* prob, const void* u, const void* v, const void* w,
                       const double* alpha, void* Lu, void* Lv, void* Lw,
                       void* vtilde, void* wtilde, void* ws, hipStream_t stream);

/*
 * One SSP-RK3 step (fully-hweno)/(2Dfully-hweno), in place on (u, v, w).
 * Each stage takes its alphas from its own state (stage 1 from (u, v, w)).
 * dt from dt_rule (hweno_dt_rule) with `cfl`, or dt_fixed, from the stage-1
 * alphas, then clipped so that *t + dt does not pass t_end; when *t >= t_end
 * on entry the step leaves every buffer untouched.
 *   t          device double, in/out: advanced by dt (set to t_end on the
 *              clipped last step).
 *   dt_used    device double, out (may be NULL): the dt taken (0 if skipped).
 *   alpha_rec  device double[3][2], out (may be NULL): the alphas of the
 *              three stages, as needed by hweno_adjoint_step.
 *   stages     device buffer of 2 * 3 * ncomp planes (2D; 2 * 2 * ncomp in
 *              1D) of the array type, out (may be NULL): the stage states
 *              X^(1), X^(2) as [stage][field u,v,w][comp][ny][nx].
 */
hweno_status hweno_step(const hweno_problem* prob, void* u, void* v, void* w,
                        int32_t dt_rule, double cfl, double dt_fixed, double t_end,
                        double* t, double* dt_used, double* alpha_rec, void* stages,
                        void* ws, hipStream_t stream);

/*
 * hweno_step with instrumentation for timing: `events` (host array of 4
 * hipEvent_t created by the caller, or NULL) are recorded on `stream` right
 * before the stage-1 launch, after stage 1, after stage 2 and after stage 3,
 * so the elapsed times between consecutive events are the durations of the
 * three stage kernels. Arguments and results are otherwise those of
 * hweno_step.
 */
hweno_status hweno_step_profiled(const hweno_problem* prob, void* u, void* v, void* w,
                                 int32_t dt_rule, double cfl, double dt_fixed, double t_end,
                                 double* t, double* dt_used, double* alpha_rec, void* stages,
                                 void* ws, hipStream_t stream, hipEvent_t* events);

/*
 * nsteps consecutive SSP-RK3 steps, as nsteps calls of hweno_step (same
 * results, bit for bit) without stage states: the per-step outputs go to
 * dt_used[k] (device double[nsteps], may be NULL) and alpha_rec + 6k (device
 * double[nsteps][3][2], may be NULL). The stage-1 alphas of the first step
 * come from a reduction over the initial state; those of every later step
 * from the epilogue of the previous step's last stage, which evaluates the
 * spectral radii of the new state as it stores it (no separate pass).
 * Steps past t_end leave the state untouched (dt_used 0). `events`: NULL or
 * a host array of 4 * nsteps hipEvent_t, recorded as in hweno_step_profiled
 * for each step.
 */
hweno_status hweno_steps(const hweno_problem* prob, void* u, void* v, void* w, int32_t nsteps,
                         int32_t dt_rule, double cfl, double dt_fixed, double t_end, double* t,
                         double* dt_used, double* alpha_rec, void* ws, hipStream_t stream,
                         hipEvent_t* events);

/*
 * hweno_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step, with the same arguments except that it takes no workspace and
 * no stage-state buffer, and the same results bit for bit. Its workspace is
 * a static device array of the library, 128 MiB (134217728 bytes) per GPU,
 * held from the first call on that GPU until the process ends; nothing is
 * allocated or freed, by the library or by any routine it calls. It runs on
 * the current device, whose stream `stream` must be.
 *   Limit: the step's workspace (4 KiB + 16 KiB + 2 stage states of 2 or 3
 *   fields + the RK base derivatives; for 2D Euler 256 bytes per cell in
 *   FP64, i.e. up to 724^2 cells, and 128 bytes per cell in FP32, up to
 *   1023^2) must fit in the 128 MiB, else HWENO_ESCRATCH is returned before
 *   anything is enqueued.
 *   Sharing: every call on one GPU uses that GPU's one array, which keeps the
 *   last call's contents (each call clears what must start at zero). Calls
 *   that overlap in time on one GPU (different streams, or threads) race:
 *   order them on one stream. The state flags of hweno_health are not
 *   reported by this entry point.
 */
hweno_status hweno_step_noalloc(const hweno_problem* prob, void* u, void* v, void* w,
                                int32_t dt_rule, double cfl, double dt_fixed, double t_end,
                                double* t, double* dt_used, double* alpha_rec,
                                hipStream_t stream);

/*
 * Strip height (rows marched by one wavefront) of the 2D forward stage
 * kernels, for every later launch in the process: rows > 0 forces it,
 * 0 restores the choice of the occupancy model. Results do not depend on it
 * (bit for bit); it exists to test exactly that. HWENO_EINVAL if rows < 0.
 */
hweno_status hweno_set_strip_rows(int32_t rows);

/*
 * One SSP-RK3 step on (u, v, w) with a given time step (device double) and
 * given stage alphas (device double[3][2], e.g. the alpha_rec of an earlier
 * hweno_step): the map whose Jacobian hweno_adjoint_step transposes. No
 * clipping, no time update. The new state goes to (u_out, v_out, w_out) if
 * u_out is not NULL (then (u, v, w) are left unchanged and the outputs must
 * not overlap any input), else in place. `stages` as in hweno_step.
 * HWENO_EUNSUPPORTED for split sides (the step carries no time).
 */
hweno_status hweno_step_frozen(const hweno_problem* prob, void* u, void* v, void* w,
                               void* u_out, void* v_out, void* w_out, const double* dt,
                               const double* alpha_rec, void* stages, void* ws,
                               hipStream_t stream);

/*
 * Discrete adjoint of one hweno_step: the transpose of the Jacobian of the
 * SSP-RK3 step (fully-hweno)/(2Dfully-hweno), obtained by the chain rule
 * through every stage. Given lambda = dJ/dX^{n+1} (lam_*_in) it writes
 * dJ/dX^n (lam_*_out), where X = (u, v, w), with the recorded dt (device
 * double) and stage alphas (device double[3][2]) held fixed, i.e. not
 * differentiated. With B(X) = (u, v~(X), w~(X)) the RK base and
 * vjp(X; a, b) = (dB/dX)^T a + (dL/dX)^T b for one stage:
 *   lambda2 = vjp(X^(2); 2/3 lambda, 2/3 dt lambda),
 *   lambda1 = vjp(X^(1); 1/4 lambda2, 1/4 dt lambda2),
 *   out     = vjp(X^n; lambda1 + 3/4 lambda2 + 1/3 lambda, dt lambda1).
 * (u_n, v_n, w_n) is the step's initial state. `stages` holds X^(1), X^(2)
 * as written by hweno_step, or is NULL, in which case they are recomputed
 * (in the workspace, which also holds lambda2 and lambda1). At the kinks of
 * |beta0 - beta_k| the derivative of |.| is taken as sign(0) = 0. Output
 * buffers must not alias any input. The result is deterministic: every sum
 * is formed in a fixed order, without atomics. With the interface basis
 * the basis of each face's Roe matrix is differentiated with respect to
 * both cells that define it. Returns HWENO_EUNSUPPORTED for split sides.
 */
hweno_status hweno_adjoint_step(const hweno_problem* prob, const void* u_n, const void* v_n,
                                const void* w_n, const void* stages, const double* dt,
                                const double* alpha_rec, const void* lam_u_in,
                                const void* lam_v_in, const void* lam_w_in, void* lam_u_out,
                                void* lam_v_out, void* lam_w_out, void* ws, hipStream_t stream);

/* Synchronises `stream` and reports the sticky state flags of `ws`:
 * HWENO_ENONFINITE, HWENO_ENONPHYSICAL or HWENO_OK. clear != 0 resets them. */
hweno_status hweno_health(const hweno_problem* prob, void* ws, hipStream_t stream, int32_t clear);

#ifdef __cplusplus
}
#endif

#endif /* HWENO_H */
