/*
 * ps.h - pressure-Poisson / projection library for AMD MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of a wall-bounded, staggered-grid
 * Navier-Stokes solver (Zhu et al., "AFiD-GPU", arXiv 1705.01423):
 *
 *   - the direct pressure-Poisson solve of Sec. 2.2: 2-D FFT in the two
 *     periodic directions with modified wavenumbers, one tridiagonal solve per
 *     wavenumber pair in the wall-normal direction, inverse 2-D FFT;
 *   - the projection and pressure update that follow it (Sec. 2.1 "delta"
 *     form, end of Sec. 2.2);
 *   - the wall-normal Crank-Nicolson solves of the implicit viscous and
 *     diffusive terms (Sec. 2.1-2.2);
 *   - one RK3 / Crank-Nicolson substep of Eqs. (1)-(3) (Sec. 2.1);
 *   - adjoints (vector-Jacobian products) of the solve, the projection and
 *     the substep.
 *
 * Axes: z is wall-normal (the paper's x); x and y are periodic (the paper's
 * y and z).
 *
 * Storage: every field is a device pointer to FP64 values, C order [z][y][x]
 * (x fastest), contiguous, 16-byte aligned (checked: PS_EINVAL otherwise),
 * owned by the caller.
 *   centre fields (p, phi, f, u, v):  nz x ny x nx
 *   z-face fields (w, T):             (nz+1) x ny x nx, wall rows 0 and nz stored
 * u sits on x-faces (x = i*dx), v on y-faces (y = j*dy), w and T on z-faces
 * (Fig. 1 of the paper).
 *
 * Streams: every call is enqueued on the HIP stream passed in (NULL = the
 * legacy default stream) and returns without waiting, except where a call
 * says it synchronises.  Calls that share one plan must not run concurrently
 * on different streams: the plan owns one workspace.
 *
 * Errors: functions return ps_status.  Arguments are validated before any
 * device work is enqueued; on an error nothing is enqueued and
 * ps_last_error() returns a message (thread-local, valid until the next call
 * on the same thread).  No exception crosses this boundary.
 */
#ifndef PS_H
#define PS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_plan_s* ps_plan_t;

typedef enum {
    PS_OK = 0,
    PS_EINVAL = 1,          /* bad argument (dims, grid, pointer, size)           */
    PS_ENOMEM = 2,          /* device allocation failed                          */
    PS_EDEVICE = 3,         /* HIP runtime error                                 */
    PS_ENOTCOMPAT = 4,      /* right-hand side incompatible (STRICT_COMPAT)       */
    PS_ENONFINITE = 5,      /* non-finite input (CHECK_FINITE)                   */
    PS_ENOTCONVERGED = 6    /* refinement stopped above the tolerance             */
} ps_status;

typedef enum {
    PS_FP64 = 0,            /* FFTs and tridiagonal solves in FP64               */
    PS_FP32_REFINED = 1,    /* FP32 solves, refined on the FP64 residual          */
    PS_FP32 = 2             /* one FP32 solve, FP64 in/out (for measurement)      */
} ps_precision;

enum {
    PS_FLAG_STRICT_COMPAT = 1u,   /* return PS_ENOTCOMPAT for an incompatible rhs  */
    PS_FLAG_CHECK_FINITE = 2u     /* scan the input for NaN/Inf (synchronises)     */
};

enum { PS_CENTER = 0, PS_FACE = 1 };   /* cn_solve kinds */

typedef struct {
    int iterations;        /* FP32 solves performed (FP64 path: 1)                   */
    double rel_update;     /* last ||delta||_2 / ||phi||_2 of the refinement (0 FP64) */
    double rel_residual;   /* ||r||_2/||f~||_2 of the iterate before the last update  */
                           /* (refined path; -1 when not computed)                   */
    double compat_defect;  /* dz-weighted mean removed from the right-hand side       */
    double gauge_shift;    /* dz-weighted mean of the final phi before re-gauging      */
} ps_info;

/*
 * poisson_plan_create - grid, tables and workspace for one box.
 *
 * Defines the discrete problem of Sec. 2.1-2.2: periodic x, y with nx, ny
 * uniform cells over lengths lx, ly; wall-normal faces zf_host[0..nz]
 * (host array, strictly increasing, zf[0] = 0 and zf[nz] = 1 expected but
 * any increasing faces are accepted), copied.  Derived metrics (all FP64,
 * formed identically on every path):
 *   dz[k] = zf[k+1]-zf[k];  dzc[k] = (dz[k-1]+dz[k])/2;  o[k] = 1/dzc[k]
 *   lamx[kx] = (4/dx^2) sin^2(pi kx/nx)  (modified wavenumbers, Sec. 2.2)
 * nx, ny must be of the form 2^a 3^b with b <= 1 (one factor 3 at most: the
 * transform lengths the library is built for), nx even, 4 <= nx, ny <= 4096;
 * 2 <= nz <= 2048.  Other sizes return PS_EINVAL.
 * prec: ps_precision.  tol: relative error target of the refinement (<= 0
 * selects 1e-12): it stops when the last correction ||delta_i||/||phi|| is
 * <= tol, or, from the second correction on, when the error it predicts is,
 * rho_i ||delta_i||/||phi|| with rho_i = ||delta_i|| / ||delta_{i-1}||.  A
 * correction that shrinks by less than half (the rounding floor) or the cap
 * max_iter ends it without convergence (PS_ENOTCONVERGED from the solve).
 * max_iter: refinement cap (<= 0 selects 10).  flags: PS_FLAG_*.
 * The plan is bound to the current HIP device and allocates its workspace
 * there (see poisson_plan_workspace_bytes).  It also allocates its own
 * tables: metrics, twiddles and the pivot excesses entering each 8-row chunk
 * of every z column (8 bytes FP64 / 4 bytes FP32 per entry, (nx/2+1 rounded
 * up to 8 / 16) * ny * ceil(nz/8) entries, 0.27 GB at 1024^2 x 512 FP64),
 * formed by one kernel on the null stream before the call returns.  *out
 * receives the plan.
 */
ps_status poisson_plan_create(ps_plan_t* out, int nx, int ny, int nz, double lx, double ly,
                              const double* zf_host, int prec, double tol, int max_iter,
                              unsigned flags);

/* Device workspace the plan uses, in bytes (spectral buffers and scratch). */
size_t poisson_plan_workspace_bytes(ps_plan_t plan);

/*
 * poisson_plan_set_workspace - hand the plan caller-owned device memory of at
 * least poisson_plan_workspace_bytes() bytes, 256-byte aligned (as the
 * paper's solver shares one work area among its FFT plans, Sec. 3.3).  The
 * plan frees the workspace it allocated itself and uses this one until it is
 * destroyed; the caller keeps ownership and must keep it alive.  dev = NULL
 * returns the plan to a workspace of its own.
 */
ps_status poisson_plan_set_workspace(ps_plan_t plan, void* dev, size_t bytes);

/* Release the plan and the device memory it allocated.  NULL is accepted. */
ps_status poisson_plan_destroy(ps_plan_t plan);

/*
 * poisson_solve - phi = L^+ (f - mean_dz f), dz-weighted zero mean.
 *
 * L = D G is the flux-form staggered Laplacian: periodic in x and y, zero
 * normal gradient at the walls (Sec. 2.1-2.2).  The right-hand side is made
 * compatible by removing its dz-weighted mean (reported in info; under
 * PS_FLAG_STRICT_COMPAT the call returns PS_ENOTCOMPAT, phi written, when
 * |mean| exceeds 1e-8 max|f|: one more read of f and a synchronisation).
 * f and phi: centre fields (nz x ny x nx); f is not modified; phi may not
 * alias f.  PS_FLAG_CHECK_FINITE: PS_ENONFINITE, nothing written, when f
 * holds a NaN or Inf.  FP32_REFINED synchronises once per refinement
 * iteration; info != NULL synchronises at the end.  Returns
 * PS_ENOTCONVERGED (phi still written, info filled) when the refinement
 * stops above the tolerance (see poisson_plan_create).
 */
ps_status poisson_solve(ps_plan_t plan, const double* f, double* phi, void* stream, ps_info* info);

/*
 * poisson_solve_static - poisson_solve without the plan's workspace and without
 * any allocation: for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The spectral buffers and reduction scratch come from
 * one statically allocated device array of 256 MiB (268435456 bytes) that the
 * library holds on every GPU it runs on until the process ends; the call
 * returns PS_EINVAL, enqueuing nothing, when the plan needs more than that
 * (poisson_plan_workspace_bytes() > 268435456, e.g. beyond about 256 x 256 x
 * 192 in FP64).  Same results as poisson_solve (the same kernels), same
 * arguments and synchronisation rules; the plan's device must be current.
 * Every call on a GPU shares that GPU's array and leaves its contents behind
 * (no result depends on them): calls that overlap on one GPU, on any streams
 * or plans, race and must be serialised by the caller.
 */
ps_status poisson_solve_static(ps_plan_t plan, const double* f, double* phi, void* stream, ps_info* info);

/*
 * project - projection and pressure update (Sec. 2.1, end of Sec. 2.2):
 *     L phi = D u* / s,   u <- u* - s G phi,   p <- p + phi - c Dzz phi
 * u, v: centre-z fields (nz x ny x nx), updated in place; w: z-face field,
 * interior faces updated (wall rows left as given; the divergence uses them);
 * p: centre field updated in place (may be NULL: no pressure update);
 * phi_out: receives phi (may be NULL).  s > 0 (alpha_l dt; 1 for a plain
 * projection), c >= 0 (alpha_l dt nu / 2).  The plan's flags apply to the
 * right-hand side D u* / s as in poisson_solve (with either flag set it is
 * stored before the solve instead of formed inside the first transform);
 * on PS_ENOTCONVERGED the update is still applied.
 */
ps_status project(ps_plan_t plan, double* u, double* v, double* w, double* p, double* phi_out,
                  double s, double c, void* stream, ps_info* info);

/*
 * cn_solve - (I - beta Dzz) x = rhs for every (x, y) column, in place
 * (wall-normal Crank-Nicolson solve, Sec. 2.1-2.2; only the wall-normal
 * direction is implicit).  Homogeneous Dirichlet walls (delta form).
 * kind PS_CENTER: rhs_inout is a centre field, nz unknowns per column, the
 *   wall half a cell beyond the first / last centre;
 * kind PS_FACE: rhs_inout is a z-face field, the nz-1 interior faces are
 *   solved and the wall rows are set to zero.
 * beta >= 0.
 */
ps_status cn_solve(ps_plan_t plan, int kind, double beta, double* rhs_inout, void* stream);

/*
 * poisson_solve_adjoint - g_rhs = S^T g_phi, the transpose of poisson_solve's
 * linear map S.  L is self-adjoint in the dz-weighted inner product and the
 * compatibility projection and gauge are dz-orthogonal, so
 * S^T = Vc S Vc^-1 with Vc = diag(dz[k]); it is applied that way.
 * Same layout, precision and synchronisation rules as poisson_solve.
 */
ps_status poisson_solve_adjoint(ps_plan_t plan, const double* g_phi, double* g_rhs,
                                void* stream, ps_info* info);

/*
 * project_adjoint - transpose of project's map u* -> u (with the same s),
 * P^T = Vf P Vf^-1 with Vf = dz[k] on u, v and dzc[k] on interior w:
 * writes gu_star = P^T g_u etc.  When g_p != NULL, the pressure output's
 * cotangent is added: project's p_out depends on u* through
 * phi - c Dzz phi with phi = S D u* / s.  Wall rows of gw_star are zero.
 * Inputs are not modified; outputs may not alias inputs.
 */
ps_status project_adjoint(ps_plan_t plan, const double* g_u, const double* g_v, const double* g_w,
                          const double* g_p, double* gu_star, double* gv_star, double* gw_star,
                          double s, double c, void* stream, ps_info* info);

/*
 * ps_cfl - maximum CFL number of Listing 1 of the paper, for unit time step:
 *   max over cells of 0.5 (|w_k + w_{k+1}|/dz_k + |v_j + v_{j+1}|/dy + |u_i + u_{i+1}|/dx)
 * (at least 1e-8).  Writes one double to the device pointer cfl_dev.  A NaN
 * velocity gives a NaN (the maximum propagates NaN).
 */
ps_status ps_cfl(ps_plan_t plan, const double* u, const double* v, const double* w,
                 double* cfl_dev, void* stream);

/*
 * rk3_substep - one substep l (1..3) of the low-storage RK3 / Crank-Nicolson
 * scheme with pressure in delta form (Sec. 2.1), for Eqs. (1)-(3) with
 * Boussinesq buoyancy +T on w, viscosity nu, diffusivity kappa, no-slip walls
 * and T fixed at the walls (its wall rows):
 *   H_q = -A(q) + nu (Dxx + Dyy) q   (+ T for w; kappa for T)
 *   (I - alpha dt nu/2 Dzz) dq = dt [gamma H_q + rho H_q^prev - alpha G p + alpha nu Dzz q]
 *   q* = q + dq;  L phi = D u* / (alpha dt);  u = u* - alpha dt G phi;
 *   p += phi - (alpha dt nu/2) Dzz phi;  T likewise (its advection uses the
 *   substep's input velocity).
 * gamma = (8/15, 5/12, 3/4), rho = (0, -17/60, -5/12), alpha = gamma + rho.
 * state: u, v, w, t, p, updated in place.  h_prev: the previous substep's H
 * (four fields u, v, w, t; ignored for l = 1, may then be NULL).  h_out:
 * receives this substep's H (may be NULL); h_prev and h_out may be the same
 * buffers (each point's H is read before it is overwritten).  The Poisson
 * solve runs at the plan's precision.
 */
ps_status rk3_substep(ps_plan_t plan, int l, double dt, double nu, double kappa,
                      double* u, double* v, double* w, double* t, double* p,
                      const double* const* h_prev, double* const* h_out,
                      void* stream, ps_info* info);

/*
 * rk3_substep_adjoint - vector-Jacobian product of rk3_substep (substep l,
 * dt fixed) at the input state (u, v, w, t, p), which is not modified: the
 * substep is linear in everything but the advection, whose derivative is
 * formed from that state (Sec. 2.1 discretisation).  Cotangents in:
 *   g_out[0..4]  of the output state (u, v, w, t, p);
 *   g_hout[0..3] of the substep's H output (u, v, w, t), or NULL when H is
 *                not used downstream (the substep's H feeds substep l + 1).
 * Cotangents out:
 *   g_in[0..4]    of the input state;
 *   g_hprev[0..3] of the previous substep's H (h_prev of rk3_substep), or
 *                 NULL; for l = 1 it is zero (rho_1 = 0).
 * g_hprev may share g_hout's buffers (g_hout is consumed first); g_in may not
 * alias g_out or g_hout, nor g_hprev g_in or g_out.  Wall rows of w and t
 * carry zero cotangent.  The Poisson solves run at the plan's precision
 * (status as project_adjoint).
 */
ps_status rk3_substep_adjoint(ps_plan_t plan, int l, double dt, double nu, double kappa,
                              const double* u, const double* v, const double* w,
                              const double* t, const double* p,
                              const double* const* g_out, const double* const* g_hout,
                              double* const* g_in, double* const* g_hprev,
                              void* stream, ps_info* info);

/*
 * rk3_step_adjoint - vector-Jacobian product of rk3_step with a fixed dt > 0
 * (the Courant-limited step size is a non-differentiable maximum and is not
 * differentiated; pass the dt the forward step used).  The three substeps
 * (Sec. 2.1) are recomputed from the input state (u, v, w, t, p, not
 * modified), then their adjoints run in reverse, each handing the cotangent
 * of H^l down to substep l.  g_out[0..4]: cotangents of the step's output
 * state; g_in[0..4] receive those of its input.  Allocates 32 field-sized
 * temporaries in the plan on first use.  Returns PS_ENOTCONVERGED (outputs
 * written) when a refinement stopped above the tolerance.
 */
ps_status rk3_step_adjoint(ps_plan_t plan, double dt, double nu, double kappa,
                           const double* u, const double* v, const double* w,
                           const double* t, const double* p,
                           const double* const* g_out, double* const* g_in,
                           void* stream, ps_info* info);

/*
 * rk3_step - one full time step of the low-storage RK3 scheme (Sec. 2.1): the
 * substeps l = 1, 2, 3 of rk3_substep with the same dt, each handing its H to
 * the next through plan-owned temporaries.  dt > 0 is taken as given; dt <= 0
 * selects the Courant-limited step of Listing 1, dt = min(dt_max, cfl_target /
 * ps_cfl(u, v, w)), which reads the Courant number back to the host (one
 * synchronisation); a non-finite Courant number returns PS_ENONFINITE before
 * anything is enqueued.  State as rk3_substep, updated in place.  *dt_used
 * (host, may be NULL) receives the step taken; info (may be NULL) sums the
 * Poisson solves of the three substeps.  When a substep's refinement stops
 * above the tolerance the step is still completed and PS_ENOTCONVERGED is
 * returned.
 */
ps_status rk3_step(ps_plan_t plan, double dt, double cfl_target, double dt_max, double nu, double kappa,
                   double* u, double* v, double* w, double* t, double* p, double* dt_used, void* stream,
                   ps_info* info);

/*
 * ps_heat_flux - wall-normal statistics of a convection state (the Nusselt
 * number reported in Sec. 5, Table 3): plane means of T on the nz + 1 z-faces,
 *   mean_t[k] = <T>_k,
 * and the total vertical heat flux through the nz cell-centre planes,
 *   flux[k] = < wbar Tbar >_k - kappa (<T>_{k+1} - <T>_k) / dz_k,
 * wbar, Tbar the averages of the two z-faces bounding cell k, < > the x-y
 * plane average.  For unit height and wall temperatures 1 and 0 the Nusselt
 * profile is flux / kappa.  mean_t (nz + 1) and flux (nz): device arrays.
 * Plane sums run in a fixed order (deterministic for a given box).  Uses the
 * plan's scratch: order it with the plan's other calls.
 */
ps_status ps_heat_flux(ps_plan_t plan, const double* w, const double* t, double kappa, double* mean_t,
                       double* flux, void* stream);

/*
 * Multiple-resolution temperature grid (Sec. 6: the temperature on a grid of
 * higher resolution than the momentum, with its own refined time step).
 *
 * The temperature grid refines the plan's grid by integer factors (rx, ry,
 * rz), every momentum cell split into rx ry rz equal sub-cells: nxf = rx nx,
 * nyf = ry ny, nzf = rz nz, fine wall-normal faces zf'[rz k + m] = zf[k] +
 * (m / rz) dz[k].  The temperature tf is a fine z-face field, (nzf + 1) x
 * nyf x nxf, wall rows stored (fixed there).  Fine velocities: uf, vf
 * nzf x nyf x nxf, wf (nzf + 1) x nyf x nxf, at the fine faces.
 */
typedef struct ps_mr_s* ps_mr_t;

/*
 * mr_create - temperature grid on top of a plan (which must outlive it).
 * rx, ry, rz: 1 or 2 each (the factors the prolongation kernels are built
 * for; nzf <= 2048).  nsub (1..64): RK3 steps of the temperature per
 * momentum step.  Allocates the fine grid's tables and eight fine fields
 * (two velocity time levels, right-hand side, H) plus one coarse face field.
 */
ps_status mr_create(ps_mr_t* out, ps_plan_t plan, int rx, int ry, int rz, int nsub);
ps_status mr_destroy(ps_mr_t mr);
ps_status mr_shape(ps_mr_t mr, int* nxf, int* nyf, int* nzf);

/*
 * mr_prolong_velocity - momentum-grid face velocity (u, v, w) -> fine face
 * velocity (uf, vf, wf), second-order accurate and with every fine cell's
 * divergence equal to that of its momentum cell (so a divergence-free
 * velocity stays divergence free; the temperature advection needs it):
 * linear profiles across each coarse face with slopes from the neighbouring
 * faces (coarse fluxes kept; the no-slip wall value 0 as the outer point in
 * z), linear interpolation along the normal inside each cell, then the
 * smallest correction G psi, psi = -(L_loc)^+ r, of the cell's interior
 * fine faces (r: sub-cell divergences; L_loc: the Laplacian of the cell's
 * sub-cells with its coarse faces closed).
 */
ps_status mr_prolong_velocity(ps_mr_t mr, const double* u, const double* v, const double* w,
                              double* uf, double* vf, double* wf, void* stream);

/*
 * mr_restrict_temperature - tc[k][j][i] (coarse z-face field) = mean of
 * tf[rz k][ry j + b][rx i + a] over a < rx, b < ry: the temperature the
 * momentum equations' buoyancy sees.
 */
ps_status mr_restrict_temperature(ps_mr_t mr, const double* tf, double* tc, void* stream);

/*
 * mr_temperature_step - advance tf over dt by nsub RK3 / Crank-Nicolson
 * steps of dt / nsub on the temperature grid (the substep formulas of
 * rk3_substep for T, diffusivity kappa); each stage's advecting velocity is
 * (1 - s) vel0 + s vel1 at its start time s (fraction of dt; RK3 stages
 * start at 0, 8/15, 2/3 of a sub-step).  vel0, vel1: fine face velocities
 * (three pointers each).
 */
ps_status mr_temperature_step(ps_mr_t mr, double dt, double kappa, const double* const* vel0,
                              const double* const* vel1, double* tf, void* stream);

/*
 * rk3_step_mr - one coupled step: the momentum RK3 step (three substeps,
 * Sec. 2.1) with the buoyancy of the restricted temperature, frozen over
 * the step, then mr_temperature_step over the same dt with the prolonged
 * velocities of the step's start and end.  dt, cfl_target, dt_max, dt_used,
 * info as rk3_step (the Courant number is the momentum grid's).  u, v, w, p:
 * momentum-grid state; tf: temperature-grid temperature; all in place.
 */
ps_status rk3_step_mr(ps_mr_t mr, double dt, double cfl_target, double dt_max, double nu, double kappa,
                      double* u, double* v, double* w, double* p, double* tf, double* dt_used,
                      void* stream, ps_info* info);

/*
 * ps_debug_stage - run one stage of poisson_solve on the plan's own layout
 * (test and measurement entry; same kernels as poisson_solve).
 *   stage 0: forward x FFT   f (nz x ny x nx FP64)     -> spectral buffer A
 *   stage 1: forward y FFT   spectral A                 -> spectral buffer B
 *   stage 2: z solves        spectral B -> out (incl. the (0,0) column); the kernels
 *            run as in poisson_solve: from B into A where the solve works out of place
 *            (FP64 register-tile path), else in place in B.  With out NULL the result
 *            stays in that buffer.
 *   stage 3: inverse y FFT   spectral B                 -> spectral A
 *   stage 4: inverse x FFT   spectral A                 -> phi (FP64)
 * in/out: device pointers; spectral buffers are complex (FP64 pairs for
 * PS_FP64, FP32 pairs otherwise) of ps_spectral_elems() elements in the
 * tiled layout ps_spectral_layout() describes.  NULL selects the plan's own
 * buffer for a spectral argument.
 */
ps_status ps_debug_stage(ps_plan_t plan, int stage, const void* in, void* out, void* stream);

/*
 * ps_spectral_layout - the tiled spectral layouts:
 *   buffer A (after the x FFT): [nz][nkxb][ny][W]
 *   buffer B (after the y FFT): [nkxb][ny][nz][W]
 * with kx = kxb*W + w, kx in [0, nx/2]; columns kx > nx/2 are padding.
 */
ps_status ps_spectral_layout(ps_plan_t plan, int* w_tile, int* nkxb);
size_t ps_spectral_elems(ps_plan_t plan);

/*
 * ps_stream_copy - dst[0..bytes) = src[0..bytes) on the device (16-byte
 * non-temporal loads and stores).  A measurement utility: the HBM rate of a
 * plain one-read / one-write pass, the practical ceiling of the solve's
 * stages.  src, dst: 16-byte aligned, not overlapping.  Asynchronous.
 */
ps_status ps_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

const char* ps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PS_H */
