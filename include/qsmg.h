/*
 * qsmg.h -- C ABI of the quasi-static projection library for AMD MI355X (gfx950).
 *
 * The library implements the hot path of the three-dimensional quasi-static
 * projection method for hypo-elastoplastic solids (Boffi & Rycroft,
 * "Parallel three-dimensional simulations of quasi-static elastoplastic
 * solids"): the geometric-multigrid solve of the velocity system (Sec. 3.3,
 * Eq. proj; Sec. 3.6) and the pointwise STZ plastic update that feeds it
 * (Sec. 3.1, Eqs. stz_dpl, stz_C_form, chi_evo; Sec. 3.3, Eq. sig_star_qs).
 *
 * Grid and layouts (all arrays C order, device memory unless stated):
 *   cells nx * ny * nz, spacing h; x and y periodic; cell (i,j,k) has its
 *   lower corner at node (i,j,k) (Sec. 3.5).  Nodes i < nx, j < ny,
 *   0 <= k <= nz; the planes k = 0 and k = nz are Dirichlet walls (Sec. 4).
 *   node vector   double[3][nz+1][ny][nx]   components (x, y, z)
 *   cell tensor   double[6][nz][ny][nx]     Voigt order (xx, yy, zz, yz, xz, xy)
 *   cell scalar   double[nz][ny][nx]
 *
 * Linear system.  K v := -div(C : grad v), discretised at the nodes with the
 * collocated second difference (Eq. col_snd_deriv) and the four-point mixed
 * difference (Sec. 3.4); C is homogeneous isotropic with Lame parameters
 * lambda, mu (Sec. 2.1).  K is symmetric positive definite (Sec. 3.3) and
 * couples each node to its 3x3x3 neighbourhood with 3x3 blocks (Sec. 3.6).
 * The projection system is K v = D_h sigma* / dt (Eq. proj times -1/dt),
 * D_h the staggered divergence (Eq. stag_stenc, shifted to the nodes).
 *
 * Ownership.  Every array argument is caller-owned.  The library allocates
 * no device memory: its hierarchy lives in a caller-provided device
 * workspace of qs_workspace_bytes() bytes that must stay valid until
 * qs_destroy().  The handle itself (host memory, plus a few bytes of pinned
 * host memory into which the device writes the residual norms) is owned by
 * the library.
 *
 * Streams.  All work is enqueued on the stream given to qs_setup() (a
 * hipStream_t passed as void*; NULL = default stream).  Entry points that
 * return host-visible results (qs_mg_solve, qs_projection_step) wait for that
 * stream once per V-cycle (the calling thread polls it) to read the residual
 * norm; the others are asynchronous.  Calls on one handle must not overlap.
 *
 * Errors.  Every entry point returns a qs_status; nothing is thrown and the
 * process is never aborted.  On QS_ERR_HIP the stream may hold partial work.
 *
 * Alignment.  Node vectors handed to qs_mg_solve (b, x), qs_projection_step
 * (v), qs_smooth (x, b), qs_level_restrict (r) and qs_level_prolong_add (x)
 * must be 16-byte aligned, as every device allocation is (an offset view may
 * not be); otherwise those entry points return QS_ERR_ARG.
 */
#ifndef QSMG_H
#define QSMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QS_OK = 0,
  QS_ERR_ARG = -1,            /* null pointer, bad enum, negative size          */
  QS_ERR_SHAPE = -2,          /* grid not coarsenable / too small / too large   */
  QS_ERR_HIP = -3,            /* a HIP runtime call failed                       */
  QS_ERR_NOT_CONVERGED = -4,  /* max_cycles reached; x holds the last iterate   */
  QS_ERR_NONFINITE = -5,      /* a residual norm was NaN or Inf                  */
  QS_ERR_WORKSPACE = -6       /* workspace null, misaligned or too small         */
} qs_status;

typedef enum { QS_FP64 = 0, QS_FP32_IR = 1 } qs_precision;

/* Multigrid parameters (Sec. 3.6).  Coarsening halves every dimension while
 * nz > min_coarse_nz (at least 2); each coarsened level needs even nx, ny, nz
 * and at least 4 cells per dimension, while the coarsest level (the only one
 * when nz <= min_coarse_nz) may have odd sizes down to 2 cells per dimension;
 * it is solved with a dense FP64 inverse (at most QS_MAX_COARSE unknowns).  Kernels index arrays with 32-bit
 * integers, so 3 (nz+1) ny nx (node vector) and 6 nz ny nx (cell tensor)
 * must stay below 2^31 (512^3 passes, 640 x 640 x 1024 does not); larger
 * grids are refused with QS_ERR_SHAPE.  colour_order lists the 8 node
 * colours c = (i&1) + 2*(j&1) + 4*(k&1) in the order pre-smoothing visits
 * them; post-smoothing visits them in reverse. */
#define QS_MAX_COARSE 6144
typedef struct {
  int nx, ny, nz;          /* cells                                             */
  double h;                /* grid spacing                                      */
  double lambda, mu;       /* Lame parameters                                   */
  int min_coarse_nz;       /* default 8                                         */
  int n_pre, n_post;       /* Gauss-Seidel sweeps, default 2 and 2 (Sec. 3.6)   */
  int precision;           /* qs_precision                                      */
  int colour_order[8];     /* permutation of 0..7; e.g. {0,1,2,3,4,5,6,7}       */
} qs_params;

#define QS_HIST 64
typedef struct {
  int cycles;                      /* V-cycles performed                     */
  int levels;                      /* multigrid levels                       */
  double rel_res;                  /* final ||b_eff - K x|| / ||b_eff||      */
  double rel_res_hist[QS_HIST];    /* before cycle 0, after cycle 1, ...;
                                      NaN after a V-cycle with no residual
                                      check (FP32_IR, see qs_mg_solve)       */
} qs_solve_info;

/* STZ constants in units of stress E, time t_s = L/c_s and chi in e_z/k_B
 * (Table 1).  Eq. stz_dpl: tau0 D^pl = exp(-1/chi) exp(-delta_over_T)
 * cosh(beta sbar) (1 - s_y/sbar) for sbar > s_y, else 0. */
typedef struct {
  double s_y, tau0, beta, delta_over_T, c0, chi_inf;
  double dt;               /* quasi-static time step                           */
  double l_diff;           /* diffusion length l of Eq. chi_evo (units of L);
                              0 leaves the diffusion term out; the reverse-mode
                              entry points require 0                          */
  int n_sub;               /* plastic terms of qs_stz_step: 0 or 1, the single
                              step of Eq. sig_star_qs; M > 1, M sub-steps;
                              -1, a per-cell count; -2, backward Euler; the
                              reverse-mode entry points require 0 or 1        */
  int advect;              /* 0 (Eq. sig_star_qs) or 1: sigma* also carries
                              -dt (v . grad) sigma (qs_stz_step); the reverse-
                              mode entry points require 0                     */
  int chi_wall;            /* chi diffusion at the walls (qs_stz_step): 0, the
                              face to the ghost cell carries the mean of the
                              cell's D^pl and D^pl of the extrapolated ghost
                              state; 1, the wall faces carry no flux          */
} qs_stz_params;

typedef struct qs_handle qs_handle;

const char* qs_status_string(int status);

/* Text of the last HIP failure seen by this thread (the failing call and the
 * HIP error string), or "" if none. */
const char* qs_last_error(void);

/* Bytes of device workspace qs_setup needs for these parameters. */
qs_status qs_workspace_bytes(const qs_params* p, size_t* bytes);

/* Number of multigrid levels and the dimensions of level `level`. */
qs_status qs_level_dims(const qs_params* p, int level, int* nlev, int* nx, int* ny, int* nz);

/* Build the hierarchy (host FP64 Galerkin stencils per z-plane, A_k =
 * T^T A_{k-1} T, Sec. 3.6; dense inverse of the coarsest operator) and copy
 * it into `workspace` (device, 256-byte aligned, >= qs_workspace_bytes).
 * `stream` is a hipStream_t or NULL. */
qs_status qs_setup(const qs_params* p, void* workspace, size_t workspace_bytes,
                   void* stream, qs_handle** out);
qs_status qs_destroy(qs_handle* hd);

/* y = K x at the interior nodes (wall planes of x are Dirichlet data; wall
 * planes of y are set to 0).  FP64, level 0 operator. */
qs_status qs_apply(qs_handle* hd, const double* x, double* y);

/* Solve K x = b for the interior of x by V-cycles (Sec. 3.6) until
 * ||b_eff - K x||_2 <= rtol ||b_eff||_2 (b_eff = b - K_IB x_B, 2-norm over
 * the 3 nx ny (nz-1) interior unknowns), checked before each cycle (FP64) or
 * before each refinement step (FP32_IR: the FP64 residual, scaled, is the
 * right-hand side of up to six FP32 V-cycles, fewer when the last step's
 * contraction says fewer reach rtol; cycles counts V-cycles).
 * x: in = initial guess with the wall velocities in planes 0 and nz (never
 * written); out = solution.  Wall planes of b are ignored.  rtol <= 0 runs
 * exactly max_cycles cycles and returns QS_OK.  b_eff == 0 gives x = 0 and
 * 0 cycles.  `info` may be NULL.  K = K^T, so this is also the adjoint solve. */
qs_status qs_mg_solve(qs_handle* hd, const double* b, double* x, double rtol,
                      int max_cycles, qs_solve_info* info);

/* Pointwise STZ step at every cell (Sec. 3.1; Eq. sig_star_qs):
 * L = G_h v (velocity gradient at cell centres, Eq. stag_stenc),
 * sigma* = sigma + dt (L sigma + sigma L^T - tr(L) sigma - C : (D^pl/sbar) sigma_0),
 * chi'   = chi + (dt/c0) (2 sbar D^pl / s_y) (chi_inf - chi)
 *              + (dt/c0) l^2 div(D^pl grad chi)                (Eq. chi_evo),
 * the last term when l_diff = l > 0: the 7-point flux form over the six faces
 * of a cell, each face carrying the mean of D^pl in its two cells, divided by
 * h^2; x and y wrap; below the first and above the last cell layer a ghost
 * layer holds the linear extrapolation of sigma and chi from the two nearest
 * layers (Sec. 3.5), with D^pl evaluated on it (0 where the extrapolated chi
 * is not positive; with chi_wall = 1 the wall faces carry no flux instead).
 * D^pl, sbar and chi are those of step n.
 * Sub-steps (an extension; the paper takes the single step above): with
 * n_sub = M > 1, or n_sub = -1 and M = ceil(4 mu dt dD^pl/dsbar) at the state
 * of step n clamped to [1, 65536] per cell, the plastic terms take M forward-
 * Euler steps of dt/M, each from the state the previous one left:
 *   sigma_{m+1} = sigma_m - (dt/M) 2 mu (D^pl/sbar)(sigma_m) sigma_{0,m},
 *   chi_{m+1}   = chi_m + (dt/M)/c0 (2 sbar_m D^pl_m / s_y) (chi_inf - chi_m),
 * then sigma* = sigma_M + dt (L sigma + sigma L^T - tr(L) sigma) with sigma
 * of step n, and chi' = chi_M + the diffusion term above.  For n_sub = -1 each
 * sub-step keeps (dt/M) 2 mu dD^pl/dsbar <= 1/2 at the start state, below the
 * explicit step's stability limit of 2.  n_sub = -2 takes the plastic
 * terms by backward Euler instead (an extension, stable for any dt): with chi
 * held at step n, sbar' is the root of s - sbar + 2 mu dt D^pl(s, chi) in
 * [s_y, sbar] (64 bisections), the deviator shrinks by sbar'/sbar, the
 * pressure is kept, and chi_M = (chi + c chi_inf)/(1 + c) with
 * c = (dt/c0) 2 sbar' D^pl(sbar', chi) / s_y.  n_sub < -2: QS_ERR_ARG.
 * Advection (advect = 1; the stress equation of Eq. sig_star_evol carries it,
 * the quasi-static Eq. sig_star_qs leaves it out): sigma* -= dt (u . grad)
 * sigma with sigma and v of step n, u the mean of the cell's eight corner
 * velocities, and each derivative by Eq. ENO along its axis (upwind
 * three-point formula where the cell is more curved than its upwind
 * neighbour, centred difference otherwise); x and y wrap, and in z two ghost
 * layers continue the two nearest layers linearly (Sec. 3.5).  l > 0 or
 * advect = 1 need nz >= 2 (else QS_ERR_SHAPE).  With l > 0, D^pl of every
 * cell is first written into a fine-level buffer of the handle's workspace
 * that holds nothing between solves (calls on one handle must not overlap).
 * Outputs may not alias inputs. */
qs_status qs_stz_step(qs_handle* hd, const qs_stz_params* sp, const double* v,
                      const double* sigma, const double* chi, double* sigma_star,
                      double* chi_next);

/* b = D_h sigma* / dt at interior nodes (walls of b set to 0). */
qs_status qs_rhs(qs_handle* hd, const double* sigma_star, double dt, double* b);

/* sigma_out = sigma* + dt C : sym(G_h v) (Eq. sig_n+1).  May alias sigma_star. */
qs_status qs_stress_update(qs_handle* hd, const double* sigma_star, const double* v,
                           double dt, double* sigma_out);

/* One quasi-static step n -> n+1, in place (Sec. 3.3): STZ step, wall
 * velocities (-U,0,0) at k = 0 and (+U,0,0) at k = nz (Eq. u_bc), RHS,
 * solve warm-started from v^n, stress correction.  `scratch` is caller
 * device memory of qs_step_scratch_bytes() bytes. */
qs_status qs_step_scratch_bytes(qs_handle* hd, size_t* bytes);
qs_status qs_projection_step(qs_handle* hd, const qs_stz_params* sp, double U_wall,
                             double* v, double* sigma, double* chi, void* scratch,
                             double rtol, int max_cycles, qs_solve_info* info);

/* The same step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the step scratch comes from a fixed device array of the library instead of
 * a `scratch` argument.  Each GPU the library runs on holds that array
 * (QS_NOALLOC_SCRATCH_BYTES) until the process ends; its device address is
 * resolved for the current device in qs_setup.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the caller still
 * passes v, sigma and chi.  Grids whose step scratch,
 * (7 nx ny nz + 3 (nz+1) ny nx) doubles plus alignment (qs_step_scratch_bytes),
 * exceeds QS_NOALLOC_SCRATCH_BYTES are refused with QS_ERR_SHAPE (96 MiB holds
 * 96^3 or 128 x 128 x 64; not 128^3).  Every call on one GPU shares the array
 * and leaves its contents behind; each call writes all of it that it reads,
 * so nothing carries over between calls.  Calls that overlap on one GPU (on
 * any handles or streams) race on the array and must not be made.
 * QS_ERR_HIP if the array's address could not be resolved at setup.
 * Otherwise arguments, results and errors as qs_projection_step. */
#define QS_NOALLOC_SCRATCH_BYTES (96u * 1024u * 1024u)
qs_status qs_projection_step_noalloc(qs_handle* hd, const qs_stz_params* sp, double U_wall,
                                     double* v, double* sigma, double* chi, double rtol,
                                     int max_cycles, qs_solve_info* info);

/* The same step with wall velocities given node by node, for boundary data
 * that varies in x and y, such as the spinning discs of the friction-welding
 * runs (Sec. 5, Eqs. u_weld and v_weld): the planes k = 0 and k = nz of
 * v^{n+1} are copied from wall_lo and wall_hi, each double[3][ny][nx]
 * (components x, y, z; device memory, caller-owned, not overlapping v; a
 * fixed wall is passed as zeros).  The STZ step still sees the walls of v^n.
 * Errors as qs_projection_step; QS_ERR_ARG also for a null or overlapping
 * wall array. */
qs_status qs_projection_step_walls(qs_handle* hd, const qs_stz_params* sp,
                                   const double* wall_lo, const double* wall_hi, double* v,
                                   double* sigma, double* chi, void* scratch, double rtol,
                                   int max_cycles, qs_solve_info* info);

/* One forward-Euler step of the explicit method (Sec. 3.2), in place, every
 * term from the state of step n:
 *   v'     = v + dt ((D_h sigma)/rho - (v . grad) v + kappa lap v)
 *            at interior nodes (Eq. vel_evo_exp per unit mass: kappa is a
 *            kinematic viscosity, kappa = kappa' h in the paper's runs, with
 *            the bound dt <= h^2/(6 kappa)); the Laplacian by Eq. col_snd_deriv,
 *            the advection by Eq. ENO with the node's own velocity and a
 *            ghost node 2 v_wall - v past each wall (Sec. 3.5);
 *            walls (-U,0,0) at k = 0 and (+U,0,0) at k = nz (Eq. u_bc);
 *   sigma' = sigma* + dt C : sym(G_h v) with sigma* from qs_stz_step with
 *            advect = 1 (Eq. stress_evo_exp; Truesdell term -tr(L) sigma);
 *   chi'   = chi' of that STZ step (Eq. chi_evo_exp).
 * sp->advect is ignored (always on); n_sub and l_diff act as in
 * qs_stz_step.  rho > 0 is the density in units of E t_s^2 / L^2 (mu/E when
 * t_s = L / c_s).  `scratch`: qs_step_scratch_bytes() bytes, 256-aligned.
 * No solve and no host synchronisation; nz >= 2. */
qs_status qs_explicit_step(qs_handle* hd, const qs_stz_params* sp, double U_wall, double rho,
                           double kappa, double* v, double* sigma, double* chi, void* scratch);

/* Adjoint building blocks (reverse mode of one step; plain Euclidean inner
 * products on the stored arrays, so Voigt off-diagonals are single entries).
 *  qs_stz_step_vjp:      given g_sstar (6 cells) and g_chi1 (cells), return
 *                        g_sigma, g_chi (cells) and ADD the velocity
 *                        cotangent into g_v (node vector; walls untouched);
 *                        `scratch`: device memory of qs_step_scratch_bytes().
 *                        At sbar == s_y the one-sided derivative of the
 *                        elastic branch (D^pl = 0) is used.  Refuses l > 0,
 *                        n_sub outside {0, 1} or advect (QS_ERR_ARG) and grids with 9 nz ny nx >= 2^31
 *                        (QS_ERR_SHAPE: the gradient cotangent is indexed
 *                        with 32-bit integers as [9][cells]).
 *  qs_rhs_vjp:           g_sstar += D_h^T g_b / dt (g_b interior nodes).
 *  qs_stress_update_vjp: g_v += dt (C : sym G_h)^T g_sigma (interior nodes). */
qs_status qs_stz_step_vjp(qs_handle* hd, const qs_stz_params* sp, const double* v,
                          const double* sigma, const double* chi, const double* g_sstar,
                          const double* g_chi1, double* g_sigma, double* g_chi, double* g_v,
                          void* scratch);
qs_status qs_rhs_vjp(qs_handle* hd, const double* g_b, double dt, double* g_sstar);
qs_status qs_stress_update_vjp(qs_handle* hd, const double* g_sigma, double dt, double* g_v);

/* Test-facing pieces of the V-cycle on level `level` (arrays in the level's
 * node layout, FP64; the handle must have been set up with QS_FP64):
 *  qs_level_colour_pass: block Gauss-Seidel update of colour `colour`;
 *  qs_level_residual:    r = b - A_level x (interior);
 *  qs_level_restrict:    b_coarse = T^T r (level -> level+1);
 *  qs_level_prolong_add: x += T e_coarse (level+1 -> level);
 *  qs_coarse_solve:      x_interior = A_coarsest^{-1} (b - A x_walls). */
qs_status qs_level_colour_pass(qs_handle* hd, int level, double* x, const double* b, int colour);
qs_status qs_level_residual(qs_handle* hd, int level, const double* x, const double* b, double* r);
qs_status qs_level_restrict(qs_handle* hd, int level, const double* r, double* b_coarse);
qs_status qs_level_prolong_add(qs_handle* hd, int level, double* x, const double* e_coarse);
qs_status qs_coarse_solve(qs_handle* hd, double* x, const double* b);

/* `sweeps` full smoothing sweeps (colour order as given at setup) on level
 * `level`, in the handle's working precision: x and b are float for a
 * QS_FP32_IR handle and double otherwise, in the level's node layout.
 * Used to time the smoother on its own and to test it. */
qs_status qs_smooth(qs_handle* hd, int level, void* x, const void* b, int sweeps);

/* Copy the FP64 per-plane stencil of level `level` to host memory:
 * out[(nz+1)][27][3][3], offset index (oz+1)*9 + (oy+1)*3 + (ox+1). */
qs_status qs_level_stencil(qs_handle* hd, int level, double* out_host);

#ifdef __cplusplus
}
#endif
#endif /* QSMG_H */
