/*
 * dgnp -- C ABI of the MI355X (gfx950) solver for the discontinuous-Galerkin
 * discretisation of the charge-conservation Nernst-Planck (CNP) equations of
 * arXiv 2112.09271 ("A scalable DG solver for the electroneutral
 * Nernst-Planck equations").
 *
 * Problem (paper Sec. 2.2, Eqs. NP2, charge2, substitution; nondimensional
 * form of Sec. 2.3): m ions with valences z_k and diffusivities D_k; ion m is
 * eliminated by electroneutrality, c_m = -(1/z_m) sum_{k<m} z_k c_k.  The
 * unknowns are phi and c_1..c_{m-1} in the broken space V_h^p of tensor-product
 * polynomials of degree p per axis on a structured box of hexahedra (d = 3) or
 * quadrilaterals (d = 2).  The discrete residual is Eqs. NPDG / chargeDG
 * (Sec. 3.3): SIPG diffusion with penalty C_IP p^2/h (Eq. deltap, h = cell
 * diameter), upwinded advection-migration with q_k = u - z_k D_k grad phi,
 * SIPG potential with the concentration-dependent conductivity
 * kappa = sum_k z_k (z_k D_k - z_m D_m) c_k.
 *
 * Conventions common to every call:
 *  - Vectors are caller-owned DEVICE buffers of length N = m * N_f, field-major:
 *    index = f * N_f + e * n_b + l with f = 0 for phi, f = k for c_k;
 *    e = ix + nx*(iy + ny*iz); l = a + (p+1)*(b + (p+1)*c) over the
 *    Gauss-Lobatto nodes of the element (a along x).  N_f = E * n_b,
 *    n_b = (p+1)^d.  Element/face tables follow the same order.
 *  - `prec` selects the arithmetic of a vector argument: DGNP_F64 (double)
 *    or DGNP_F32 (float).  The residual is always double.
 *  - `stream` is a hipStream_t (NULL = default stream).  Apply calls are
 *    stream-ordered and return without synchronising.  dgnp_setup,
 *    dgnp_set_state, dgnp_solve and dgnp_adjoint synchronise.
 *  - Every call returns a DGNP_* status; no C++ exception crosses the ABI.
 *    dgnp_last_error() returns the text of the last failure on this thread.
 *  - The library never keeps a caller pointer after returning (apart from the
 *    allocator hook of dgnp_options).  The context owns all device workspace
 *    (hipMalloc, or the caller's allocator hook) and frees it in dgnp_destroy.
 *  - One context per host thread at a time.
 */
#ifndef DGNP_H
#define DGNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DGNP_OK = 0,
  DGNP_E_ARG = 1,        /* invalid argument (sizes, enums, NULL pointers) */
  DGNP_E_ALLOC = 2,      /* device or host allocation failed */
  DGNP_E_HIP = 3,        /* a HIP runtime call failed */
  DGNP_E_STATE = 4,      /* call order violated (e.g. apply before set_state) */
  DGNP_E_NOCONV = 5,     /* Newton / Krylov did not reach the tolerance */
  DGNP_E_BREAKDOWN = 6,  /* Krylov breakdown or line-search failure */
  DGNP_E_NONFINITE = 7   /* NaN/Inf met in a residual or norm */
};
enum { DGNP_F64 = 0, DGNP_F32 = 1 };
/* flags OR-ed into the `prec` of dgnp_set_state: ASSEMBLE_ONLY assembles the
 * blocks but skips the factorisations and the multigrid setup (block
 * inspection); APPLY_ONLY stores the linearisation point for
 * dgnp_jacobian_apply and builds no preconditioner at all. */
enum { DGNP_STATE_ASSEMBLE_ONLY = 0x100, DGNP_STATE_APPLY_ONLY = 0x200 };
/* boundary kinds per box face, faces tagged 0..5 = x-, x+, y-, y+, z-, z+ */
enum { DGNP_C_WALL = 0, DGNP_C_DIRICHLET = 1, DGNP_C_INFLOW = 2, DGNP_C_OUTFLOW = 3, DGNP_C_ELECTRODE = 4 };
/* exchange-current profile of electrode faces across the box in z: constant,
 * or the parabola of Sec. 5.2, 0.6 (2 - ((z - z_mid) / (w / 2))^2) with mean 1
 * over the box's z extent w (3-D only) */
enum { DGNP_J0_CONST = 0, DGNP_J0_PARABOLIC_Z = 1 };
/* objectives of dgnp_objective / dgnp_adjoint: 0 the outflow flux of species 1
 * through the x = x_max face; 1 the reaction rate g of the reacting ion
 * integrated over the first electrode face (the electrode's current over its
 * valence) */
enum { DGNP_OBJ_OUTFLOW = 0, DGNP_OBJ_ELECTRODE = 1 };
enum { DGNP_PHI_NEUMANN0 = 0, DGNP_PHI_DIRICHLET = 1 };
/* concentration-block preconditioners (dgnp_options.conc_pc) */
enum { DGNP_CPC_BILU = 0, DGNP_CPC_GMG = 1 };
/* velocity u = Pe * u_hat(x):
 *   VORTEX        u_hat = (sin(pi x) cos(pi y), -cos(pi x) sin(pi y), 0)
 *   POISEUILLE_X  u_hat = (6 y'(H - y')/H^2, 0, 0), y' = y - lo[1], H = hi[1] - lo[1]
 *   CONST         u_hat = (param[0], param[1], param[2])                         */
enum { DGNP_VEL_VORTEX = 0, DGNP_VEL_POISEUILLE_X = 1, DGNP_VEL_CONST = 2 };
/* built-in manufactured solutions (m = 2 only); they supply the volume sources
 * and all Dirichlet data:
 *   TRIG2D   c1 = 1 + sin(pi x) sin(pi y)/2,  phi = cos(pi x) cos(pi y)/10
 *   PAPER3D  c1 = cos x + sin y + 3,          phi = sin x + cos y + 3 (Sec. 5.1) */
enum { DGNP_MMS_NONE = 0, DGNP_MMS_TRIG2D = 1, DGNP_MMS_PAPER3D = 2 };
/* block-triangular preconditioner order (Sec. 4.1 Eq. P1, Sec. 4.2 Eq. P2) */
enum { DGNP_PC_P2 = 0, DGNP_PC_P1 = 1 };

typedef struct dgnp_ctx dgnp_ctx; /* opaque; owned by the library */

typedef struct {
  int32_t dim;        /* 2 or 3 */
  int32_t n[3];       /* elements per axis (n[2] ignored when dim = 2) */
  double lo[3], hi[3];
  int32_t c_bc[6];    /* DGNP_C_* per box face (all concentrations alike) */
  int32_t phi_bc[6];  /* DGNP_PHI_* per box face */
  double phi_val[6];  /* potential on DIRICHLET faces (ignored with a manufactured solution) */
} dgnp_mesh;

typedef struct {
  int32_t m;          /* number of ions, 2 or 3; ion m is eliminated (z[m-1] != 0) */
  const double *z;    /* host [m] valences */
  const double *D;    /* host [m] nondimensional diffusivities (> 0) */
} dgnp_species;

typedef struct {
  int32_t kind;       /* DGNP_VEL_* */
  double Pe;          /* velocity scale */
  double param[3];    /* CONST direction */
} dgnp_velocity;

/* Butler-Volmer electrodes (Sec. 2.1 Eqs. electrode and bv, nondimensional
 * form of Sec. 2.3): on a face tagged DGNP_C_ELECTRODE the reacting ion r, the
 * oxidant of a one-step redox reaction whose reductant has constant
 * concentration (the electrode metal, Sec. 5.2), reacts at the rate
 *   g = J0 [exp(alpha_a (phi_app - phi)) - c_r exp(-alpha_c (phi_app - phi))]
 * (gamma = 1; alpha_a, alpha_c are the products alpha n); g enters the
 * equation of ion r as -int g v (when r < m) and the charge equation as
 * -int z_r g v.  The potential is free on electrode faces (phi_bc must be
 * DGNP_PHI_NEUMANN0 there); the velocity is expected tangential. */
typedef struct {
  int32_t ion;            /* reacting ion, 1..m (m: the eliminated one) */
  double alpha_a, alpha_c;
  double j0[6];           /* exchange current per box face (amplitude of the profile) */
  double phi_app[6];      /* applied potential per box face */
  int32_t j0_profile;     /* DGNP_J0_* */
} dgnp_electrode;

typedef struct {
  double c_ip;             /* interior-penalty constant C_IP (paper: 10) */
  int32_t mms;             /* DGNP_MMS_* */
  const double *bc_conc;   /* host [m-1][n_bnode] nodal data on DIRICHLET / INFLOW
                              faces (ignored with a manufactured solution); order:
                              box faces 0..5, element faces by element index,
                              face nodes with the lower tangential axis fastest */
  int32_t phi_mg;          /* potential-block multigrid, DGNP_PHIMG_*:
                              Q1: smooth the assembled order-p block and start the
                              coarse levels at the trilinear (Q1) Galerkin operator;
                              P (orders 2, 3): p-multigrid (paper Sec. 4.2), the
                              order-p level smoothed matrix-free and the next level
                              the same DG discretisation at p = 1 (penalty for
                              p = 1, state injected at the element corners), then
                              the Q1 and smoothed-aggregation levels;
                              PG (orders 2, 3): as P, with the p = 1 level the
                              Galerkin product P^T A_p P of the order-p block;
                              AUTO (0, the default): Q1 for p <= 2, PG for p = 3 */
  /* Optional data of a forced or manufactured problem, copied at setup (NULL:
   * none).  Gauss points per axis: nq = p + 2; volume point q = qx + nq (qy +
   * nq qz); face point qf = qi + nq qj, qi along the face's first tangential
   * axis (x-faces: y, y- and z-faces: x), qj along the second (x- and
   * y-faces: z, z-faces: y); boundary faces in the order of the box faces
   * 0..5, then by element index. */
  const double *src_vol;   /* host [m][E][nq^d]: volume sources at the Gauss points,
                              field 0 the charge equation (S_phi), field k species k;
                              they enter the residual as -int S_f v */
  const double *dir_face;  /* host [m][n_bface][nq^(d-1)]: boundary data at the face
                              Gauss points of every boundary face: field 0 the
                              potential on potential-Dirichlet faces, field k the
                              concentration c_k on DIRICHLET / INFLOW faces (other
                              entries are not read); replaces bc_conc and phi_val.
                              dgnp_set_params and the boundary-data gradient of
                              dgnp_adjoint are then unavailable (DGNP_E_ARG) */
  /* Optional device allocator for the context's workspace (for instance
   * PyTorch's caching allocator): both or neither of alloc and free_.  alloc
   * returns a device pointer of at least `bytes` bytes on the context's device,
   * aligned to 256 bytes, or NULL (the call then fails with DGNP_E_ALLOC);
   * free_ releases it (the library synchronises its streams before freeing
   * memory that kernels may still use).  Used for allocations made on the
   * calling thread during calls on this context; NULL: hipMalloc / hipFree. */
  void *(*alloc)(size_t bytes, void *alloc_ctx);
  void (*free_)(void *ptr, void *alloc_ctx);
  void *alloc_ctx;
  const dgnp_electrode *electrode;  /* required when a face is DGNP_C_ELECTRODE, else NULL */
  /* Concentration-block preconditioner (Sec. 4.1), DGNP_CPC_*: BILU (0, the
   * default) one block-ILU(0) solve per concentration block; GMG one V-cycle
   * of geometric multigrid per block: the box coarsened by 2 along every axis
   * while every element count is even (down to one element where they allow),
   * Galerkin coarse operators with the nested DG prolongation, gmg_nu
   * Richardson steps with the level's block ILU(0) before and after the coarse
   * correction, and the coarsest level solved with its dense inverse (at most
   * 1024 unknowns per field: DGNP_E_ARG otherwise). */
  int32_t conc_pc;
  int32_t gmg_nu;          /* smoothing steps per side, 1..8; 0: 2 */
} dgnp_options;
enum { DGNP_PHIMG_AUTO = 0, DGNP_PHIMG_Q1 = 1, DGNP_PHIMG_P = 2, DGNP_PHIMG_PG = 3 };

typedef struct {
  double rtol;        /* Newton stop: ||R(x)||_2 <= rtol * ||R(x_0)||_2 */
  double atol;        /* ... or ||R(x)||_2 <= atol */
  int32_t max_newton;
  int32_t prec;       /* DGNP_F64, or DGNP_F32 = FP32 apply + preconditioner under
                         FP64 Newton residual, FP64 Arnoldi and FP64 iterative refinement */
  double lin_rtol;    /* outer FGMRES tolerance per Newton step (paper: 1e-3) */
  int32_t restart;    /* FGMRES restart length, 1..120 */
  int32_t max_lin_it; /* FGMRES iterations per linear solve */
  int32_t pc_kind;    /* DGNP_PC_P2 or DGNP_PC_P1 */
  int32_t verbose;
} dgnp_solve_opts;

#define DGNP_MAX_HIST 64
typedef struct {
  int32_t newton_its;
  int32_t lin_its_total;       /* FGMRES iterations over all Newton steps */
  int32_t refine_its_total;    /* iterative-refinement passes (mixed precision) */
  int32_t status;
  double res0, res_final;      /* ||R(x_0)||_2, ||R(x)||_2 */
  double t_total, t_setup, t_krylov; /* seconds: whole call, set_state, FGMRES */
  double res_hist[DGNP_MAX_HIST];
  int32_t lin_its[DGNP_MAX_HIST];
} dgnp_solve_stats;

/* Sets up the DG discretisation of Sec. 3.3 (Eqs. NPDG and chargeDG, the
 * nondimensional model of Sec. 2.3 in the charge-conservation form of
 * Sec. 2.2) on a structured box of hexahedra of order p (Sec. 4: tensor-product
 * elements): mesh/face/DOF tables, reference tables (Gauss-Lobatto nodes, p+2
 * Gauss points per axis), boundary data (Sec. 2.1 boundary conditions;
 * Butler-Volmer faces Eqs. electrode and bv) and the symbolic part of the
 * block preconditioner of Sec. 4.1 / 4.2; uploads them on `stream`.
 * order = p in 1..3.  The caller's arrays are copied; *out receives the new
 * context (owned by the library until dgnp_destroy).  Errors: DGNP_E_ARG for
 * unsupported sizes or kinds and for a potential that no face fixes,
 * DGNP_E_NONFINITE for non-finite data, DGNP_E_ALLOC / DGNP_E_HIP. */
int dgnp_setup(const dgnp_mesh *mesh, int32_t order, const dgnp_species *sp,
               const dgnp_velocity *vel, const dgnp_options *opt, void *stream,
               dgnp_ctx **out);

/* Replaces the problem parameters that the adjoint differentiates: the nodal
 * boundary data (host [m-1][n_bnode], same order as dgnp_options.bc_conc; may
 * be NULL to keep them) and the velocity scale Pe.  Invalidates the
 * linearisation point.  DGNP_E_ARG with a manufactured solution. */
int dgnp_set_params(dgnp_ctx *ctx, const double *bc_conc, double Pe);

/* Replaces the exchange currents and applied potentials of the electrode
 * faces (the other fields of e must equal those given at setup).  Invalidates
 * the linearisation point.  DGNP_E_ARG without electrode faces. */
int dgnp_set_electrode(dgnp_ctx *ctx, const dgnp_electrode *e);

/* Sizes: E elements, N_f = E * n_b DOFs per field, m fields, n_bnode nodal
 * boundary-data entries per concentration.  Any pointer may be NULL. */
int dgnp_sizes(const dgnp_ctx *ctx, int64_t *E, int64_t *n_dof_field,
               int32_t *n_fields, int64_t *n_bnode);

/* Host copies of the mesh tables (any pointer may be NULL):
 *   elem_nbr   [E][2d]  neighbour across slot (x-, x+, y-, y+, z-, z+) or -1
 *   face_elems [F][2]   interior faces: lower ("-") and upper ("+") element;
 *                       all x-normal faces by lower element, then y, then z
 *   face_axis  [F]      normal axis of each interior face
 * dgnp_n_faces gives F.                                                       */
int dgnp_n_faces(const dgnp_ctx *ctx, int64_t *n_interior, int64_t *n_boundary);
int dgnp_connectivity(const dgnp_ctx *ctx, int32_t *elem_nbr, int32_t *face_elems,
                      int32_t *face_axis);

/* r = R(x), Eqs. NPDG / chargeDG.  x, r: device double [N]. */
int dgnp_residual(dgnp_ctx *ctx, const double *x, double *r, void *stream);

/* r = dR/dPe at x (exact derivative of the residual with respect to the
 * velocity scale, |s|' = sign(s), sign(0) = 0).  Device double [N]. */
int dgnp_residual_dpe(dgnp_ctx *ctx, const double *x, double *r, void *stream);

/* Sets the linearisation point x (device double [N]) of the Newton step
 * (Sec. 4, Eq. blockmatrix): stores x (and a float copy), tabulates the
 * state at the quadrature points for the Jacobian apply, assembles the
 * diagonal field blocks A_phiphi, A_ckck on the device, and builds the
 * preconditioner of Sec. 4.1 / 4.2: element-block ILU(0) of every A_ckck (or
 * their multigrid levels with conc_pc = DGNP_CPC_GMG) and the multigrid
 * hierarchy of A_phiphi.  prec = DGNP_F32 also prepares float copies of all of
 * it (the mixed-precision solve).  The flags DGNP_STATE_APPLY_ONLY (tables
 * only, no preconditioner) and DGNP_STATE_ASSEMBLE_ONLY (blocks without
 * factorisation) may be or-ed into prec.  x is read during the call only.
 * Synchronises.  Errors: DGNP_E_ARG, DGNP_E_BREAKDOWN (singular coarsest
 * multigrid level), DGNP_E_ALLOC / DGNP_E_HIP. */
int dgnp_set_state(dgnp_ctx *ctx, const double *x, int32_t prec, void *stream);

/* y = J(x) v (transpose = 0) or y = J(x)^T v (transpose = 1), matrix-free,
 * at the point of the last dgnp_set_state (Sec. 4, Eq. blockmatrix).  v, y:
 * device [N] of the type `prec` names.  DGNP_E_STATE before set_state. */
int dgnp_jacobian_apply(dgnp_ctx *ctx, const void *v, void *y, int32_t prec,
                        int32_t transpose, void *stream);

/* y = A_phiphi v, the potential-potential block of J at the point of the last
 * dgnp_set_state (the derivative of the charge equation, Eq. chargeDG, with
 * respect to the potential; Sec. 4.2 smooths with it): kind =
 * DGNP_PHIOP_ASSEMBLED multiplies the assembled element blocks, kind =
 * DGNP_PHIOP_MATFREE applies it matrix-free (3-D, with phi_mg = P or PG, where
 * p-multigrid uses it).  v, y: device [E * nb] (the potential part) of the
 * type `prec` names.  DGNP_E_STATE before a set_state that built the potential
 * part of the preconditioner in that precision, DGNP_E_ARG for a matrix-free
 * request the context does not provide. */
enum { DGNP_PHIOP_ASSEMBLED = 0, DGNP_PHIOP_MATFREE = 1 };
int dgnp_phi_apply(dgnp_ctx *ctx, const void *v, void *y, int32_t prec, int32_t kind, void *stream);

/* y = A_phi,c v_c: the potential rows of J(x) applied to the concentration
 * part of v (the coupling block that Eq. P2 of Sec. 4.2 subtracts from the
 * potential right-hand side; the potential part of v is not read), at the
 * point of the last dgnp_set_state.  v: device [N] of type `prec`; y: device
 * [E * nb] (the potential rows).  DGNP_E_STATE before set_state. */
int dgnp_coupling_apply(dgnp_ctx *ctx, const void *v, void *y, int32_t prec, void *stream);

/* z = P r, the block-triangular preconditioner (Eq. P2 when pc_kind =
 * DGNP_PC_P2, Eq. P1 otherwise): one element-block ILU(0) solve per
 * concentration block, one AMG V-cycle on the potential block, coupling
 * blocks applied matrix-free.  transpose = 1 applies P^T.  r, z: device [N] of
 * type `prec`.  DGNP_E_STATE before set_state. */
int dgnp_precond_apply(dgnp_ctx *ctx, const void *r, void *z, int32_t prec,
                       int32_t transpose, int32_t pc_kind, void *stream);

/* Newton with backtracking line search (Sec. 4) around right-preconditioned
 * FGMRES with FP64 classical Gram-Schmidt (twice).  x: device double [N]; on
 * entry an initial guess, or all-NaN to request the paper's initial guess
 * (Sec. 4.3: constant concentrations = mean boundary data, potential from
 * the charge equation at those concentrations); on exit the solution.
 * opts may be NULL (defaults: rtol 1e-8, lin_rtol 1e-3, restart 120, P2, FP64).
 * stats may be NULL.  Synchronises.  DGNP_E_NOCONV if max_newton is reached. */
int dgnp_solve(dgnp_ctx *ctx, double *x, const dgnp_solve_opts *opts, dgnp_solve_stats *stats);

/* Adjoint of objective J (DGNP_OBJ_*: 0 the outflow flux
 * int_{x = x_max} (q_1 . n) c_1 ds, 1 the first electrode's reaction rate)
 * at the converged state x (device double [N]): solves
 * J(x)^T lambda = dJ/dx with FGMRES using the transposed
 * Jacobian apply and the transposed preconditioner, then
 *   dJ/d(bc data) = -lambda^T dR/d(bc data)      host double [m-1][n_bnode]
 *   dJ/dPe        = dJ/dPe|_x - lambda^T dR/dPe   host double [1]
 * J_out (host [1]) receives J(x); lambda (device double [N]) may be NULL.
 * Synchronises. */
int dgnp_adjoint(dgnp_ctx *ctx, const double *x, int32_t objective, double *dJ_dbc,
                 double *dJ_dPe, double *J_out, double *lambda, const dgnp_solve_opts *opts,
                 dgnp_solve_stats *stats);

/* Gradient of objective `objective` with respect to the exchange currents
 * and applied potentials of the electrode faces, from the adjoint solution
 * lambda of that objective at x (both device double [N], lambda from
 * dgnp_adjoint): dJ/dtheta = dJ/dtheta|_x - lambda^T dR/dtheta, host double
 * [6] each (zero on faces without an electrode).  Synchronises. */
int dgnp_electrode_gradient(dgnp_ctx *ctx, const double *x, int32_t objective, const double *lambda,
                            double *dJ_dj0, double *dJ_dphi_app);

/* J(x) at x (device double [N]) into host J_out: objective 0 =
 * int_{x = x_max} (q_1 . n) c_1 ds, objective 1 = the reaction rate integrated
 * over the first electrode face (DGNP_OBJ_*).  Synchronises. */
int dgnp_objective(dgnp_ctx *ctx, const double *x, int32_t objective, double *J_out);

/* Allocation-free form of dgnp_objective, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): J(x) at x (device double [N]) into J_dev (a
 * caller-owned device double [1]), stream-ordered on `stream`, with no
 * synchronisation and no allocation.  Its per-element partial sums live in a
 * static device array of the library (2^20 doubles, 8 MiB, held on each GPU
 * the library runs on until the process ends), so problems of at most 2^18 =
 * 262,144 elements are accepted (DGNP_E_ARG beyond).  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU race.  objective:
 * DGNP_OBJ_*. */
int dgnp_objective_noalloc(dgnp_ctx *ctx, const double *x, int32_t objective, double *J_dev, void *stream);

/* Copies the assembled block (field f, element e, slot s: 0 = diagonal,
 * 1 + j = coupling to neighbour slot j) of the last set_state into host
 * double [n_b][n_b] (row = test function).  For tests and diagnostics. */
int dgnp_get_block(dgnp_ctx *ctx, int32_t field, int64_t elem, int32_t slot, double *out);

/* Per-kernel event timing.  dgnp_profile(ctx, 1) makes the library record HIP
 * events around its kernels on the stream they run on (small overhead per
 * launch); dgnp_timer returns the summed device time in seconds and the number
 * of launches of one region since the last reset (reset != 0 clears all).
 * Region names: residual, jac_apply, jac_apply_f32, jacT_apply, jacT_apply_f32,
 * assemble, block_inverse, ilu_factor, ilu_fwd, ilu_bwd, ilu_fwdT, ilu_bwdT,
 * ilu_fwd_f32, ilu_bwd_f32, ilu_fwdT_f32, ilu_bwdT_f32, vcycle, vcycle_f32,
 * bspmv, bspmv_f32, cgs2. */
int dgnp_profile(dgnp_ctx *ctx, int32_t enable);
int dgnp_timer(dgnp_ctx *ctx, const char *name, double *seconds, int64_t *calls, int32_t reset);

void dgnp_destroy(dgnp_ctx *ctx);
const char *dgnp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGNP_H */
