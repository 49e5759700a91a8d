/*
 * dfdg.h — C ABI of the MI355X explicit divergence-free DG library.
 *
 * Method: G. Fu, "An explicit divergence-free DG method for incompressible flow".
 * The library advances the velocity-only semi-discrete system
 *      M du/dt = L(u),   u in V_h^{k,-1} = { v in BDM_k : div v = 0 }          (Sec. 2.3)
 * with L(u)(v) = -C_h(u; u, v) - B_h(u, v): upwind convection (Sec. 2.2, eq. (adv))
 * plus symmetric interior-penalty viscosity with penalty nu*alpha*k^2/h (Sec. 3,
 * eq. (viscous)).  The divergence-free mass inversion M^{-1} is done as the
 * hybrid-mixed Poisson problem of eq. (FE3): element-local static condensation onto
 * facet multipliers, a global symmetric positive semi-definite facet system solved by
 * preconditioned CG, and element-local recovery (Theorem 2).  Time stepping is
 * TVD-RK3 (eq. (rk3)).  Triangle (d = 2) and tetrahedral (d = 3; the method is posed for
 * d = 2, 3, Sec. 2) meshes, periodic or with walls in the directions without period
 * (no-flow, eq. (euler-3) with g = 0; free-slip for nu > 0, eq. (ns-3)-(ns-4)), or with
 * inflow and outflow boundaries there (Sec. 2.5, dfdg_mesh_set_outflow).  The element-local unknowns of the condensation are
 * those of eq. (FE3) or, on triangles, the locally divergence-free ones of eq. (FE4)
 * (dfdg_params.local_space).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Ownership.  Pointers named *_dev are device pointers owned by the caller.  The
 *   library never allocates device memory: dfdg_ctx_workspace_bytes() reports the
 *   size of one workspace the caller allocates and hands over with
 *   dfdg_ctx_bind_workspace(); it must stay alive and untouched until
 *   dfdg_ctx_destroy().  Pointers named *_host are host pointers, read or written
 *   during the call only.  The library keeps one pinned host buffer per context.
 * Streams.  All device work of a context is enqueued on the HIP stream given to
 *   dfdg_ctx_create() (or dfdg_ctx_set_stream(), which first waits for the work
 *   queued on the previous stream).  Calls that return numbers to the host (solve/step
 *   info, diagnostics) wait for those numbers; work that does not feed them (the final
 *   recovery of a step, the next step's start values) may still be running on the
 *   stream when they return, like the work of the calls that only enqueue.
 * Errors.  Every int-returning function returns DFDG_OK (0) or a negative status.
 *   Arguments, mesh and workspace are validated on the host before any device work;
 *   dfdg_last_error() gives a message for the last failing call on a context,
 *   dfdg_mesh_last_error() for mesh creation.  A context is not thread safe.
 * Layouts (all FP64 unless stated).
 *   T elements, E facets, d the dimension, P = dim P^k(element) ((k+1)(k+2)/2 on
 *   triangles, (k+1)(k+2)(k+3)/6 on tetrahedra), n_f = dim P^k(facet) (k+1 on edges,
 *   (k+1)(k+2)/2 on faces).
 *   Velocity-like vectors (U, L, F, adjoints): [d][P][T] — component c, basis
 *   function i, element t at index (c*P + i)*T + t.  The basis of element t is
 *   psi_i(x) = psihat_i(xhat)/sqrt(|det J_t|) e_c, with psihat_i the L2-orthonormal
 *   Dubiner polynomials of the reference simplex, so the element mass matrix is the
 *   identity, kinetic energy is 0.5*sum(U^2), and a functional F is stored by its
 *   values F(psi_i e_c).  xhat are the reference coordinates with respect to the
 *   element's vertices as passed to dfdg_mesh_create: x = v0 + sum_r xhat_r (v_{r+1}-v0).
 *   Facet multipliers lambda: [E][n_f], coefficients in an L2(F)-orthonormal basis of
 *   P^k on the facet, in the parametrisation of the facet's first element (Legendre
 *   polynomials along an edge; the triangle's Dubiner polynomials on a face spanned from
 *   its lowest-numbered local vertex); the facet numbering is the library's (see
 *   dfdg_mesh_facets).
 */
#ifndef DFDG_H
#define DFDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DFDG_OK = 0,
  DFDG_E_INVALID_ARG = -1,  /* null pointer, out-of-range parameter, bad size */
  DFDG_E_MESH = -2,         /* unmatched facet, inverted or degenerate element */
  DFDG_E_WORKSPACE = -3,    /* workspace missing, too small or misaligned */
  DFDG_E_HIP = -4,          /* a HIP runtime call failed */
  DFDG_E_NOT_CONVERGED = -5,/* PCG hit its iteration limit (result still written) */
  DFDG_E_NONFINITE = -6,    /* NaN/Inf met in a reduction */
  DFDG_E_BREAKDOWN = -7,    /* non-positive curvature (p, S p) <= 0 in PCG */
  DFDG_E_UNSUPPORTED = -8   /* valid request this build does not implement */
};

enum { DFDG_FP64 = 0, DFDG_MIXED = 1 };            /* dfdg_params.precision */
#define DFDG_HISTORY_DEPTH 6  /* earlier multipliers kept per stage for warm starts */
#define DFDG_EXTRAPOLATE_ADAPTIVE 5  /* dfdg_params.extrapolate: order chosen per solve */
#define DFDG_EXTRAPOLATE_PROJECT 6   /* dfdg_params.extrapolate: projection onto earlier solutions */
enum { DFDG_JACOBI = 0, DFDG_BLOCK_JACOBI = 1, DFDG_AMG = 2 };  /* dfdg_params.precond */
enum { DFDG_LOCAL_FE3 = 0, DFDG_LOCAL_FE4 = 1 };  /* dfdg_params.local_space */

typedef struct dfdg_mesh dfdg_mesh;
typedef struct dfdg_ctx dfdg_ctx;

typedef struct {
  int k;             /* polynomial degree of BDM_k, 1..3 */
  double nu;         /* viscosity >= 0 (0: Euler) */
  double alpha;      /* SIPG penalty constant, > 0 (the paper uses 2, Sec. 4) */
  int precision;     /* DFDG_FP64 or DFDG_MIXED */
  double cg_rtol;    /* PCG stop: ||g - S lambda||_2 <= cg_rtol ||g||_2 (FP64 path) */
  int cg_maxit;      /* PCG iteration limit per solve */
  int precond;       /* DFDG_JACOBI, DFDG_BLOCK_JACOBI, or DFDG_AMG: one smoothed-
                        aggregation multigrid V-cycle (Chebyshev(2) smoothing on the
                        finest level, one Chebyshev(1) step before and after the
                        correction on the coarser levels; coarse space spanned by the
                        constant multiplier; built on the host at context creation) */
  double ir_rtol;    /* MIXED: outer FP64 refinement target (relative residual) */
  double inner_rtol; /* MIXED, mixed_solver = 0: FP32 inner PCG reduction per refinement step */
  int extrapolate;   /* rk3_step: 0 = warm start from the last same-stage multiplier,
                        1..4 = polynomial extrapolation of that order in time from the
                        last extrapolate+1 steps, DFDG_EXTRAPOLATE_ADAPTIVE = the order
                        1..4 whose prediction of the last multiplier from the ones before
                        it was best (decided on the device per solve, among the orders the
                        DFDG_HISTORY_DEPTH kept multipliers allow), DFDG_EXTRAPOLATE_PROJECT
                        (FP64 contexts) = the element closest in the S-norm to the solution
                        among the combinations of up to 24 earlier forward stage solutions
                        (of any stage): an S-orthogonal basis of them, grown by two
                        Gram-Schmidt passes per solve and rebuilt from the latest 8 when
                        full; its start value needs the new right-hand side only.  Costs
                        65 vectors of n_lambda doubles of workspace.  The
                        adjoint's stage solves keep the extrapolation of order 4. */
  int graphs;        /* 1: replay PCG iterations from captured HIP graphs (default);
                        0: launch every kernel individually.  Same results bit for bit. */
  int mg_fp32;       /* DFDG_AMG with DFDG_FP64: 1 = run the V-cycle in FP32 (default; the
                        PCG vectors, residuals and stopping test stay FP64), 0 = FP64 */
  int mg_fine_fp16;  /* FP32 V-cycle (mg_fp32 = 1, or a DFDG_MIXED context): 1 = the
                        V-cycle's smoothing on the finest level
                        reads S stored in FP16 (scaled by the largest |S_ij|; arithmetic in
                        FP32), 0 = S in FP32.  The preconditioner then uses a symmetric
                        perturbation of S of relative size 2^-11; the PCG itself keeps the
                        FP64 S and its stopping test. */
  int facet_blocks;  /* blocks of 256 threads of the facet-row kernels: 0 = ceil(E/256) up to
                        1024 (default); 1..1024 = at most that many.  With fewer blocks
                        than rows/256, each thread walks several facet rows in a grid-
                        stride loop (the path every mesh above 262144 facets takes); the
                        results are the same up to the order of the partial sums. */
  int matrix_free;   /* tetrahedral meshes, FP64 PCG: 1 = form S p element by element as
                        sum_T C_T W_T C_T^T p from the element data (two passes, no matrix
                        read) instead of reading the assembled S; 0 = assembled S (default).
                        The multigrid smoothing still reads S.  Triangle meshes: must be 0. */
  int mixed_solver;  /* MIXED facet solves (the residual is FP32 in both):
                        1 = Krylov refinement (default): FP64 PCG iterations (FP64 S, vectors,
                        dot products, stopping test at ir_rtol) whose preconditioner, the
                        multigrid cycle, runs in FP32 (FP16 S on the finest level with
                        mg_fine_fp16); with Jacobi the FP32 part is the residual alone;
                        0 = restarted refinement: FP32 PCG on an FP32 copy of S to inner_rtol,
                        FP64 refinement residual g - S lambda, restarted until ir_rtol. */
  int mg_fine_smooth;/* DFDG_AMG: damped-Jacobi steps smoothing the finest level's tentative
                        prolongator, 1..3 (default 2; the coarser levels take one): more steps
                        give a wider interpolation, fewer PCG iterations and costlier
                        finest-level transfers (rows of up to 16 entries stay packed in FP16
                        when the next level has fewer than 65536 unknowns) */
  int local_space;   /* element-local unknowns of the condensation (triangle meshes):
                        DFDG_LOCAL_FE3 (default): broken [P^k]^2 velocity with the P^{k-1}
                        pressure w of eq. (FE3), the local projector applied as
                        I - D^T (D D^T)^{-1} D (per element: packed (D D^T)^{-1});
                        DFDG_LOCAL_FE4: the locally divergence-free velocity of eq. (FE4)
                        (remark "More efficient implementation", Sec. 2.4) without w, in the
                        basis Z_T = Piola image of the orthonormalised reference curls of
                        P^{k+1}, the projector applied as Z (Z^T Z)^{-1} Z^T (per element:
                        packed (Z^T Z)^{-1}, (2P-n_p)(2P-n_p+1)/2 doubles).  Same facet
                        system and velocity up to rounding.  Tetrahedral meshes: must be
                        DFDG_LOCAL_FE3 (else DFDG_E_UNSUPPORTED). */
} dfdg_params;

typedef struct {
  int32_t T, E, k, P, n_f, n_p;
  int64_t n_broken;   /* 2*P*T, length of velocity-like vectors */
  int64_t n_lambda;   /* n_f*E */
  int64_t n_bdm;      /* dim BDM_k = E*n_f + T*(d P - (d+1) n_f) */
  int32_t nq_proj;    /* points of the projection rule (dfdg_proj_rule) */
  int32_t dim;        /* d: 2 (triangles) or 3 (tetrahedra) */
} dfdg_sizes;

typedef struct {
  int iterations;      /* PCG iterations (FP64, and MIXED with the Krylov refinement) or the
                          total inner FP32 iterations (MIXED, restarted refinement) */
  int refinements;     /* MIXED: FP64 refinement steps (= the FP64 iterations of the Krylov
                          refinement); FP64: 0 */
  double rel_residual; /* final ||g - S lambda|| / ||g|| (FP64 recomputed for MIXED) */
  int status;          /* DFDG_OK, DFDG_E_NOT_CONVERGED, ... */
  double initial_rel_residual; /* ||g - S lambda_0|| / ||g|| of the start value (0 for a
                                  right-hand side at rounding level) */
} dfdg_solve_info;

typedef struct {
  int iterations[3];   /* PCG iterations of the three stages */
  int max_refinements;
  double max_rel_residual;
  int status;
  double initial_rel_residual[3]; /* of the three stage solves (warm-start quality) */
} dfdg_step_info;

typedef struct {
  int iterations[4];   /* PCG iterations of the four stage solves of dfdg_rk4_step */
  double max_rel_residual;
  int status;
} dfdg_rk4_info;

typedef struct {
  double energy;         /* 0.5 ||u_h||^2 */
  double enstrophy;      /* ||curl_h u_h||^2 (element-wise curl) */
  double max_div;        /* max |div u_h| over element quadrature points */
  double max_normal_jump;/* max |[[u_h . n]]| over facet quadrature points (on a closed
                            boundary facet |u_h . n|, the inflow speed on an inflow; outflow
                            facets are skipped) */
} dfdg_diag;

/* ---- mesh (host only; a0 of the hot path) ---------------------------------------
 * dfdg_mesh_create: dim = 2: elem_xyz_host[T][3][2] vertex coordinates of each triangle,
 * counter-clockwise and non-degenerate; dim = 3: elem_xyz_host[T][4][3] of each
 * tetrahedron, positively oriented (det[v1-v0, v2-v0, v3-v0] > 0).  period_host[dim]:
 * > 0 for a periodic direction (every facet must then match another one modulo the
 * period); 0 for a direction with walls, where the facets without a partner are boundary
 * facets (element R = -1 in dfdg_mesh_facets), closed (walls or inflows) unless
 * dfdg_mesh_set_outflow marks them as outflow.  On a wall the velocity space
 * has u.n = 0 (BDM_k in H_0(div), eq. (space-3)), enforced by the facet multiplier of the
 * boundary facet in the hybrid-mixed solve; the residual has no term there: the
 * convective flux vanishes with u.n, and the viscous facet terms of eq. (viscous) run
 * over interior facets only, which makes the free-slip condition (ns-4) natural (Sec. 3).
 * Facets are identified by their barycentres modulo the period; a local facet f is the
 * edge (f+1)%3 -> (f+2)%3 of a triangle, the face opposite vertex f of a tetrahedron.
 * Copies its inputs. */
int dfdg_mesh_create(int dim, int n_elem, const double* elem_xyz_host,
                     const double* period_host, dfdg_mesh** out);
void dfdg_mesh_destroy(dfdg_mesh* mesh);
const char* dfdg_mesh_last_error(void);
/* facets_host[E][4]: element L, local facet of L, element R, local facet of R (R and its
 * local facet -1 for a boundary facet). */
int dfdg_mesh_counts(const dfdg_mesh* mesh, int* T, int* E);
int dfdg_mesh_facets(const dfdg_mesh* mesh, int32_t* facets_host);
/* dfdg_mesh_set_outflow: marks boundary facets as an outflow boundary (Sec. 2.5):
 * open_host[E] (the library's facet numbering), 1 = outflow, 0 = closed; nonzero entries
 * only on boundary facets (else DFDG_E_INVALID_ARG, and the mesh is left unchanged); a
 * later call replaces the marks.  Contexts created afterwards use them.  A closed boundary
 * facet is a wall or an inflow boundary: its normal velocity is fixed, so the stage
 * increments have u.n = 0 there (an inflow's normal velocity u_in enters through the
 * initial state, which the stages keep; a caller builds it as a lift carrying u.n = u_in
 * plus the projection of the rest).  On an outflow facet the pressure is zero: it has no
 * multiplier (its row of the facet matrix is the identity with a zero right-hand side, so
 * the facet system has no kernel and no deflation) and u.n is free; the residual keeps
 * the outgoing convective flux -int max(u.n, 0) (u . v) with the element's own trace (the
 * exterior state of backflow is zero) and, as on every boundary, no viscous facet terms.
 * The normal-jump diagnostic skips outflow facets. */
int dfdg_mesh_set_outflow(dfdg_mesh* mesh, const int32_t* open_host);

/* ---- context --------------------------------------------------------------------
 * dfdg_ctx_create validates the parameters and does the host part of setup
 * (reference tabulations, geometry, condensation matrices, facet matrix).  On
 * tetrahedral meshes it accepts k = 1, 2, DFDG_FP64 and the Jacobi or block-Jacobi
 * preconditioner (other requests return DFDG_E_UNSUPPORTED).
 * hip_stream is a hipStream_t (NULL = default stream).  The mesh may be destroyed
 * afterwards. */
void dfdg_params_default(dfdg_params* p);
int dfdg_ctx_create(const dfdg_mesh* mesh, const dfdg_params* params, void* hip_stream,
                    dfdg_ctx** out);
int dfdg_ctx_set_stream(dfdg_ctx* ctx, void* hip_stream);
int dfdg_ctx_sizes(const dfdg_ctx* ctx, dfdg_sizes* out);
int dfdg_ctx_workspace_bytes(const dfdg_ctx* ctx, size_t* bytes);
/* dev_ptr: 256-byte aligned device memory of at least the reported size.  Uploads
 * the setup data (synchronous). */
int dfdg_ctx_bind_workspace(dfdg_ctx* ctx, void* dev_ptr, size_t bytes);
const char* dfdg_last_error(const dfdg_ctx* ctx);
void dfdg_ctx_destroy(dfdg_ctx* ctx);

/* ---- initial data (a2) ------------------------------------------------------------
 * dfdg_proj_rule: reference points ref_pts_host[nq_proj][d] and weights
 * w_host[nq_proj] of the projection rule (exact for degree 2k+4 on triangles, 2k+2 on
 * tetrahedra).
 * dfdg_load_vector: F(psi_i e_c) = int_T f . psi_i e_c for f given by its values
 * f_at_q_dev[d][nq_proj][T] at those points (element t's point q is
 * v0 + J xhat_q).  dfdg_project: load vector followed by dfdg_hdiv_mass_solve, i.e.
 * the L2 projection onto V_h^{k,-1} (Sec. 2.3, with u0 divergence free). */
int dfdg_proj_rule(const dfdg_ctx* ctx, double* ref_pts_host, double* w_host);
int dfdg_load_vector(dfdg_ctx* ctx, const double* f_at_q_dev, double* F_dev);
int dfdg_project(dfdg_ctx* ctx, const double* f_at_q_dev, double* U_dev,
                 dfdg_solve_info* info);

/* ---- hot path (a3-a7) -------------------------------------------------------------
 * dfdg_dg_residual: L_dev = L(U) on the broken basis, L(u)(v) = -C_h(u;u,v) -
 *   B_h(u,v) (eqs. (adv), (viscous)); upwinding per facet quadrature point on the
 *   averaged normal velocity.
 * dfdg_hdiv_mass_solve: U_dev = the u of eq. (FE3) for the functional F_dev, i.e. the
 *   divergence-free mass inversion of F (Theorem 2).  lambda_io_dev ([E][n_f]) is
 *   the PCG start on entry and the facet multiplier on exit, which is fixed up to a
 *   constant multiplier and returned orthogonal to it; NULL = cold start.
 *   Returns DFDG_E_NOT_CONVERGED/DFDG_E_BREAKDOWN if PCG failed (U_dev still written).
 * dfdg_rk3_step: one TVD-RK3 step of size dt, in place on U_io_dev (eq. (rk3));
 *   each stage is u + dt*M^{-1}L(u) combined as in the Shu-Osher form.  Multipliers of
 *   earlier steps warm-start the PCG of the same stage. */
int dfdg_dg_residual(dfdg_ctx* ctx, const double* U_dev, double* L_dev);
int dfdg_hdiv_mass_solve(dfdg_ctx* ctx, const double* F_dev, double* U_dev,
                         double* lambda_io_dev, dfdg_solve_info* info);
int dfdg_rk3_step(dfdg_ctx* ctx, double* U_io_dev, double dt, dfdg_step_info* info);
/* dfdg_rk4_step: one step of the classical four-stage RK4 (Sec. 4, Example 1b compares it
 *   with TVD-RK3) in place on U_io_dev: k_i = M^{-1}L(u_i) (one residual and one facet
 *   solve each), u_2 = u^n + dt/2 k_1, u_3 = u^n + dt/2 k_2, u_4 = u^n + dt k_3,
 *   u^{n+1} = u^n + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4).
 * dfdg_fe_step: one forward-Euler step u^{n+1} = u^n + dt M^{-1}L(u^n) in place (eq. (FE);
 *   Example 5 steps this way).
 * Each integrator warm-starts its stage solves from its own earlier steps: calling another
 * integrator on the context (or dfdg_reset_history) starts from an empty history.
 * dfdg_history_save/_restore cover TVD-RK3's history. */
int dfdg_rk4_step(dfdg_ctx* ctx, double* U_io_dev, double dt, dfdg_rk4_info* info);
int dfdg_fe_step(dfdg_ctx* ctx, double* U_io_dev, double dt, dfdg_solve_info* info);
/* dfdg_rk3_step_stages: dfdg_rk3_step that also leaves the states entering the second
 *   and third stages in U1_dev and U2_dev (caller-owned, length n_broken, distinct from
 *   U_io_dev and from each other), for dfdg_rk3_step_vjp_stages. */
int dfdg_rk3_step_stages(dfdg_ctx* ctx, double* U_io_dev, double dt, double* U1_dev, double* U2_dev,
                         dfdg_step_info* info);
/* Forget the warm-start history of the forward stage solves (e.g. after changing U
 * externally, or before recomputing an earlier segment of a trajectory). */
int dfdg_reset_history(dfdg_ctx* ctx);
/* Forget the warm-start history of the adjoint stage solves (start of a reverse sweep). */
int dfdg_reset_adjoint_history(dfdg_ctx* ctx);
/* dfdg_history_bytes: size of the blob of dfdg_history_save for this context,
 *   3 * DFDG_HISTORY_DEPTH * n_lambda doubles.
 * dfdg_history_save: copies the forward warm-start history into hist_dev (caller-owned
 *   device memory of dfdg_history_bytes): per stage, the multipliers of up to
 *   DFDG_HISTORY_DEPTH earlier steps, newest first ([3][DFDG_HISTORY_DEPTH][n_lambda];
 *   unused entries are left alone), and the number of valid entries per stage into
 *   counts_host[3].  Asynchronous on the context stream.
 * dfdg_history_restore: the inverse (counts in 0..DFDG_HISTORY_DEPTH), e.g. at a
 *   checkpoint before a trajectory segment is recomputed, which then repeats the
 *   original solves exactly.  With DFDG_EXTRAPOLATE_PROJECT the blob holds no forward
 *   history (the projection basis is not part of it) and a restore empties the basis:
 *   a recomputed segment then starts its solves from other start values and repeats the
 *   original to the solver tolerance, not bit for bit. */
int dfdg_history_bytes(const dfdg_ctx* ctx, size_t* bytes);
int dfdg_history_save(dfdg_ctx* ctx, double* hist_dev, int* counts_host);
int dfdg_history_restore(dfdg_ctx* ctx, const double* hist_dev, const int* counts_host);

/* ---- adjoint form ------------------------------------------------------------------
 * dfdg_dg_residual_vjp: Ubar_dev = J_L(U)^T Lbar_dev, the transpose of the
 *   derivative of dfdg_dg_residual at U (upwind side frozen, the a.e. derivative).
 * dfdg_rk3_step_vjp: given U^n (Un_dev) and the cotangent of U^{n+1}, writes the
 *   cotangent of U^n (Ubar_io_dev in place) for one dfdg_rk3_step of size dt.
 *   Recomputes the stage states (two forward stage solves, which update the forward
 *   warm-start history); the mass solve is self-adjoint.
 * dfdg_rk3_step_vjp_stages: the same with the stage states U1_dev, U2_dev given (as
 *   left by dfdg_rk3_step_stages from U^n), so only the three adjoint solves run.
 *   Ubar_io_dev must not alias a state.
 * The adjoint solves are warm-started from those of the same stage in the previously
 * processed step (see dfdg_reset_adjoint_history); FP64 contexts only, triangle and
 * tetrahedral meshes. */
int dfdg_dg_residual_vjp(dfdg_ctx* ctx, const double* U_dev, const double* Lbar_dev,
                         double* Ubar_dev);
int dfdg_rk3_step_vjp(dfdg_ctx* ctx, const double* Un_dev, double* Ubar_io_dev, double dt,
                      dfdg_step_info* info);
int dfdg_rk3_step_vjp_stages(dfdg_ctx* ctx, const double* Un_dev, const double* U1_dev,
                             const double* U2_dev, double* Ubar_io_dev, double dt, dfdg_step_info* info);
/* dfdg_energy_vjp: Ubar_dev = Ebar U_dev, the cotangent of the kinetic energy
 *   E = 1/2 int |u|^2 (the energy of Sec. 4, Example 2; dfdg_diagnostics' energy) for a scalar
 *   cotangent Ebar: the broken basis is orthonormal (M_T = I), so E = 1/2 U . U and
 *   dE/dU = U.  U_dev and Ubar_dev hold n_broken doubles and may be the same buffer;
 *   asynchronous on the context stream. */
int dfdg_energy_vjp(dfdg_ctx* ctx, const double* U_dev, double Ebar, double* Ubar_dev);

/* ---- diagnostics and evaluation (a10) -----------------------------------------------
 * dfdg_eval: values out_dev[d][npts][T] of U at reference points ref_pts_host[npts][d]
 *   (npts <= 1024) of every element. */
int dfdg_diagnostics(dfdg_ctx* ctx, const double* U_dev, dfdg_diag* out_host);
int dfdg_eval(dfdg_ctx* ctx, const double* U_dev, int npts, const double* ref_pts_host,
              double* out_dev);

/* ---- allocation-free variant -------------------------------------------------------
 * dfdg_diagnostics_noalloc: dfdg_diagnostics for callers that cannot allocate device memory
 *   at the time of the call (code under HIP graph capture, tight serving loops, harnesses
 *   that forbid allocation).  Same kernels and results (bit for bit) as dfdg_diagnostics,
 *   but its scratch (one partial sum per element block and the four results) lives in a
 *   static device array of the library, 512 KiB per GPU, held until the process ends,
 *   instead of in the context's workspace.  The call allocates nothing.  Limit: meshes of at
 *   most 2097152 elements (larger ones return DFDG_E_INVALID_ARG).  Call it with the device
 *   current on which the context was bound (else DFDG_E_INVALID_ARG).  Every context on one
 *   GPU shares that array: calls that overlap on one GPU (two host threads, or two streams
 *   running at once) race and must be serialised by the caller; each call writes every
 *   value it reads, so the contents left by an earlier call do not matter. */
int dfdg_diagnostics_noalloc(dfdg_ctx* ctx, const double* U_dev, dfdg_diag* out_host);

/* ---- measurement -------------------------------------------------------------------
 * dfdg_time_kernel: launches kernel `which` `reps` times on the context stream and
 * returns the mean duration in ms.  Single kernels (which = 0, 2, 3, and 5, 6 on triangle
 * meshes) carry their own start/stop events in the dispatch (kernel execution time, as a
 * profiler reports it); the others are bracketed by a pair of events recorded on the stream.
 *   which = 0: facet SpMV + (p, S p) partials (FP64);  1: PCG vector update (FP64);
 *   2: DG residual (FP64); 3: facet SpMV (FP32, MIXED contexts only);
 *   4: multigrid V-cycle (AMG contexts only);
 *   5: condensation right-hand side (element kernel, in the context's local space);
 *   6: element recovery with the stage epilogue, in place on a work vector.
 * The kernels run on the context's current work vectors with a separate set of PCG
 * scalars whose stopping test never fires; the work vectors (not the warm-start
 * history) are clobbered.  bytes_out (may be NULL) receives the algorithmic bytes one
 * launch moves. */
int dfdg_time_kernel(dfdg_ctx* ctx, int which, int reps, float* ms_per_launch,
                     double* bytes_out);

/* ---- host inspection (no device work; used by the CPU test-suite) ----------------------
 * dfdg_debug_basis: the reference orthonormal basis psihat_i (i < P(k)) and its reference
 *   gradients at npts points pts_host[npts][2]: vals_host[npts][P],
 *   grads_host[npts][2][P] (may be NULL).
 * dfdg_debug_facet_matrix: the facet matrix S assembled on the host at context creation,
 *   as BSR: cols_host[ns][E] (column facets) and vals_host[ns][n_f][n_f][E]
 *   (slot, row mode, column mode, facet row), ns = 5 blocks per row on triangles (the
 *   facet, the other two facets of its first element, those of its second), 7 on
 *   tetrahedra (three and three).  Repeated columns of a row are merged into their first
 *   slot, the others hold zeros. */
int dfdg_debug_basis(int k, int npts, const double* pts_host, double* vals_host, double* grads_host);
int dfdg_debug_facet_matrix(const dfdg_ctx* ctx, int32_t* cols_host, double* vals_host);
/* dfdg_debug_basis3: the orthonormal Dubiner basis of the reference tetrahedron (k = 1, 2) at
 *   points pts_host[npts][3]: vals_host[npts][P], grads_host[npts][3][P] (may be NULL).
 * dfdg_debug_rule3: the tetrahedral path's rules for degree k (1, 2): which = 0 the
 *   residual's volume rule (exact for degree 3k-1, points [n][3], weights summing to 1/6),
 *   1 the face rule of the facet integrals (the fully symmetric rule of degree 4 (k = 1,
 *   6 points) or 6 (k = 2, 12 points): face parameters [n][2], weights summing to 1),
 *   2 the projection rule; pts_host / w_host may be NULL (then only *npts is set). */
int dfdg_debug_basis3(int k, int npts, const double* pts_host, double* vals_host, double* grads_host);
int dfdg_debug_rule3(int k, int which, int* npts, double* pts_host, double* w_host);
/* dfdg_debug_residual_rule: the volume quadrature rule of the residual for degree k on the
 *   reference triangle {xi, eta >= 0, xi + eta <= 1} (exact for total degree 3k-1, weights
 *   summing to the area 1/2): *npts receives the number of points; pts_host[npts][2] and
 *   w_host[npts] (each may be NULL) receive the points and weights. */
int dfdg_debug_residual_rule(int k, int* npts, double* pts_host, double* w_host);
/* dfdg_debug_multigrid: the multigrid hierarchy built at context creation (DFDG_AMG):
 *   *n_levels (0 for other preconditioners) and, for the first min(n_levels, max_levels)
 *   levels, rows_host[l], nnz_host[l] and the spectral radius estimate of D^{-1} A_l in
 *   rho_host[l].  The last level is inverted densely. */
int dfdg_debug_multigrid(const dfdg_ctx* ctx, int max_levels, int* n_levels, int64_t* rows_host,
                         int64_t* nnz_host, double* rho_host);
/* dfdg_debug_multigrid_matrix: one matrix of that hierarchy in CSR (host copies, FP64):
 *   which = 0 the operator A_level (level 0 is S, rows in facet-major order F*n_f + m),
 *   which = 1 the prolongator from level + 1 to level (rows: level's unknowns),
 *   which = 2 the dense pseudo-inverse of the coarsest operator (level = last), all n^2
 *   entries, which = 3 and 4 the products A P and R A = P^T A kept for levels 1 .. last - 1.  *n_rows, *n_cols, *nnz are always written; ptr_host[n_rows + 1],
 *   cols_host[nnz] and vals_host[nnz] are filled when all three are non-null (call once
 *   with nulls to size them).  DFDG_E_INVALID_ARG for a level or kind that does not exist. */
/* dfdg_debug_vcycle: z = one multigrid V-cycle (the context's preconditioner, FP32 or FP64
 *   cycle as configured) applied to b; b and z are device vectors of n_lambda doubles in
 *   the facet layout.  DFDG_AMG contexts only; synchronises the context stream. */
int dfdg_debug_vcycle(dfdg_ctx* ctx, const double* b_dev, double* z_dev);
/* dfdg_debug_facet_rhs: the facet right-hand side g = sum_T C_T W_T F_T of the last facet
 *   solve (before deflation), n_lambda doubles into a device vector; synchronises. */
int dfdg_debug_facet_rhs(dfdg_ctx* ctx, double* g_dev);
int dfdg_debug_multigrid_matrix(const dfdg_ctx* ctx, int level, int which, int64_t* n_rows, int64_t* n_cols,
                                int64_t* nnz, int64_t* ptr_host, int32_t* cols_host, double* vals_host);

#ifdef __cplusplus
}
#endif
#endif /* DFDG_H */
