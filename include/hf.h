/*
 * hf.h -- C ABI of the MI355X (gfx950) Newton step for the fully-coupled
 * hydraulic-fracture model of Giovanardi, Serebrinsky and Radovitzky
 * (arXiv 1911.10275).
 *
 * The library computes one Newton-Raphson iteration of the monolithic system
 * of Sec. "Computational framework": the discrete elastostatics of eq.
 * (discreteElastoStatics) on a discontinuous-Galerkin / cohesive-zone P^k
 * discretisation (interface elements on every interior face), coupled to
 * the continuous P^k lubrication equation eq. (discreteLubrication) on the
 * interface skeleton, linearised as the 2x2 block system eq.
 * (fully-coupled-fully-discrete) and solved with right-preconditioned
 * restarted GMRES (element block-Jacobi or a two-level block
 * preconditioner with a vertex coarse space) in FP64, or with an FP32
 * inner GMRES under FP64 iterative refinement (GMRES-IR).  alpha (the
 * cohesive-law activation) and beta (the fluid flag) stay frozen inside a
 * load step, as in one time step of the paper's algorithm; between load
 * steps hf_detect_activation applies the fracture and fluid activation
 * checks of eq. (fractureActivation) and eq. (fluidActivation).
 *
 * Conventions
 *  - Every call returns hf_status (HF_OK = 0); no C++ exception crosses the
 *    ABI.  hf_last_error() gives the message of the last failure of a ctx.
 *    Any call may return HF_EINVAL (a null required pointer, an instance id
 *    out of range, a size or value out of range), HF_ESTATE (call order),
 *    HF_ENOMEM and HF_EDEVICE (the HIP runtime); a call's comment names the
 *    other codes it returns.
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied; output arrays are caller-allocated.  *_device variants take
 *    device pointers that must stay valid until the ctx stream has finished
 *    the call's work.
 *  - Call order: hf_upload_mesh -> [hf_upload_interfaces, hf_set_material,
 *    hf_set_injection] -> hf_finalize -> hf_set_state -> {hf_assemble |
 *    hf_solve | hf_newton_step | hf_newton_solve | hf_end_load_step}.
 *    Any other order returns HF_ESTATE.
 *  - Batching: a context holds one or more independent fracture instances
 *    (one hf_upload_mesh call each; ids 0, 1, ... in call order) with the
 *    same dim and order but their own mesh, interfaces, material, injection
 *    and state.  Every compute call (hf_assemble .. hf_end_load_step) works
 *    on all instances in the same kernel launches and reports per-instance
 *    results in caller arrays of hf_instance_count() entries; its return
 *    value is HF_OK when every instance succeeded, else the status of the
 *    lowest failing instance (hf_last_error names it).  A failure of one
 *    instance never changes the result of another.
 *  - Context vectors (hf_apply_jacobian) are the concatenation
 *    [u_0, u_1, .., u_{B-1}, p_0, p_1, .., p_{B-1}]; hf_get_sizes gives each
 *    instance's offsets.
 *
 * Canonical orderings (shared with any caller-side checker)
 *  - Element node order: the simplex vertices as given, then (P2) edge
 *    midpoints of edges (01),(12),(20) in 2D and (01),(12),(20),(03),(13),(23)
 *    in 3D.  Displacement vector u: index (e*nodes_per_elem + a)*dim + i.
 *  - Interior faces: sorted by their ascending vertex-id tuple.  The "-"
 *    element is the lower element id; n is its outward unit normal;
 *    [[u]] = u+ - u-; opening w = [[u]] . n (eq. displacementJump).
 *  - Face integration points: conical-product Gauss rule on the face simplex
 *    whose vertices are the face vertices in ascending id order; order+1
 *    points per direction, first collapsed coordinate outermost, ascending.
 *  - Pressure unknowns: only on skeleton nodes of faces with beta = 1;
 *    vertex nodes ascending by vertex id, then edge-midpoint nodes ascending
 *    by (lo, hi) vertex ids.
 */
#ifndef HF_H
#define HF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HF_OK = 0,
  HF_EINVAL = -1,     /* bad argument (null pointer, size, index, value) */
  HF_ENOMEM = -2,     /* device or host allocation failed */
  HF_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed */
  HF_ESTATE = -4,     /* call out of order */
  HF_ESINGULAR = -5,  /* singular (to working precision) or non-finite
                         preconditioner block */
  HF_ENOCONV = -6,    /* GMRES, refinement or Newton hit its iteration cap */
  HF_ENONFINITE = -7  /* NaN or Inf in an input state or a computed result */
} hf_status;

typedef struct hf_ctx hf_ctx;

enum { HF_FP64 = 0, HF_FP32_IR = 1 };

typedef struct {
  int precision;       /* HF_FP64: FP64 GMRES; HF_FP32_IR: FP32 inner GMRES +
                          FP32 block inverses, FP64 residual and update
                          (default 0 = HF_FP64) */
  int gmres_m;         /* restart length, 1..256 (default 60) */
  int gmres_maxit;     /* GMRES iterations per linear solve (default 20000;
                          in FP32-IR the FP32 refinement and an FP64 solve
                          after it have one such budget each) */
  int ir_maxit;        /* refinement steps per linear solve (default 1000) */
  int newton_maxit;    /* iterations of hf_newton_solve (default 25) */
  double rtol;         /* true relative residual of every solve (default 1e-10) */
  double rtol_inner;   /* FP32-IR: a refinement step's inner GMRES stops once its
                          residual estimate has fallen by this factor, or
                          where the outer rtol is met (default 1e-4) */
  double newton_tol;   /* ||dU|| <= tol ||U|| and ||dP|| <= tol ||P|| (default 1e-10) */
  double b_stab;       /* DG stabilisation parameter b (default 10) */
  double p_cutoff;     /* pressure cut-off value when cutoff_on != 0 (default 0) */
  int cutoff_on;       /* clamp p >= p_cutoff after each update (default 0) */
  int device;          /* HIP device ordinal (default 0) */
  int profile;         /* 1: time kernel classes with HIP events (default 0);
                          with use_graphs = 1 only the launches outside the
                          captured GMRES chunks are timed */
  int use_graphs;      /* 1: replay chunks of GMRES iterations from captured HIP
                          graphs (default 1) */
  int mfma_inverse;    /* 1: in FP32-IR mode, FP32 inverses of 30 x 30 element
                          blocks on the matrix cores (16 x 16 tile Schur
                          scheme, falls back to FP64 Gauss-Jordan on a tile
                          pivot failure); 0: FP64 Gauss-Jordan rounded to
                          FP32 (default 1) */
  int ir_inner_cycles; /* FP32-IR: GMRES(m) cycles per refinement step, >= 1
                          (default 1: the refinement steps are the restarts) */
  int ir_stall_steps;  /* FP32-IR: an instance with this many refinement
                          steps (consecutive or not) whose true residual
                          falls by less than 90% and by less than a tenth of
                          what the FP32 cycle estimated (FP32 accuracy, not
                          the Krylov space, limits it: kappa u_32 near 1) is
                          solved again in FP64: FP64 GMRES on J dx = b from
                          dx = 0, with a gmres_maxit budget of its own (its
                          iterations are added to the solve's count and
                          reported as fp64_iters).  So is an instance after
                          a step that raised the true residual, or at the
                          refinement's caps.  Three steps with less than 1%
                          reduction double the inner restart length (up to
                          256; at 256 the instance goes to FP64).  An
                          instance that went to FP64 is solved in FP64 at
                          once in the later solves of the same load step
                          (until hf_end_load_step or hf_set_state; a stall
                          in the predictor's solve of hf_initial_guess
                          carries into the first load step, whose operator
                          is conditioned alike).  0:
                          every instance in FP64 at once, < 0: never
                          (default 2) */
  int incremental_assembly; /* 1: after the first full assembly, re-assemble
                          only the row panels of elements that touch a
                          cohesive or fluid interface, evaluate the other
                          residual rows as the product with their (constant)
                          cached blocks, and keep the constant blocks'
                          inverses; a material or b_stab change triggers a
                          full assembly (default 1); 0: full assembly and
                          all inverses every time */
  int fold_preconditioner; /* 1: after each block-Jacobi build, form the
                          right-preconditioned operator J M^-1 explicitly
                          (every Jacobian block times its column element's
                          inverse, the C strips times their element's
                          inverse; S^-1 is applied to the pressure part at
                          product time), so a GMRES iteration makes one
                          product instead of a preconditioner apply and a
                          product; 0: apply M^-1, then J (default 1) */
  int two_level;       /* 1: two-level block preconditioner (needs
                          fold_preconditioner = 1): the displacement block
                          is approximated by a coarse correction on P1
                          vertex functions (continuous across intact
                          interfaces, split across cracked ones; the coarse
                          matrix P^T A P factorised by multifrontal
                          Gauss-Jordan on a nested-dissection tree) followed
                          by the element blocks, and the pressure unknowns
                          by the Schur block D - C Ah^-1 B of that
                          approximation, combined as the full block
                          factorisation of J; a build whose coarse factor
                          meets a zero pivot falls back to block-Jacobi
                          (hf_profile.n_tl_fail); 0: block-Jacobi
                          (default 0) */
  int coarse_leaf;     /* vertex classes per leaf of the nested-dissection
                          tree, 4..4096 (default 64); fixed at the first
                          two-level build of a context */
  int coarse_reuse;    /* two-level builds that keep the last coarse
                          factorisation (and Z_c = A_c^-1 P^T B) instead of
                          refactorising P^T A P, 0..1000 (default 16): the
                          coarse matrix then lags the current one in the
                          rows of cracked elements, the only blocks that
                          change between Newton iterations; A P, W and the
                          Schur block are recomputed at every build, so the
                          preconditioner stays the exact full block
                          factorisation built on that coarse matrix.  A full
                          assembly or a failed build forces a new
                          factorisation; 0 refactorises at every build */
  int coarse_fp32;     /* 1: the coarse factorisation is rounded to FP32
                          once and FP64 solves apply that rounded factor
                          (FP64 arithmetic, half the bytes per coarse
                          solve); Z_c is computed with the same factor, so
                          the preconditioner is an exact block
                          factorisation on the rounded coarse matrix and
                          every solve still reaches rtol; 0: FP64 factor
                          (default 0) */
  int scale_fluid_rows; /* 1: the fluid rows carry the scale s_p of
                          hf_set_state (default 1); 0: s_p = 1, the rows of
                          eq. (discreteLubrication) as written.  The Newton
                          iterates do not depend on it; the relative
                          residuals of the linear solves do */
  int cohesive_unloading; /* 1: cohesive points unload irreversibly: each
                          face point keeps the largest opening w_max reached
                          at the end of a load step (hf_end_load_step; set
                          and read with hf_set_history / hf_get_history),
                          and a state-1 point with 0 < w < w_max follows the
                          secant T = (T_env(w_max) / w_max) w back to the
                          origin (w < 0: contact, k_c w), the envelope of
                          eq. (tsl) from w_max on -- the irreversible law of
                          the cohesive model the paper cites, whose
                          unloading it does not print (a reading); 0: the
                          envelope only (default 0) */
  void *stream;        /* hipStream_t to run on; NULL: a stream the ctx creates */
} hf_options;

typedef struct {
  double E, nu;        /* Young's modulus, Poisson ratio (plane strain in 2D) */
  double sigma_c;      /* cohesive strength of eq. (tsl) */
  double G_c;          /* fracture energy, delta_c = 2 G_c / sigma_c */
  double mu;           /* fluid viscosity of eq. (lubrication) */
  double dt;           /* backward-Euler time step */
} hf_material;

typedef struct {
  int64_t n_elem, nodes_per_elem, n_u, n_p, n_face, n_blocks;  /* of the instance */
  int64_t u_offset, p_offset;  /* its u and p in the context vectors (after hf_finalize) */
  int64_t n_total;             /* length of the context vectors, all instances */
  int32_t dim, order, nq_face, block_size;
} hf_sizes;

typedef struct {
  int gmres_iters;     /* total (inner) GMRES iterations */
  int ir_steps;        /* refinement steps (FP32-IR), 0 for FP64 */
  int restarts;        /* GMRES cycles */
  int status;          /* hf_status of this instance's solve */
  int fp64_iters;      /* FP32-IR: iterations of the FP64 GMRES that finished
                          the solve after the refinement stalled (included in
                          gmres_iters), 0 otherwise */
  double true_relres;  /* ||b - J dx|| / ||b||, recomputed in FP64 */
  double seconds;      /* wall time of the (batched) solve */
  double relres_u;     /* per-block true residuals after the solve (FP64,
                          compensated): ||(b - J dx)_u|| / ||b_u|| over the
                          displacement rows and */
  double relres_p;     /* ||(b - J dx)_p|| / ||b_p|| over the pressure rows;
                          a block whose part of b is zero is measured
                          against ||b||; 0 for an instance not solved */
} hf_solve_stats;

typedef struct {
  hf_solve_stats lin;  /* of the last linear solve (summed in hf_newton_solve) */
  double du_rel, dp_rel;   /* ||dU||/||U||, ||dP||/||P|| of the last update */
  double res_norm;     /* ||R|| at the start of the last iteration */
  int iterations;      /* Newton iterations taken */
  int converged;       /* 1 when both relative increments <= newton_tol */
  int status;          /* hf_status of this instance */
  int reserved;
} hf_newton_stats;

/* Kernel schedules and solver choices (all zero = defaults).  Changing them
   never changes what is solved: the schedules only change the rounding
   order, the solver choices the Krylov iterates, and every solve still
   reaches the true relative residual rtol. */
typedef struct {
  int spmv_var;        /* lanes per element row of the Jacobian product:
                          0 = 64/32/16 for block size 30/12/6, 1 = half */
  int prec_var;        /* the same for the block-Jacobi apply */
  int ortho_var;       /* rows per thread of the Gram-Schmidt passes:
                          0 = 4, 1 = 8, 2 = 2 (1024-row chunks) */
  int reorth;          /* orthogonalisation of the Krylov basis.
                          CGS2 = classical Gram-Schmidt with a second pass
                          when ||w1|| < ||w|| / sqrt(2); MGS1 = modified
                          Gram-Schmidt in its single-reduction form (the
                          projections on all basis vectors from one pass
                          over the basis plus the basis' new Gram row, then
                          one update pass).
                          0 (default): CGS2; 1: classical Gram-Schmidt with
                          the second pass always; 2: one classical pass in
                          FP64 solves; 3: MGS1 in FP64 solves; 4: MGS1 in
                          both precisions.  With 2 and 3 the FP32 inner
                          solves of GMRES-IR use CGS2 (single-pass schemes
                          lose orthogonality faster in FP32).  hf_autotune
                          level 1 chooses between 0 and 3 (FP64) or 0 and 4
                          (FP32-IR: 4 only for single-instance contexts and
                          restart lengths up to 60). */
  int gmres_m;         /* restart length (0 = keep hf_options.gmres_m) */
  int dense_wide_min;  /* pressure blocks with at least this many nodes are
                          inverted by a grid-wide Gauss-Jordan blocked over
                          panels of 32 pivots, the smaller ones by one
                          workgroup each (0 = 192; both with partial
                          pivoting, their results differ by rounding) */
  int inv_var;         /* element-block inverses of the FP32-IR
                          preconditioner (block size 30): 0 = as
                          hf_options.mfma_inverse, 1 = FP32 Gauss-Jordan on
                          the matrix cores, 2 = FP64 Gauss-Jordan rounded to
                          FP32; hf_autotune (level >= 0, FP32-IR) times both
                          on every block and keeps the faster */
  int reserved;
} hf_tuning;

typedef struct {
  /* accumulated device time (ms) and launch counts of kernel classes, when
     hf_options.profile = 1; reset by hf_reset_profile */
  double ms_assemble, ms_blockinv, ms_spmv64, ms_spmv32, ms_precond, ms_ortho;
  int64_t n_assemble, n_blockinv, n_spmv64, n_spmv32, n_precond, n_ortho;
  /* preconditioner builds with the matrix-core FP32 inverses, and those that
     fell back to FP64 Gauss-Jordan (counted whatever hf_options.profile is) */
  int64_t n_inv_mfma, n_inv_fallback;
  /* FP64 residuals b - J x of the restarts and refinement steps (compensated
     accumulation) */
  double ms_resid;
  int64_t n_resid;
  /* FP64 solves that went on with M^-1 then J after the folded operator held
     the true residual above the target for two cycles (counted whatever
     hf_options.profile is) */
  int64_t n_unfold;
  /* restart-length doublings after three cycles (FP64 solves) or three
     refinement steps (FP32-IR) with less than 1% progress (restarted-GMRES
     stagnation) */
  int64_t n_mgrow;
  /* FP32-IR refinement steps that raised the true residual (each sends its
     instance to the FP64 solve at once) */
  int64_t n_ir_rise;
  /* two-level preconditioner builds, and those whose coarse factor failed
     (block-Jacobi used for that solve) */
  int64_t n_tl_builds, n_tl_fail;
  /* coarse factorisations among the builds (the others kept the last one,
     coarse_reuse) */
  int64_t n_tl_factor;
} hf_profile;

/* Fill *opt with the defaults listed above. */
void hf_default_options(hf_options *opt);

/* Create a context on opt->device (NULL opt: defaults).  *out owns all the
   device memory of the instance; release it with hf_destroy. */
hf_status hf_create(const hf_options *opt, hf_ctx **out);
void hf_destroy(hf_ctx *ctx);
const char *hf_last_error(const hf_ctx *ctx);
/* Change options after creation (precision, tolerances, caps, profile). */
hf_status hf_set_options(hf_ctx *ctx, const hf_options *opt);
/* Number of instances uploaded so far. */
hf_status hf_instance_count(hf_ctx *ctx, int32_t *n);

/* Bulk mesh (Sec. "Computational framework": partition of the domain into
   simplices carrying independent P^k displacement nodes).
   dim 2|3, order 1|2; xyz (n_vert*dim) coordinates; elem_vert
   (n_elem*(dim+1)) vertex ids of straight-sided simplices; dirichlet_vert
   (n_vert, 0/1, nullable): a node copy is clamped (u = 0, strong) when it
   lies on a boundary facet whose vertices are all flagged.  Builds the
   interior-face list.  Each call adds one instance: *inst_out = its id
   (nullable).  All instances share dim and order. */
hf_status hf_upload_mesh(hf_ctx *ctx, int dim, int order, int64_t n_vert, const double *xyz,
                         int64_t n_elem, const int32_t *elem_vert,
                         const uint8_t *dirichlet_vert, int32_t *inst_out);

/* Interior faces after hf_upload_mesh: *n_face; face_vert (n_face*dim
   ascending vertex ids, nullable); face_elem (n_face*2: minus, plus element,
   nullable); *nq_face = integration points per face (nullable). */
hf_status hf_get_faces(hf_ctx *ctx, int32_t inst, int64_t *n_face, int32_t *face_vert,
                       int32_t *face_elem, int32_t *nq_face);

/* Interface state (eq. weakElastoStatics, the alpha and beta fields):
   qp_state (n_face*nq, face-major): 0 intact (DG flux + stabilisation),
   1 cohesive law of eq. (tsl) active, 2 traction-free (pre-crack); alpha = 1
   where state >= 1.  beta (n_face): 1 = the face carries fluid.  Default:
   all 0. */
hf_status hf_upload_interfaces(hf_ctx *ctx, int32_t inst, const uint8_t *qp_state,
                               const uint8_t *beta);

/* Material of an instance; required before hf_finalize, may change later
   (e.g. between load steps). */
hf_status hf_set_material(hf_ctx *ctx, int32_t inst, const hf_material *mat);

/* Point injections Q0 (right-hand side of eq. discreteLubrication) at
   skeleton vertices; each vertex must belong to a face with beta = 1. */
hf_status hf_set_injection(hf_ctx *ctx, int32_t inst, int32_t n_src, const int64_t *vert,
                           const double *q0);

/* Build layout, block pattern, geometry and pressure numbering on the
   device for all instances.  No mesh, interface or injection uploads after
   this call.  Limit: 16384 pressure nodes per instance (dense pressure
   block, inverted by a blocked Gauss-Jordan above 192 nodes). */
hf_status hf_finalize(hf_ctx *ctx);
hf_status hf_get_sizes(hf_ctx *ctx, int32_t inst, hf_sizes *out);
/* Pressure-node keys (n_p*2): (vertex, -1) or (lo, hi) of an edge node. */
hf_status hf_get_pnodes(hf_ctx *ctx, int32_t inst, int64_t *keys);

/* State at the start of a load step: u (n_u), p (n_p), w_old (n_face*nq,
   the opening of the previous step, source of eq. discreteLubrication;
   nullable = keep).  Rejects non-finite values (HF_ENONFINITE).  Also fixes
   the fluid-row scale s_p = 12 mu (L / w_ref)^3 with L the largest bounding
   box extent and w_ref the largest opening of the start state on the fluid
   faces' points (of w_old and of u's own opening w(u)), at least 0.01
   delta_c, per instance.  Instances never given a state start from zero. */
hf_status hf_set_state(hf_ctx *ctx, int32_t inst, const double *u, const double *p,
                       const double *w_old);
/* u, p, w (current opening at face points), w_old: each nullable. */
hf_status hf_get_state(hf_ctx *ctx, int32_t inst, double *u, double *p, double *w,
                       double *w_old);
/* Device-pointer variants on the ctx stream (FP64 arrays, same layouts). */
hf_status hf_set_state_device(hf_ctx *ctx, int32_t inst, const double *u, const double *p,
                              const double *w_old);
hf_status hf_get_state_device(hf_ctx *ctx, int32_t inst, double *u, double *p);

/* Residual R and Jacobian J = [[A, B], [C, D]] at the current state
   (eq. discreteElastoStatics, eq. discreteLubrication and their exact
   derivative), all instances.  res_norm[b] = ||R_b|| (nullable array). */
hf_status hf_assemble(hf_ctx *ctx, double *res_norm);
/* The linear solve of one Newton iteration: the 2x2 block system of eq.
   (fully-coupled-fully-discrete), J dx = -R with J = [[A, B], [C, D]], which
   the paper solves at every nonlinear iteration with a preconditioned Krylov
   method (Sec. "Computational framework", implementation paragraph; here
   element block-Jacobi with the pressure unknowns as one Schur block).
   Builds the preconditioner and solves every instance to the true relative
   residual rtol (GMRES or GMRES-IR per options); dx is kept in the ctx;
   stats[b] per instance (nullable array).  HF_ESINGULAR: a preconditioner
   block of the instance is singular to working precision (a pivot at most
   1e-13 of the block's largest entry, or not finite); HF_ENOCONV: the
   iteration caps were reached; HF_ENONFINITE: a non-finite right-hand side
   or Krylov vector.  The failing instance's dx is undefined. */
hf_status hf_solve(hf_ctx *ctx, hf_solve_stats *stats);
/* One Newton-Raphson iteration of every instance (Sec. "Computational
   framework": the system is linearised at the current iterate, solved, and
   the increments of both nodal arrays U and P are added; convergence is
   judged on the Euclidean norms of the relative increments): assemble +
   solve + update u, p (+ optional cut-off of the remark on fluid lag).  An
   instance whose solve fails (HF_ENOCONV, HF_ESINGULAR, HF_ENONFINITE)
   keeps its state.  stats[b] per instance. */
hf_status hf_newton_step(hf_ctx *ctx, hf_newton_stats *stats);
/* The Newton loop of one time step (Sec. "Computational framework"):
   iterations until every instance has converged (||dU|| <= newton_tol
   ||U||, ||dP|| <= newton_tol ||P||) or failed; an instance stops iterating
   once converged.  An instance that has not converged within newton_maxit
   (HF_ENOCONV) or failed gets back its state at the start of the call.
   stats[b] per instance (nullable array). */
hf_status hf_newton_solve(hf_ctx *ctx, hf_newton_stats *stats);
/* One iteration of the staggered (sequential) comparison scheme of Sec.
   "Fully-coupled vs. staggered hydro-mechanics with applied inflow boundary
   conditions": each field is solved from its own equations with the other
   taken from the previous iteration, the decoupled forms A U = E - B P and
   D P = F - C U of eq. (fully-coupled-fully-discrete).  First the solid rows
   with the pressure held, A dU = -R_u(U, P) (same solver and options as
   hf_solve; one solve for the linear solid, a Newton sub-step where cohesive
   tractions make it nonlinear), then the fluid rows with the new opening
   held, D dP = -R_p(U, P) with D = dR_p/dP the Poiseuille flux operator
   alone: the decoupled fluid equation is elliptic and needs an essential
   condition, here the row of pressure node dir_node[b] (instance-local
   index, see hf_get_pnodes) replaced by P[dir_node[b]] = dir_value[b]
   (dir_value nullable = 0).  dir_node may be null only when no instance has
   pressure nodes.  The optional cut-off applies to the new pressure.
   stats[b]: lin = the solid solve, du_rel and dp_rel of the two halves,
   res_norm = hypot(||R|| at the start with the fluid rows held, ||R|| after
   the solid half), converged when both relative increments <= newton_tol.
   An instance whose solid solve fails (its status) or whose modified
   pressure block is singular (HF_ESINGULAR: a zero or non-finite pivot,
   e.g. a node whose faces are all closed and conduct nothing) gets back its
   state from the start of the call.  The assembled system is left modified:
   assemble again before hf_solve. */
hf_status hf_staggered_step(hf_ctx *ctx, const int32_t *dir_node, const double *dir_value,
                            hf_newton_stats *stats);
/* End of a given-length load step: the opening of the converged state
   becomes the previous opening w^n of the storage term (w - w^n)/dt of eq.
   (discreteLubrication), w_old <- w(u) at every face point, and the
   fluid-row scale s_p is recomputed from it; with cohesive_unloading the
   unloading history becomes max(w_max, w) at every face point. */
hf_status hf_end_load_step(hf_ctx *ctx);
/* Unloading history of instance inst (cohesive_unloading; the irreversible
   form of the cohesive law of eq. (tsl)): w_max per face point,
   n_face * nq_face values in the order of hf_get_faces (host array, read or
   written during the call, owned by the caller).  hf_finalize sets it to
   zero; hf_end_load_step raises it to the opening of the converged state
   when cohesive_unloading is 1.  A negative entry acts as 0 (no history).
   The history is kept whatever cohesive_unloading says, and only read when
   it is 1.  HF_ESTATE before hf_finalize, HF_EINVAL for an instance out of
   range or a null array (when the instance has faces), HF_ENONFINITE on a
   NaN or Inf (nothing is copied then). */
hf_status hf_set_history(hf_ctx *ctx, int32_t inst, const double *w_max);
hf_status hf_get_history(hf_ctx *ctx, int32_t inst, double *w_max);
/* Starting state of the first load step: the uniform-pressure elastic
   predictor.  With the pressure held fixed at 1 the displacement rows are
   solved for u1 (one linear solve, same solver options); V1 = crack volume
   of u1 over the fluid faces; then p0 = (sum Q0) dt / V1 and the state
   becomes u = p0 u1, p = p0 on every pressure node (w_old unchanged).  This
   gives the opening and pressure of a crack that stores the first step's
   injected volume under uniform pressure, so the cubic-law conductivity is
   not degenerate at the first Newton iterate (the paper starts the same
   test from uniform pressure and opening, Sec. "Verification of the
   fully-coupled algorithm").  p0_out[b] (nullable array) = p0 of instance b;
   instances without pressure nodes or injection keep their state (p0 = 0);
   an instance whose predictor fails keeps its state.  The fluid-row scale
   s_p is then recomputed from the predictor's opening (as hf_set_state
   does). */
hf_status hf_initial_guess(hf_ctx *ctx, double *p0_out);

/* ---- fracture and fluid activation (end of a load step) ---- */
/* Normal traction the DG method exchanges at every face point of instance
   inst at the current state (the flux of the consistency and stabilisation
   terms of eq. weakElastoStatics): tn[f*nq + q] = n.{sigma(u)} n +
   (b/h_f)(lambda + 2G) [[u]].n, the quantity the fracture activation of eq.
   (fractureActivation) compares with sigma_c.  tn: caller array of
   n_face*nq_face doubles (instance-local face order of hf_get_faces). */
hf_status hf_get_interface_traction(hf_ctx *ctx, int32_t inst, double *tn);
/* Activation checks on the current (converged) state of instance inst,
   eq. (fractureActivation) and eq. (fluidActivation): an intact point
   (state 0) whose DG normal traction exceeds sigma_c becomes cohesive
   (state 1, irreversible); a face without fluid whose points are all in
   state >= 1 becomes a fluid face (beta = 1) once its opening exceeds
   delta_c at any point (the fluid threshold taken as delta_c).  Writes the
   new states into the caller arrays qp_state (n_face*nq_face) and beta
   (n_face) in the layout of hf_upload_interfaces, and n_new[0] = points
   newly activated, n_new[1] = faces newly fluid (nullable).  The context is
   not changed: the fluid unknowns follow beta, so applying the new states
   means uploading them to a new context (hf_create ... hf_finalize) and
   carrying the state over (pressure nodes matched by hf_get_pnodes keys). */
hf_status hf_detect_activation(hf_ctx *ctx, int32_t inst, uint8_t *qp_state, uint8_t *beta,
                               int64_t *n_new);

/* ---- inspection hooks (tests, benchmarks) ---- */
/* R_u (n_u), R_p (n_p) of the last hf_assemble. */
hf_status hf_get_residual(hf_ctx *ctx, int32_t inst, double *R_u, double *R_p);
/* Block rows of A for n_rows elements: cols (n_rows*(dim+2), -1 = no block),
   blocks (n_rows*(dim+2)*bs*bs, row-major bs x bs; slot 0 = diagonal, slot
   1+f = neighbour across local face f). */
hf_status hf_get_block_rows(hf_ctx *ctx, int32_t inst, int64_t n_rows, const int32_t *elems,
                            int32_t *cols, double *blocks);
/* Dense coupling blocks (small meshes): B (n_u*n_p), C (n_p*n_u),
   D (n_p*n_p), row-major; each nullable. */
hf_status hf_get_coupling(hf_ctx *ctx, int32_t inst, double *B, double *C, double *D);
/* Increment dx = (du, dp) of an instance from the last solve. */
hf_status hf_get_increment(hf_ctx *ctx, int32_t inst, double *du, double *dp);
/* Element-block inverses of the block-Jacobi preconditioner after a solve:
   n_rows*bs*bs row-major blocks of the elements given (instance numbering);
   precision HF_FP64 = the FP64 inverses (in FP32-IR mode with the matrix-
   core inverses these exist only for elements with coupling strips),
   HF_FP32_IR = the FP32 inverses the inner solves use. */
hf_status hf_get_block_inverse(hf_ctx *ctx, int32_t inst, int64_t n_rows, const int32_t *elems,
                               int precision, double *out);
/* y = J x on device context vectors (length n_total, all instances);
   precision HF_FP64 uses the
   FP64 matrix (double*), HF_FP32_IR the FP32 copy (float*) built by the
   last hf_solve in FP32-IR mode. */
hf_status hf_apply_jacobian(hf_ctx *ctx, int precision, const void *x, void *y);
/* y = J M^-1 x, the right-preconditioned operator of GMRES, on device context
   vectors, with the factors of the last hf_solve in that precision:
   folded = 1 uses the block-Jacobi M folded into the blocks (built by that
   solve when hf_options.fold_preconditioner = 1; HF_ESTATE otherwise),
   folded = 0 applies the block-Jacobi M^-1 and then J, folded = 2 uses the
   two-level block preconditioner of that solve (hf_options.two_level = 1;
   HF_ESTATE when it was not built).  HF_ESTATE when the last solve ran in the
   other precision or the system was re-assembled since. */
hf_status hf_apply_preconditioned(hf_ctx *ctx, int precision, int folded, const void *x, void *y);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   folded form (folded = 1) of hf_apply_preconditioned, y = J M^-1 x on
   device context vectors, enqueued on the ctx stream with no allocation
   and no host synchronisation.  The S^-1 x_p staging vector lives in a
   fixed 512 KiB device array that the library holds on each GPU until the
   process ends; HF_EINVAL when the context has more than 65,536 pressure
   unknowns.  Every call on a GPU shares that array (its contents are fully
   rewritten before use): calls that overlap on one GPU, from contexts on
   different streams, race.  HF_ESTATE as for hf_apply_preconditioned. */
hf_status hf_apply_preconditioned_noalloc(hf_ctx *ctx, int precision, const void *x, void *y);
hf_status hf_get_profile(hf_ctx *ctx, hf_profile *out);

/* ---- tuning ---- */
hf_status hf_get_tuning(hf_ctx *ctx, hf_tuning *out);
/* Out-of-range fields give HF_EINVAL and change nothing. */
hf_status hf_set_tuning(hf_ctx *ctx, const hf_tuning *t);
/* Autotuner (after hf_assemble; uses the assembled system and leaves it
   in place).  level 0: times every variant of the Jacobian product, the
   block-Jacobi apply and the Gram-Schmidt passes (HIP events, 10 launches
   each after warm-up) in the context's precision and keeps the fastest;
   level 1: then also times complete linear solves for restart lengths
   {30, 60, 120} (30 for one instance only) x orthogonalisation {0, 3}
   (FP32-IR: {0, 4}, the latter for one instance at m <= 60 only) and keeps
   the fastest whose solves all
   converge (the candidates are timed on the context's current system;
   later solves do not re-check the choice, but a restart length that
   stagnates there is doubled by the solver itself and an FP32-IR instance
   that stalls is solved in FP64).  At both levels a candidate replaces an
   earlier one only when it is faster by more than 2%, so near-ties keep the
   first candidate.  cache_path (nullable): a text file of
   "key choices" lines; the key names the GPU architecture, dim, order,
   sizes, instance count, precision and level.  A line with the context's
   key is applied without timing; otherwise the result is appended.
   level -1: apply the cached level-1 choice, else the level-0 one, else
   keep the current choice; never times.  *out (nullable) receives the
   choice. */
hf_status hf_autotune(hf_ctx *ctx, int level, const char *cache_path, hf_tuning *out);
hf_status hf_reset_profile(hf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HF_H */
