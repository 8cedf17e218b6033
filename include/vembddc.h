/*
 * vembddc -- BDDC-preconditioned CG for the interface saddle-point problem of
 * divergence-free virtual element discretisations of 3D Stokes, on MI355X.
 *
 * The method (Bevilacqua, Dassi, Zampini, Scacchi, "BDDC preconditioners for
 * virtual element approximations of the three-dimensional Stokes
 * equations"):
 *   - subdomain saddle matrices glued by the interface restrictions R_Gamma^(i)
 *     (Sec. 4.2, eqs. discMat, ScapGdef);
 *   - static condensation of interior velocity and mean-zero pressure by
 *     Dirichlet solves (eq. uipi) onto the interface problem
 *     S_hat u_hat = g_hat (eq. globInt) with S_Gamma^(i) of eq. firstSchur;
 *   - the BDDC preconditioner M^-1 = Rt_D^T St^-1 Rt_D (eq. BDDCprec) with the
 *     primal recipe of Sec. 5.1 (vertices, averages, face fluxes; change of
 *     basis; dependent constraints dropped) and deluxe scaling (Sec. 6);
 *   - preconditioned CG to a relative residual (Sec. 7) and recovery of the
 *     interior unknowns (eq. uipi).
 *
 * Conventions (all entry points):
 *   - every call returns VB_OK (0) or a negative VB_ERR_* code and never
 *     throws; vb_last_error() gives a message;
 *   - host arrays passed in are copied; the caller keeps ownership;
 *   - "device" pointers are HIP device memory owned by the caller, accessed in
 *     stream order on the context's stream (vb_options.stream);
 *   - calls must be ordered create -> assemble (every subdomain) -> setup ->
 *     (apply | schur_apply | pcg_solve | get_local_solution)*; otherwise
 *     VB_ERR_STATE;
 *   - a context is not thread-safe.
 *
 * The global interface vector layout (all vectors of length vb_interface_size)
 * is [u_Gamma (n_iface entries, indexed by global interface id) | p0 (one
 * per subdomain, in subdomain order)].
 */
#ifndef VEMBDDC_H
#define VEMBDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VB_OK = 0,
  VB_ERR_ARG = -1,             /* invalid argument or inconsistent sizes */
  VB_ERR_STATE = -2,           /* call out of order */
  VB_ERR_OOM = -3,             /* device allocation failed */
  VB_ERR_DEVICE = -4,          /* a HIP runtime call failed */
  VB_ERR_NOT_SPD = -5,         /* a pivot of a local factorisation had the wrong sign */
  VB_ERR_SINGULAR_COARSE = -6, /* the coarse problem could not be factorised */
  VB_ERR_BREAKDOWN = -7,       /* p^T S p <= 0 or NaN inside PCG */
  VB_ERR_NOT_CONVERGED = -8    /* maxit reached; the last iterate is returned */
};

enum { VB_PREC_FP64 = 0, VB_PREC_MIXED = 1 };
enum { VB_SCALING_DELUXE = 0, VB_SCALING_COUNTING = 1 };
enum { VB_KIND_INTERIOR = 0, VB_KIND_INTERFACE = 1, VB_KIND_PRESSURE = 2 };
enum { VB_ENT_VERTEX = 0, VB_ENT_EDGE = 1, VB_ENT_FACE = 2 };

typedef struct vb_options {
  int precision;     /* VB_PREC_FP64, or VB_PREC_MIXED: local Dirichlet and
                        Neumann factors and Schur operators stored in FP32 (FP64
                        accumulation; coarse factorisation, deluxe scaling and
                        PCG recurrences stay FP64), FP64
                        residuals of the local systems drive an iterative
                        refinement of the whole saddle system (see vb_pcg_solve) */
  int scaling;       /* VB_SCALING_DELUXE (Sec. 6) or VB_SCALING_COUNTING (eq. pseudoinv) */
  double tol;        /* PCG relative residual ||g - S x|| <= tol ||g|| (default 1e-8) */
  int maxit;         /* PCG iteration cap (default 1000) */
  double svd_tol;    /* relative rank tolerance for dependent constraints (default 1e-10) */
  int panel;         /* dense factorisation panel width (32 or 64), 0 = default 64 */
  void *stream;      /* hipStream_t for all work; NULL = default stream */
  int profile;       /* nonzero: time every launch of the dominant kernels with HIP
                        events on `stream` (see vb_kernel_stats) */
  double adaptive_theta; /* > 0: adaptive face constraints (Sec. 6) with tolerance
                            theta (nu_tol): eigenvalues below 1/theta of every face
                            pencil add primal rows; 0 = the given constraints only */
  void *predictor;       /* NULL, or a trained vb_mlp: with adaptive_theta > 0 the
                            face eigenproblems first try a Chebyshev-filtered
                            subspace iteration whose block size and starting
                            vectors come from the network; faces where it does
                            not converge with a margin fall back to the dense
                            exact eigensolve */
  double setup_mem_limit; /* bytes of device memory the setup may hold at once for
                             the augmented local Neumann matrices (they are formed
                             and factored in waves of consecutive subdomains that
                             fit); 0 = 60% of the free device memory at that step.
                             A single subdomain larger than the limit still forms
                             a wave of its own. Results do not depend on it. */
  double local_mem_limit; /* bytes of device memory for the dense bordered local
                             Dirichlet matrices (FP64 only). When all of them
                             exceed it, they are formed, factored and condensed
                             in waves of consecutive subdomains sharing one
                             buffer of at most this size (a single larger
                             subdomain forms a wave of its own): the condensed
                             interface blocks are kept in a compact array and
                             vb_recover_all / vb_get_local_solution factor each
                             wave again. 0 = 45% of the free device memory at
                             the first vb_setup. Results do not depend on it. */
  int pcg_launch;         /* how the PCG iterations are launched: VB_PCG_AUTO (0),
                             VB_PCG_GRAPH (1: the launches of one iteration
                             captured as a HIP graph and replayed, the host
                             reading the convergence flags between replays) or
                             VB_PCG_PERSISTENT (2: one cooperative launch runs
                             every iteration of every problem, phases separated
                             by grid barriers, convergence decided on the
                             device; falls back to the graph where cooperative
                             launches are unavailable).  Same arithmetic in the
                             same order: the results are identical.  AUTO picks
                             the persistent launch when one S_hat application
                             reads less than 1 GB, else the graph. */
  int schur_kernel;       /* the symmetric per-iteration operators (S_hat p, and
                             S_DeltaDelta^-1 of the local Neumann solves): 0 =
                             each chosen by the autotuner, 1 = full-matrix GEMVs,
                             2 = the tiled symmetric kernel reading the lower
                             triangle only (half the bytes). */
  double fp32_pivot_min;  /* VB_PREC_MIXED: an FP32 pivot of a local Dirichlet
                             factorisation (its sign times the diagonal entry,
                             before the square root) at or below this value
                             counts as a breakdown of that subdomain's block, as
                             a wrong-signed or zero pivot does; such blocks are
                             factored again in FP64 (see vb_setup).  0 (default):
                             only wrong-signed or zero pivots.  In the units of
                             the local matrices; must be finite and >= 0. */
  int tune_factor;        /* the dense factorisations' panel width and outer
                             super-panel (the rank of each trailing update),
                             one of (64, 1024), (64, 512), (64, 2048),
                             (32, 512) columns, chosen per class
                             (local Dirichlet or its fronts, the second level
                             of the two-level scheme, local Neumann) by timing
                             the context's first factorisation of that class
                             with each candidate: 0 = when that factorisation
                             is large (more than 2e11 e n^2 summed over its
                             matrices), 1 = always, 2 = never (panel and
                             16-panel super-panels).  Results differ only by
                             rounding.  See vb_tuned_tile. */
  double inner_tol;       /* VB_PREC_MIXED: the relative residual reduction each
                             inner PCG solve of the refinement aims at (on the
                             FP32 operators; the last step aims only at what the
                             outer tolerance still needs); each step reduces
                             the FP64 residual by about that much.  0 =
                             default: 1e-3 for operators of 1e9 bytes or more
                             (looser steps, fewer iterations in all), 1e-4 below
                             (fewer steps: their fixed cost dominates).
                             Otherwise in (0, 1).  See vb_refinement_history. */
} vb_options;

enum { VB_PCG_AUTO = 0, VB_PCG_GRAPH = 1, VB_PCG_PERSISTENT = 2 };

/* One face of the adaptive coarse space (Sec. 6), as selected by vb_setup. */
typedef struct vb_face_info {
  int entity;        /* entity index (vb_assemble order) */
  int sub_i, sub_j;  /* the two subdomains sharing the face */
  int n_dual;        /* dual coordinates of the face in the minimal primal space */
  int n_selected;    /* eigenvalues below 1/theta (= new primal rows) */
  int predicted;     /* the network's count for the face, -1 without predictor */
  int path;          /* 0 dense exact eigensolve, 1 predicted subspace iteration
                        accepted, 2 predicted path rejected and exact fallback */
  int passes;        /* filter passes of the predicted path */
  double sum_shift;  /* 0, or the relative diagonal shift (1e-13, 1e-11, ... 1e-1
                        of max|diag|) that made the sum of the two face Schur
                        complements factorisable: needed when both neighbours
                        float and share rigid-mode traces on the face (FP64
                        factors: <= 1e-11 seen; the FP32 factors of the mixed
                        path: larger at a contrast inside a subdomain) */
} vb_face_info;

/* Device-time statistics of one kernel, accumulated over its launches. */
typedef struct vb_kernel_stat {
  int launches;
  double total_ms;   /* sum of the launch durations (HIP events) */
  double work;       /* algorithmic flops (which = 0) or bytes (which = 1) */
} vb_kernel_stat;

/* One subdomain's reduced local saddle problem (Sec. 4.2, eq. discMat):
 * rows/cols are the local DoFs, CSR with both triangles.  Velocity DoFs are
 * interior (VB_KIND_INTERIOR) or on the interface (VB_KIND_INTERFACE, with
 * their global interface id in gid); pressure DoFs (VB_KIND_PRESSURE) are
 * one constant per element with its volume |K| in pweight.  Dirichlet DoFs
 * must already be eliminated into rhs. */
typedef struct vb_subdomain {
  int32_t n;              /* number of local DoFs */
  int64_t nnz;
  const int64_t *indptr;  /* [n+1] */
  const int64_t *indices; /* [nnz] */
  const double *data;     /* [nnz] */
  const int32_t *kind;    /* [n] VB_KIND_* */
  const int64_t *gid;     /* [n] global interface id, -1 if not interface */
  const double *pweight;  /* [n] element volume for pressure DoFs, else ignored */
  const double *rhs;      /* [n] local right-hand side */
  const int32_t *part;    /* [n] or NULL: a one-level nested dissection of the local
                             Dirichlet problem (eq. uipi).  part[i] = b >= 0 puts
                             interior velocity or pressure DoF i in sub-box b,
                             whose eliminated DoFs must not couple to those of
                             another sub-box; part[i] = -1 puts an interior
                             velocity on the separator; every pressure needs a
                             sub-box; interface DoFs are ignored.  When every
                             subdomain of the context has labels, each sub-box is
                             condensed onto its separator and interface DoFs
                             first and the separators are eliminated second
                             (same results, far fewer operations than one dense
                             factorisation per subdomain); otherwise the labels
                             are not used. */
} vb_subdomain;

/* One interface entity (macro vertex, edge or face; Sec. 5.1): its global
 * interface ids (all DoFs shared by the same set of subdomains) and a dense
 * row-major block of candidate primal functionals over those DoFs. */
typedef struct vb_entity {
  int32_t kind;           /* VB_ENT_* */
  int32_t n;              /* number of DoFs */
  const int64_t *gids;    /* [n] */
  int32_t n_con;          /* number of constraint rows (may be 0) */
  const double *con;      /* [n_con * n] row-major */
} vb_entity;

typedef struct vb_solve_info {
  int iterations;
  double rel_residual;       /* recursive relative residual at exit */
  double true_rel_residual;  /* ||g - S x|| / ||g|| recomputed at exit */
  double lambda_min, lambda_max; /* Lanczos estimates of M^-1 S on the benign space */
  int n_coarse;              /* primal coarse dimension (+ one p0 per subdomain) */
  double setup_ms, solve_ms; /* device times of the last vb_setup / vb_pcg_solve */
  int status;                /* VB_OK or VB_ERR_* */
  int refinement_steps;      /* VB_PREC_MIXED: outer refinement steps taken (0 for FP64) */
  double latency_ms;         /* device clock from the start of the solve to this
                                problem's convergence (per problem, see
                                vb_problem_solve_info); the largest for the whole */
} vb_solve_info;

typedef struct vb_ctx vb_ctx;

/* Create a context; opt may be NULL for defaults (fields left 0 take their
 * defaults too).  VB_ERR_ARG for an unknown precision or scaling, a panel
 * width other than 32 or 64, a negative or NaN memory limit or adaptive
 * threshold, or a non-finite tolerance. */
int vb_create(vb_ctx **ctx, const vb_options *opt);
void vb_destroy(vb_ctx *ctx);
const char *vb_last_error(const vb_ctx *ctx);

/* Copy one problem: n_sub subdomains and n_ent entities covering every
 * interface id 0..n_iface-1 of the problem exactly once (Sec. 4.2:
 * R_Gamma^(i)).  Called again before vb_setup, it appends another,
 * independent problem: the context then solves all of them together (every
 * setup and iteration launch covers the subdomains of all problems; PCG keeps
 * separate scalars and convergence per problem).  Problem p's interface ids
 * are offset by the interface sizes of the problems before it, its
 * subdomains by their subdomain counts (see vb_problem_layout).  The host
 * arrays are copied.  Returns VB_ERR_ARG (reason in vb_last_error) for
 * inconsistent data: sizes, a CSR whose row pointers do not rise from 0 to
 * nnz or whose column indices leave 0..n-1, unknown DoF kinds, interface ids
 * outside 0..n_iface-1 or not covered by exactly one entity, a subdomain
 * holding part of an entity, fewer than two pressures, or a pressure weight
 * (element volume) that is not positive; a failed call leaves the context
 * as it was.  VB_ERR_STATE after vb_setup.
 * The split of each subdomain's pressures into a mean-zero part and a
 * global constant p0 (eq. discVQ) assumes no-slip boundaries: a subdomain's
 * summed pressure rows must vanish on its interior velocity DoFs, so that
 * p0 tests only interface fluxes.  Problems with natural (Neumann) boundary
 * sides break that for the subdomains touching them and are not supported;
 * the library does not detect them. */
int vb_assemble(vb_ctx *ctx, int64_t n_iface, int n_sub, const vb_subdomain *subs,
                int n_ent, const vb_entity *ents);

/* Everything the iteration needs (Sec. 4.2-4.3, 5.1, 6): local Dirichlet
 * factorisations and Schur complements S_Gamma^(i) with the condensed
 * right-hand side, change of basis, deluxe (or counting) scaling, local
 * constrained Neumann operators and the coarse problem.  Returns
 * VB_ERR_NOT_SPD (subdomain index in vb_last_error) on a pivot breakdown.
 * In VB_PREC_MIXED a subdomain whose FP32 Dirichlet factorisation breaks
 * down (eq. uipi: either level of the two-level scheme) is densified and
 * factored again in FP64, and its FP64 factors, inverse diagonal blocks and
 * Schur complement are rounded into its FP32 storage (the outer FP64
 * refinement corrects the rounding); vb_fp64_retries lists those
 * subdomains.  VB_ERR_NOT_SPD only when the FP64 factorisation breaks down
 * too.  A breakdown of an FP32 local Neumann factorisation is reported, not
 * retried. */
int vb_setup(vb_ctx *ctx);

/* Device time of the phases of the last vb_setup, in milliseconds (HIP
 * events on the context's stream, host work in between included): 0 local
 * Dirichlet factorisations and Schur complements, 1 primal constraints
 * (with the adaptive face eigenproblems), 2 change of basis, 3 condensed
 * right-hand side, 4 local Neumann problems, 5 coarse problem, 6 scaling,
 * 7 iteration structures (with the autotuner), 8 recovery structures.
 * Writes min(9, max) values to ms (host); returns 9 (VB_ERR_ARG for a
 * negative max or a NULL ms with max > 0); -1 for a phase not timed. */
int vb_setup_phases(const vb_ctx *ctx, int max, double *ms);

/* Subdomains (vb_assemble order, ascending) whose local Dirichlet
 * factorisation the last vb_setup redid in FP64 after an FP32 breakdown.
 * Returns their number (0 in VB_PREC_FP64 or before a setup) and writes the
 * first min(number, max) of them to subs (host memory; may be NULL when
 * max = 0); a negative max is VB_ERR_ARG. */
int vb_fp64_retries(const vb_ctx *ctx, int max, int32_t *subs);

/* The refinement steps of the last VB_PREC_MIXED vb_pcg_solve for one
 * problem (vb_assemble_batch order): rel[k] is the relative condensed FP64
 * residual before step k (rel[0] = 1; the value after the last step is
 * rel[steps]) and inner[k] the inner PCG iterations of step k.  Writes
 * min(steps + 1, max) values to rel and min(steps, max) to inner (host
 * memory; either may be NULL when max = 0) and returns steps (0 before a
 * mixed solve or in VB_PREC_FP64); VB_ERR_ARG for a problem out of range or
 * a negative max. */
int vb_refinement_history(const vb_ctx *ctx, int problem, int max, double *rel, int32_t *inner);

/* Length of the global interface vector: the interface ids of all problems
 * (problem order), then one p0 entry per subdomain (subdomain order). */
int64_t vb_interface_size(const vb_ctx *ctx);

/* Where problem `problem` sits in the global vectors and subdomain list. */
typedef struct vb_problem {
  int64_t iface_offset, n_iface;  /* its interface ids [offset, offset + n) */
  int64_t p0_offset;              /* its subdomains' p0 entries [p0_offset, + n_sub) */
  int sub_offset, n_sub;          /* its subdomains [sub_offset, + n_sub) */
} vb_problem;
int vb_num_problems(const vb_ctx *ctx);
/* Columns per workgroup that the autotuner chose (at the context's first
 * vb_setup, by timing 8/16/32/64 on the operators themselves) for the
 * per-iteration GEMVs: which = 0 S_hat p, 1 Neumann, 2 deluxe restriction,
 * 3 coarse; 0 before the first setup.  which = 4: 1 if S_hat p reads only
 * the lower triangle of each symmetric local operator (the tiled symmetric
 * kernel, timed against the best full-matrix tile), else 0.  which = 5: 1 if
 * the local Neumann solves read only the lower triangle of the symmetric
 * S_DeltaDelta^-1 block of [S_DeltaDelta^-1 | Phi] (the same kernel, plus a
 * GEMV of the Phi block), else 0.  which = 6, 7, 8: the panel width of the
 * local Dirichlet factorisation (single level, or the fronts of the
 * two-level scheme), of its second level, of the local Neumann
 * factorisation; which = 9, 10, 11: their outer super-panel columns (see
 * vb_options.tune_factor); 0 before that factorisation has run. */
int vb_tuned_tile(const vb_ctx *ctx, int which);
int vb_problem_layout(const vb_ctx *ctx, int problem, vb_problem *out);
/* Per-problem result of the last vb_pcg_solve (the info that call returns
 * combines them: largest iteration count, residual and latency, extreme
 * Lanczos values, worst status). */
int vb_problem_solve_info(const vb_ctx *ctx, int problem, vb_solve_info *out);

/* g_dev <- g_hat (eq. globInt) in the global interface layout (device). */
int vb_rhs(vb_ctx *ctx, double *g_dev);

/* y_dev <- S_hat x_dev (eq. globInt) (device vectors, global layout). */
int vb_schur_apply(vb_ctx *ctx, const double *x_dev, double *y_dev);

/* z_dev <- M^-1 r_dev (eq. BDDCprec) (device vectors, global layout). */
int vb_apply(vb_ctx *ctx, const double *r_dev, double *z_dev);

/* PCG on S_hat u = g_hat from x0 = x_dev (Sec. 7); x_dev receives the
 * solution (also on VB_ERR_NOT_CONVERGED).  info may be NULL.
 * VB_PREC_MIXED: iterative refinement.  Each step forms the FP64 residual of
 * every local system at the current (x, interior) iterate, condenses it with
 * the FP32 factor (eq. globInt applied to the residual), solves the interface
 * correction by PCG on the FP32 operators to a loose relative tolerance
 * (max(1e-4, tol/2 relative to the current residual)), recovers the interior
 * correction (eq. uipi) and updates.  It stops when the condensed FP64
 * residual has dropped to tol times the first one; rel_residual and
 * true_rel_residual both report that ratio, iterations the total inner PCG
 * iterations, refinement_steps the outer steps, lambda_* the first inner
 * solve.  The interior iterate is kept for vb_recover_all. */
int vb_pcg_solve(vb_ctx *ctx, double *x_dev, vb_solve_info *info);

/* Interior recovery (eq. uipi) for subdomain `sub` from the interface
 * solution x_dev: writes the subdomain's local DoF vector (n entries of its
 * vb_subdomain, in that CSR DoF order; interface entries copied from x_dev,
 * element pressures = Q_I part + p0) to u_host.  Runs vb_recover_all for
 * every subdomain and copies one out: to read several, call vb_recover_all
 * once instead. */
int vb_get_local_solution(vb_ctx *ctx, const double *x_dev, int sub, double *u_host);

/* Number of local DoFs of subdomain `sub` (the n of its vb_subdomain: the
 * length vb_get_local_solution writes), or with sub = -1 their sum over all
 * subdomains of all problems (the length vb_recover_all writes to out_dev).
 * VB_ERR_ARG before vb_assemble or for sub outside -1..n_sub-1. */
int64_t vb_local_size(const vb_ctx *ctx, int sub);

/* Interior recovery for every subdomain at once: out_dev (device, may be
 * NULL to only refresh the internal copy) receives the concatenation over
 * subdomains of their local DoF vectors, each in its own CSR DoF order.
 * VB_PREC_MIXED: FP64 refinement of the interior equations with the FP32
 * factor, the interface data fixed at x_dev: two passes from the interior
 * iterate of the last vb_pcg_solve when x_dev holds that solve's solution
 * bit for bit, else four passes from zero.  FP64 with local matrices in
 * waves (vb_options.local_mem_limit): every wave but the resident one is
 * factored again. */
int vb_recover_all(vb_ctx *ctx, const double *x_dev, double *out_dev);

/* Adaptive coarse space of the last vb_setup (Sec. 6): fills up to
 * max_faces entries of `faces` (may be NULL) and, in face order, the selected
 * eigenvalues (ascending per face, n_selected each) into up to max_eigs
 * entries of `eigs` (may be NULL; a face with every eigenvalue selected
 * contributes none).  Returns the number of faces (>= 0), or VB_ERR_STATE
 * before setup. */
int vb_adaptive_info(vb_ctx *ctx, int max_faces, vb_face_info *faces, int max_eigs, double *eigs);

/* ---- learned predictor of the adaptive constraints
 * A fully connected network 12 -> 32 -> 32 -> 1 (tanh, tanh, sigmoid), FP32,
 * on per-coordinate features of each face's reduced pencil (the matrix
 * L^-1 (At_i:At_j) L^-T, with L L^T = A_i:A_j): its output is the
 * coordinate's participation sum_t y_t[c]^2 in the eigenvectors below
 * 1/theta, so the sum over a face predicts the number of new constraints
 * and the largest scores give the starting block of the subspace iteration.
 * Labels come from the exact eigensolves of the method itself.
 * Parameter layout (VB_MLP_NPARAMS floats): [W1 (32 x 12, row-major), b1 (32),
 * W2 (32 x 32), b2 (32), w3 (32), b3]. */
#define VB_MLP_FEATURES 12
#define VB_MLP_NPARAMS 1505
typedef struct vb_mlp vb_mlp;
/* init: VB_MLP_NPARAMS host floats (copied).  stream: the hipStream_t every
 * call of the model runs on, in order after the caller's earlier work on it;
 * NULL = the default stream (training then drains the default stream and
 * runs its captured epochs on a stream of the model's own, since the default
 * stream cannot be captured).  Inside vb_setup the predictor runs on the
 * context's stream: the model must not be trained concurrently. */
int vb_mlp_create(vb_mlp **m, const float *init, void *stream);
void vb_mlp_destroy(vb_mlp *m);
const char *vb_mlp_last_error(const vb_mlp *m);
/* Append the (features, labels) of every face coordinate of ctx's last setup
 * (adaptive, faces solved by the exact eigensolve only).  Returns the number
 * of samples added (>= 0) or an error. */
int vb_mlp_add_samples(vb_mlp *m, vb_ctx *ctx);
int64_t vb_mlp_num_samples(const vb_mlp *m);
/* Standardise the features over the collected samples, then `epochs` steps
 * of full-batch Adam (one epoch captured once in a HIP graph and replayed);
 * loss_history (host, may be NULL) receives the loss before every step. */
int vb_mlp_train(vb_mlp *m, int epochs, float lr, double *loss_history);
/* Forward pass on n device samples (n x VB_MLP_FEATURES floats, row-major),
 * with the model's standardisation. */
int vb_mlp_forward(vb_mlp *m, const float *X_dev, int64_t n, float *s_dev);
/* Mean squared error and its gradient (device, VB_MLP_NPARAMS floats) on n
 * device samples, with the model's standardisation (identity before
 * training). */
int vb_mlp_loss_grad(vb_mlp *m, const float *X_dev, const float *y_dev, int64_t n,
                     float *grad_dev, double *loss);
int vb_mlp_get_params(const vb_mlp *m, float *params_host, float *mu_host, float *sd_host);
int vb_mlp_set_params(vb_mlp *m, const float *params_host, const float *mu_host,
                      const float *sd_host);
/* 1 (default): start the subspace iteration from the coordinates with the
 * largest scores; 0: from pseudo-random coordinates (for comparison). */
int vb_mlp_set_warm_start(vb_mlp *m, int on);
/* The last adaptive setup's per-coordinate face features (row-major,
 * VB_MLP_FEATURES each) and labels (NaN for faces not solved by the exact
 * eigensolve), copied to host buffers of max_n coordinates (either may be
 * NULL).  Returns the number of coordinates (>= 0) or an error. */
int64_t vb_face_samples(vb_ctx *ctx, int64_t max_n, float *X_host, float *y_host);
/* Append n host samples (X: n x VB_MLP_FEATURES row-major, y: n). */
int vb_mlp_add_data(vb_mlp *m, const float *X_host, const float *y_host, int64_t n);

/* Statistics of the kernels timed with vb_options.profile: which = 0 the
 * super-panel trailing update of the dense LDL^T of the local Dirichlet
 * factorisations (the setup's dominant kernel, in the precision of the local
 * matrices: FP64, or FP32 with VB_PREC_MIXED; work in flops: K*m*(m+1) per
 * matrix and super-panel of K columns with m trailing rows),
 * which = 1 the bordered local Schur GEMV of S_hat p (the iteration's
 * dominant kernel, work in bytes read/written).  reset != 0 clears them. */
int vb_kernel_stats(vb_ctx *ctx, int which, int reset, vb_kernel_stat *out);

/* Switch the per-launch timing of vb_options.profile on (nonzero) or off for
 * the calls that follow.  While it is on, the PCG iteration runs launch by
 * launch instead of as a replayed HIP graph, and every timed launch is
 * bracketed by two events. */
int vb_set_profile(vb_ctx *ctx, int on);

/* How the last PCG iterations of this context were launched: VB_PCG_GRAPH or
 * VB_PCG_PERSISTENT (see vb_options.pcg_launch; the mixed-precision solve
 * reports its last inner PCG), 0 before any solve. */
int vb_pcg_launch_used(const vb_ctx *ctx);

/* Virtual element matrices (Sec. 3).  For n_elem hexahedra with planar
 * faces, vertex coordinates X8 (device, n_elem x 8 x 3 doubles, local
 * vertex v = ix + 2 iy + 4 iz of the element's unit-cube corners) and
 * viscosities nu (device, n_elem; NULL = 1), the degree-k (2 <= k <= 4)
 * divergence-free element of Sec. 3 with degrees of freedom D1-D5 (vertex
 * values; values at the k-1 interior Gauss-Lobatto points of each edge;
 * face moments of v.n, v.t1, v.t2 against the face monomials of degree
 * <= k-2; the x-wedge volume moments of degree <= k-3; the divergence
 * moments against the non-constant monomials of degree <= k-1), numbered
 * vertex by vertex (3 components), edge by edge, face by face, then D4 and
 * D5 (see vb_vem_dofs for the sizes):
 *   A (device, n_elem x N x N, row-major): nu_K times the local form of
 *     eq. discreteA, consistency int Pi^0_{k-1} eps(u) : Pi^0_{k-1} eps(v)
 *     plus the dof-dof stabilisation sum_i sigma_i dof_i((I - Pi^nabla_k) u)
 *     dof_i((I - Pi^nabla_k) v), sigma_i = max(h_K, consistency_ii);
 *   B (device, n_elem x nP x N): int_K div(phi_j) m_a for the scaled
 *     monomials m_a of degree <= k-1 (row 0: the constant);
 *   F (device, n_elem x N; with_load != 0): eq. discreteF, int_K f .
 *     Pi^0_k phi_j for the manufactured load f = (3 pi^2 / 2) nu curl(psi),
 *     psi = sin(pi x) sin(pi y) sin(pi z) (1, 1, 1), by the rule exact to
 *     degree 2k+1 on the element's 12 cone tetrahedra.
 * Runs on the context's stream; returns when done.  VB_ERR_ARG for an
 * unsupported degree or a missing pointer. */
int vb_vem_element_matrices(vb_ctx *ctx, int k, int64_t n_elem, const double *X8, const double *nu,
                            int with_load, double *A, double *B, double *F);
/* Degrees of freedom N and pressure monomials nP of the degree-k element. */
int vb_vem_dofs(int k, int *n_dof, int *n_pressure);

/* Batched dense partial signed LDL^T (the kernel under the Dirichlet and
 * Neumann solves).  For each of `batch` column-major matrices A_b (size n_b,
 * leading dimension ld_b, lower triangle referenced) eliminate the first
 * e_b columns with pivot sign +1 for columns < p_b and -1 for columns in
 * [p_b, e_b).  On return the lower triangle holds L (eliminated columns) and
 * the Schur complement A22 - L21 D L21^T in the trailing block.  All
 * pointers (A[], n[], ld[], e[], p[], info[]) are device arrays of length
 * batch; info[b] = 0 or 1 + the column of a wrong-signed pivot. */
int vb_batched_ldl(vb_ctx *ctx, int batch, double *const *A, const int32_t *n,
                   const int32_t *ld, const int32_t *e, const int32_t *p,
                   int32_t *info, int max_n, int max_e);

/* Bytes of device working memory vb_batched_ldl_noalloc holds per GPU. */
#define VB_NOALLOC_SCRATCH_BYTES (32u << 20)

/* vb_batched_ldl for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same factorisation, arguments and results (the same kernels, so the
 * same bits), with its working memory -- the job table, the inverse
 * diagonal blocks of every panel and one flag -- in a fixed device array of
 * VB_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the process
 * ends (its address is looked up on the first call on each device).  It
 * calls no hipMalloc, hipFree or other allocating device routine.
 * Differences from vb_batched_ldl: the sizes are checked on the device, not
 * the host: a matrix with n < 0, n > max_n, e < 0, e > n, e > max_e or
 * ld < n is left untouched with info = -1 while the others are factored.
 * Returns VB_ERR_ARG when batch * ceil(max_e / 64) * 64 * 64 * 8 bytes of
 * inverse diagonal blocks, plus 256 bytes and 64 bytes per matrix, exceed
 * VB_NOALLOC_SCRATCH_BYTES.  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other threads, other contexts' streams)
 * race and must be serialised by the caller.  Stream-ordered on the
 * context's stream; returns after the factorisation has finished. */
int vb_batched_ldl_noalloc(vb_ctx *ctx, int batch, double *const *A, const int32_t *n,
                           const int32_t *ld, const int32_t *e, const int32_t *p,
                           int32_t *info, int max_n, int max_e);

#ifdef __cplusplus
}
#endif
#endif
