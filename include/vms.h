/* vms.h -- C ABI of the MI355X (gfx950) Newton-step library for the
 * variational-multiscale / generalized-alpha P1-tetrahedral discretisation of
 * hyper-elastodynamics with the nested block (Schur complement reduction)
 * preconditioned FGMRES solver (Liu & Marsden, arXiv:1809.06350).
 *
 * The calls follow the paper's statement of one Newton-Raphson iteration of
 * the predictor multi-corrector algorithm (section 3.3):
 *     assemble(mesh, state, material) -> K = [[A, B], [C, D]], R = (R_m, R_p)
 *     solve(K, R) -> Delta = (Delta v-dot, Delta p-dot)
 *     update(state, Delta)
 *
 * Conventions (all entry points)
 *  - Memory: every array pointer is a DEVICE pointer owned by the caller
 *    unless its comment says "host".  The library allocates no device memory
 *    after vms_ctx_create: solver scratch comes from a caller-provided
 *    workspace.  vms_ctx_create allocates a small device status area, the
 *    512 KB launch-timing flags, pinned host buffers and a fixed pool of HIP
 *    events (the solver's phase timing).  The code object also holds one
 *    static 64 MiB device array per GPU, the workspace of vms_step_noalloc.
 *  - Streams: all kernels are enqueued on the stream given to
 *    vms_ctx_create (in order).  Calls marked [async] return without waiting;
 *    calls marked [sync] wait for the stream work they need to take host-side
 *    decisions (convergence tests) and return after their last kernel is
 *    enqueued-and-finished.
 *  - Errors: integer status, no exceptions cross the ABI.  >0 is a warning
 *    (outputs hold the last iterate), <0 an error; vms_last_error() gives the
 *    message of the last non-OK status on that context.
 *  - Dof order per node is (v_x, v_y, v_z, p); nodal vectors [n][4] are
 *    node-interleaved, velocity vectors [n][3], pressure vectors [n].
 *  - Block values are stored entry-major over the shared node-graph pattern:
 *    A[9][nnzb] (row-major 3x3 entry e = 3*r + c), B[3][nnzb], C[3][nnzb],
 *    D[nnzb]; block b of row i couples node i to node col[b].  Rows have W
 *    fixed slots (slot_width, a multiple of 16): row i owns b = W*i + s,
 *    s < W, nnzb = W*n; its row_len[i] real blocks come first (sorted
 *    columns), the other slots are padding (column i, values zero).
 *  - Indices are int32 (nnzb = W n < 2^31, n_tets <= VMS_MAX_TETS so that the
 *    16 element-local pairs of every element are numbered in int32).
 *  - A context is not thread-safe; use one per stream.
 */
#ifndef VMS_H
#define VMS_H

#include <stddef.h>
#include <stdint.h>

#define VMS_MAX_TETS 134217727   /* 2^27 - 1: 16 * n_tets fits in int32 */
#define VMS_MAX_SHAT_ROW 128     /* longest off-diagonal row of the distance-2 pattern, in slots */
#define VMS_NOALLOC_SCRATCH_BYTES (64u << 20) /* static device scratch of vms_step_noalloc, per GPU */
#define VMS_AMG_MAX_LEVELS 8     /* levels of the aggregation multigrid hierarchy */

#ifdef __cplusplus
extern "C" {
#endif

enum vms_status {
  VMS_OK = 0,
  VMS_NOT_CONVERGED = 1,        /* Krylov or Newton iteration limit reached */
  VMS_ERR_ARG = -1,             /* bad argument (NULL, size, index out of range) */
  VMS_ERR_HIP = -2,             /* a HIP runtime call failed */
  VMS_ERR_WORKSPACE = -3,       /* workspace too small */
  VMS_ERR_INVERTED_ELEMENT = -4,/* J <= 0 in some element */
  VMS_ERR_BREAKDOWN = -5,       /* Arnoldi breakdown with a nonzero residual */
  VMS_ERR_NAN = -6,             /* NaN/Inf in a residual or Krylov norm */
  VMS_ERR_STATE = -7            /* the call needs a state the context does not hold (e.g. kernel
                                   timing read while it is off; no static scratch on this device) */
};

enum vms_material_kind { VMS_NH_COMP = 0, VMS_NH_INCOMP = 1, VMS_HGO_INCOMP = 2 };

/* assembly flags */
enum { VMS_ASM_RESIDUAL = 1, VMS_ASM_TANGENT = 2, VMS_ASM_RKCORR = 4 };

/* operator ids for vms_spmv */
enum { VMS_OP_FULL = 0, VMS_OP_A = 1, VMS_OP_B = 2, VMS_OP_C = 3, VMS_OP_D = 4 };

/* block preconditioner variants: the Schur complement reduction of Algorithm 1 (LDU) and its
 * partial factorizations (section 4.4 remark), and SIMPLE (section 4.3: exact A in the lower and
 * diagonal factors, diag(A)^-1 in the upper one, S^ for the Schur complement) */
enum { VMS_PC_LDU = 0, VMS_PC_UPPER = 1, VMS_PC_LOWER = 2, VMS_PC_DIAG = 3, VMS_PC_SIMPLE = 4 };

/* The Schur step of the block preconditioner: a Krylov solve to rtol_S (GMRES on S by the
 * matrix-free product of Algorithm 2; for SIMPLE, GMRES on the assembled S^), right-preconditioned
 * by the S^ preconditioner (shat_degree, shat_method); or one application of that S^
 * preconditioner alone, with no inner A-solve (section 4.4: the loosest choice of the Schur and
 * inner tolerances, where the method meets the coupled SIMPLE-type approach). */
enum { VMS_SCHUR_KRYLOV = 0, VMS_SCHUR_SHAT = 1 };

/* precision of the intermediate and inner levels */
enum { VMS_FP64 = 0, VMS_MIXED = 1 };

/* Arnoldi orthogonalisation: classical Gram-Schmidt with one
 * reorthogonalisation pass; modified Gram-Schmidt; classical Gram-Schmidt
 * without reorthogonalisation; classical Gram-Schmidt with a second pass only
 * when the first one removed more than half of ||w||^2 */
enum { VMS_ORTH_CGS2 = 0, VMS_ORTH_MGS = 1, VMS_ORTH_CGS1 = 2, VMS_ORTH_CGS_IFNEEDED = 3 };

/* Krylov method of the A-solves.  The paper's conclusions suggest symmetrising
 * the inner A system of the Schur product (Algorithm 2) and solving it by
 * conjugate gradients: VMS_AK_GMRES keeps GMRES on A at both A-levels;
 * VMS_AK_CG_INNER runs preconditioned CG (3x3 block-Jacobi) at the inner
 * level only; VMS_AK_CG at the inner and intermediate levels.  CG runs on
 * A_s = (A + A^T)/2 when cg_symmetrise is set (then the block-Jacobi
 * preconditioner of both A-levels is built from the symmetrised diagonal
 * blocks), otherwise on A as assembled (A is symmetric when the accelerations
 * vanish, and nearly so otherwise).  Only preconditioner applications change:
 * the outer FGMRES still solves the unsymmetrised system. */
enum { VMS_AK_GMRES = 0, VMS_AK_CG_INNER = 1, VMS_AK_CG = 2 };

/* Preconditioner of the A-level Krylov solves.  The paper preconditions them by
 * algebraic multigrid (section 5); VMS_APC_BJ is the 3x3 block-Jacobi
 * stand-in, VMS_APC_AMG one V-cycle of the library's aggregation multigrid
 * (vms_amg_create; mesh->amg), a fixed symmetric operator that CG and GMRES
 * both accept. */
enum { VMS_APC_BJ = 0, VMS_APC_AMG = 1 };

/* How the Schur solve's right preconditioner approximates S^-1 when
 * shat_degree = k > 0: the degree-k Chebyshev polynomial in diag(S^)^-1 S^
 * (a fixed linear operator), or k steps of diag(S^)-preconditioned CG on S^
 * (the Krylov-optimal degree-k polynomial for each vector; nonlinear, which
 * the flexible Schur-level GMRES allows). */
enum { VMS_SHAT_CHEBYSHEV = 0, VMS_SHAT_CG = 1, VMS_SHAT_NONE = 2 };   /* NONE: no S^ part (schur_mass > 0) */

typedef struct vms_ctx vms_ctx;
/* Aggregation multigrid hierarchy of a mesh (host object; vms_amg_create). */
typedef struct vms_amg vms_amg;

typedef struct {
  int32_t kind;     /* vms_material_kind */
  double rho0;      /* reference density */
  double mu;        /* shear modulus (neo-Hookean matrix) */
  double kappa;     /* bulk modulus (NH_COMP only) */
  double k1, k2, kd;/* HGO fibre stiffness, exponent, dispersion (HGO_INCOMP only) */
  double c_m;       /* tau_M coefficient, the paper fixes 1e-3 */
} vms_material;

typedef struct {
  double dt;        /* time step Delta t_n */
  double rho_inf;   /* spectral radius at infinity; alpha_m, alpha_f, gamma follow (section 3.2) */
  double t_n;       /* time at the start of the step */
  double t_load;    /* the dead load ramps linearly to full at t_load (<= 0: full load) */
} vms_timeint;

typedef struct {
  int32_t n_nodes, n_tets, n_bfaces;
  int32_t slot_width;       /* W: block slots per row (multiple of 16) */
  int64_t nnzb;             /* W * n_nodes */
  const double *X;          /* [n][3] reference coordinates */
  const int32_t *tets;      /* [m][4] positively oriented */
  const int32_t *bfaces;    /* [f][3] loaded boundary triangles (may be NULL if f = 0) */
  const double *traction;   /* [f][3] dead traction at full load */
  const uint8_t *dir_mask;  /* [n][4] 1 = Dirichlet on (v_x, v_y, v_z, p) */
  const double *dir_vel;    /* [n][3] prescribed velocity of Dirichlet components */
  const double *fibre;      /* [m][2][3] unit fibre directions (HGO) or NULL */
  const int32_t *col;       /* [nnzb] pattern from vms_setup_build */
  const int32_t *tpos;      /* [nnzb] position of the transposed block */
  const int32_t *diag_pos;  /* [n] */
  const int32_t *blk_src_ptr; /* [nnzb+1] contributions of each block ... */
  const int32_t *blk_src;   /* [16m] ... as e*16 + a*4 + b, increasing e within a block */
  int32_t shat_width;       /* W2: slots per row of the off-diagonal distance-2 pattern (multiple of 64) */
  const int32_t *shat_col;  /* [n * W2] off-diagonal pattern of S^ = D - C diag(A)^-1 B: sorted
                               columns first, padding slots hold the row's own node */
  const int16_t *shat_off;  /* [n * W2] or NULL: shat_col - row, when every offset fits in int16
                               (vms_setup_sizes' shat_span <= 32767); the S^ products then read
                               these 2-byte offsets instead of the 4-byte columns */
  const int32_t *nf_ptr;    /* [n+1] node -> loaded faces */
  const int32_t *nf_face;   /* [3f] */
  const vms_amg *amg;       /* HOST pointer: multigrid hierarchy uploaded by vms_amg_upload, needed
                               by a_prec = VMS_APC_AMG (NULL otherwise) */
} vms_mesh;

typedef struct {
  /* y_n, y-dot_n (read only) */
  const double *u_n, *p_n, *v_n, *du_n, *dp_n, *dv_n;
  /* the current iterate y_{n+1,(l)}, y-dot_{n+1,(l)} (updated in place) */
  double *u, *p, *v, *du, *dp, *dv;
} vms_state;

typedef struct {
  double *A, *B, *C, *D;          /* FP64 blocks, entry-major */
  float *A32, *B32, *C32, *D32;   /* FP32 mirrors of the scaled blocks (mixed form) or NULL */
  double *W;                      /* [n][4] symmetric diagonal scaling */
} vms_matrix;

typedef struct {
  double rtol, atol; int32_t maxit;        /* outer FGMRES (delta^r, delta^a, n^max) */
  double rtol_A, atol_A; int32_t maxit_A;  /* intermediate A-solves */
  double rtol_S, atol_S; int32_t maxit_S;  /* Schur-complement solve */
  double rtol_I, atol_I; int32_t maxit_I;  /* inner A-solve inside the Schur product */
  int32_t precond;    /* VMS_PC_* */
  int32_t precision;  /* VMS_FP64 or VMS_MIXED */
  int32_t orth;       /* VMS_ORTH_* of the A-, S- and inner levels; the outer FGMRES uses
                         VMS_ORTH_MGS if that is chosen, else VMS_ORTH_CGS2 */
  int32_t shat_degree;/* right preconditioner of the Schur solve: 0 = diag(S^)^-1; k > 0 = degree-k
                         Chebyshev polynomial in diag(S^)^-1 S^ on [lmax/shat_ratio, lmax], or k CG
                         steps on S^ (shat_method) */
  double shat_ratio;  /* lmax / lmin of the Chebyshev interval (used when shat_degree > 0) */
  int32_t a_krylov;   /* VMS_AK_*: GMRES or CG at the inner (or both) A-levels */
  int32_t cg_symmetrise; /* CG levels: 1 = on (A + A^T)/2, 0 = on A */
  int32_t shat_method;   /* VMS_SHAT_*: Chebyshev polynomial or CG steps on S^ (shat_degree > 0) */
  int32_t schur_solve;   /* VMS_SCHUR_*: Krylov solve of the Schur step, or one S^ preconditioner application */
  int32_t relax_inner;   /* 1: the inner A-solve of the Schur product at Schur iteration k stops at
                            rtol_I * ||r_0|| / ||r_k|| of the Schur level (at most 0.01), the
                            relaxation of inexact Krylov methods (Simoncini and Szyld 2003);
                            0: at rtol_I throughout, as in the paper */
  double schur_mass;     /* w >= 0: the Schur solve's right preconditioner gains the term
                            w (c M_p)^-1, M_p the lumped pressure mass matrix of the reference
                            configuration in the scaled variables and c = 1^T S 1 / 1^T M_p 1
                            (one Schur product per solve; with shat_method VMS_SHAT_NONE c = 1,
                            since GMRES iterates do not depend on the scale of a right
                            preconditioner).  A scaled mass matrix approximates S
                            when A is stiffness-dominated (section 1); with shat_method
                            VMS_SHAT_NONE it is the whole preconditioner.  Krylov Schur step of
                            P_SCR only (precond != SIMPLE, schur_solve = VMS_SCHUR_KRYLOV).
                            0: off, as in the paper */
  int32_t a_prec;        /* VMS_APC_*: preconditioner of both A-levels */
  int32_t pad_;
} vms_solver_opts;

typedef struct {
  int32_t status;
  int32_t n_outer;                  /* FGMRES iterations */
  int32_t n_A_solves, it_A;         /* intermediate A-solves and their total iterations */
  int32_t n_S_solves, it_S;         /* Schur solves and their total iterations */
  int32_t n_I_solves, it_I;         /* inner A-solves and their total iterations */
  double res0, res;                 /* outer ||r*|| at start and the final least-squares residual */
  double ms_total;                  /* host wall time of the call */
  /* Device time of the phases (HIP events recorded on the context stream, ms).  They nest:
   * ms_outer covers the whole Krylov solve after the preconditioner set-up, so it includes
   * ms_A and ms_S, and ms_S includes the ms_inner of the inner solves of its Schur products. */
  double ms_scale;                  /* Dirichlet rows, scaling, FP32 mirrors, rhs* (vms_solve only) and
                                       Delta = W x* */
  double ms_setup;                  /* preconditioner set-up: block-Jacobi inverses, S^, its
                                       Chebyshev bounds or pressure-mass fit */
  double ms_outer;                  /* outer FGMRES with its preconditioner applications */
  double ms_A;                      /* intermediate A-solves (Algorithm 1, steps 1 and 5) */
  double ms_S;                      /* Schur solves (Algorithm 1, step 3) */
  double ms_inner;                  /* inner A-solves of the Schur products (Algorithm 2) */
  int32_t phases_timed;             /* 1: every phase above was timed; 0: the context's event
                                       pool ran out and the figures are partial */
  int32_t pad_;
} vms_solve_stats;

typedef struct {
  double tol_R, tol_A;  /* relative / absolute Newton tolerances (section 3.3) */
  int32_t l_max;        /* maximum corrector iterations */
  int32_t rk_corr;      /* 1: keep the -K_{.,u-dot} R-bar_k / alpha_m term of the stage-1 rhs */
  double eps_diag;      /* scaling threshold epsilon_diag (section 4.1) */
  int32_t dir_lift;     /* Dirichlet velocity components in the predictor (section 3.3):
                           0 = preset: u = g(t_{n+1}), v = u-dot = g-dot, v-dot = 0 at once;
                           1 = lifted: they take the predictor like every node (v-dot = 0), and
                           the first corrector carries u to g(t_{n+1}) through R-bar_k, whose
                           rhs term K_{.,u-dot} R-bar_k / alpha_m spreads the boundary motion
                           into the interior (needs rk_corr; prescribed velocities constant in
                           time, as dir_vel states them).  The relative Newton test then divides
                           by the largest ||R_(l)|| so far instead of ||R_(0)||, which does
                           not yet hold the prescribed motion */
  int32_t pad_;
} vms_newton_opts;

typedef struct {
  int32_t status;
  int32_t n_newton;         /* corrector iterations taken */
  double res_norm[32];      /* ||R_(l)||, l = 1..min(l_max+1, 32) */
  vms_solve_stats last;     /* stats of the last linear solve */
  int32_t it_outer_total, it_A_total, it_S_total, it_I_total;
  double ms_assemble, ms_solve, ms_total;
  /* sums over the step's linear solves of the device phase times of vms_solve_stats */
  double ms_scale_total, ms_setup_total, ms_outer_total, ms_A_solve_total, ms_S_solve_total, ms_inner_total;
} vms_step_stats;

/* ---- context ------------------------------------------------------------ */

/* Bind a context to HIP device `device` and stream `stream` (NULL = the null
 * stream).  *out receives the context.  Returns VMS_ERR_HIP if the device is
 * not usable. */
int vms_ctx_create(vms_ctx **out, int device, void *stream);
void vms_ctx_destroy(vms_ctx *ctx);
/* Message of the last non-OK status on ctx (never NULL). */
const char *vms_last_error(const vms_ctx *ctx);

/* Launch timing of the A-block product, the solver's dominant kernel (a
 * measurement aid for the HBM roofline of its products).  vms_ctx_create
 * allocates its per-launch flags (512 KB of device memory) and a pool of
 * HIP events for the solver's phase timing.  With enable != 0
 * every launch of it -- inside vms_solve_scaled / vms_step (intermediate and
 * inner A-levels; on a CG level the CG product kernel, which fuses the
 * direction updates into the product) and from vms_spmv(VMS_OP_A) -- carries a start and a stop
 * HIP event that the dispatch itself records (hipExtLaunchKernelGGL: the
 * kernel's own begin and end on the context stream), and the kernel sets a
 * per-launch device flag when it does work (launches enqueued past a level's
 * convergence return at once and are not counted).
 * Enabling or disabling resets the counts.  [sync] */
int vms_ctx_set_timing(vms_ctx *ctx, int enable);
/* Sum of the event-timed durations (ms) and number of the counted launches
 * since the last call or reset, kind 0 = FP64 product, 1 = FP32 product;
 * resets that kind's counts.  At most 65536 launches per kind are recorded
 * between two calls.  VMS_ERR_STATE if timing is off.  [sync] */
int vms_ctx_kernel_time(vms_ctx *ctx, int kind, double *ms_total, int64_t *launches);

/* ---- setup (host, integer work) ---------------------------------------- */

/* Size of the node-graph block pattern of the P1 tangent (every pair of
 * nodes sharing a tetrahedron couples, section 3.1): *slot_width = W (the
 * longest row rounded up to a multiple of 16), *nnzb = W * n_nodes, and
 * *shat_width = W2, the longest off-diagonal row of the distance-2 pattern
 * (nodes two graph steps apart) rounded up to a multiple of 64; if shat_span
 * is not NULL, *shat_span = the largest |column - row| of that pattern (at
 * most 32767: the compact 2-byte offsets shat_off can be built).  tets: HOST
 * [m][4].  VMS_ERR_ARG on an out-of-range node, n_tets > VMS_MAX_TETS,
 * W * n_nodes or W2 * n_nodes >= 2^31, or W2 > VMS_MAX_SHAT_ROW. */
int vms_setup_sizes(int32_t n_nodes, int32_t n_tets, const int32_t *tets, int64_t *nnzb,
                    int32_t *slot_width, int32_t *shat_width, int32_t *shat_span);

/* Build, into HOST arrays sized by vms_setup_sizes: row_len[n], col[nnzb]
 * (slot layout above), tpos[nnzb] (position of the transposed block; a
 * padding slot maps to itself), diag_pos[n], the block contribution lists
 * blk_src_ptr[nnzb+1], blk_src[16m] (every element-local pair e*16 + a*4 + b
 * under the block (tets[e][a], tets[e][b]), in increasing e; padding slots
 * have none), the off-diagonal distance-2 pattern shat_col[n * W2] (sorted
 * columns first, padding slots hold the row's own node), optionally its
 * offsets shat_off[n * W2] = shat_col - row (NULL: not built; VMS_ERR_ARG if
 * one does not fit in int16), and node -> loaded-face lists nf_ptr[n+1],
 * nf_face[3f] (bfaces: HOST [f][3]). */
int vms_setup_build(int32_t n_nodes, int32_t n_tets, const int32_t *tets,
                    int32_t n_bfaces, const int32_t *bfaces,
                    int32_t *row_len, int32_t *col, int32_t *tpos, int32_t *diag_pos,
                    int32_t *blk_src_ptr, int32_t *blk_src, int32_t *shat_col, int16_t *shat_off,
                    int32_t *nf_ptr, int32_t *nf_face);

/* ---- assembly (section 3.3 steps 1-4; consistent-linearization appendix) - */

/* f_ext[n][3] = -int_Gamma N_A H dGamma_X for the dead traction at full load
 * (the traction term of R_m in the appendix), 1/3 of each reference face area
 * per vertex.  [async] */
int vms_nodal_load(vms_ctx *ctx, const vms_mesh *mesh, double *f_ext);

/* Set the iterate to the predictor y_(0) = y_n, y-dot_(0) = (gamma-1)/gamma
 * y-dot_n (section 3.3, predictor stage); Dirichlet velocity components take
 * u = dir_vel * t_{n+1}, v = u-dot = dir_vel, v-dot = 0 (dir_lift = 0), or
 * the predictor with v-dot = 0 (dir_lift = 1, vms_newton_opts.dir_lift).
 * [async] */
int vms_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti, vms_state *st, int dir_lift);

/* Workspace bytes of vms_assemble for these flags.  With the tangent on a
 * mesh of 16 slots per block row, the rows are assembled by their owners
 * straight into K, R and corr and the workspace is 1 KB; otherwise it holds
 * the element matrices and vectors (2 KB per element for the tangent, 128 B
 * each for the residual and the R-bar_k term). */
size_t vms_assemble_workspace(const vms_mesh *mesh, unsigned flags);

/* Element-by-element assembly at the generalized-alpha stages
 * y-dot_{n+alpha_m}, y_{n+alpha_f} computed from (y_n, y-dot_n) and the
 * iterate (section 3.3 step 1).  Each block (and each nodal entry) sums its
 * element contributions in increasing element order, so the result is
 * bitwise reproducible: the tangent on 16-slot rows by the row's owner, which
 * evaluates every incident element's terms itself; otherwise every element
 * writes its matrices to the workspace and the blocks gather them.
 *   VMS_ASM_RESIDUAL: R[n][4] = (R_m, R_p) of the appendix (P1, 4-point
 *     rule, tau_M frozen per element) plus load_scale * f_ext;
 *   VMS_ASM_TANGENT: K->A, B, C, D of the block reduction (eqs. defining A,
 *     B, C, D), exact linearisation of R;
 *   VMS_ASM_RKCORR: corr[n][4] = (alpha_f gamma dt / alpha_m) dR/du . R-bar_k,
 *     the K_{.,u-dot} R-bar_k / alpha_m term of the stage-1 right-hand side.
 * Outputs are overwritten.  f_ext may be NULL (no load).  workspace: at
 * least vms_assemble_workspace(mesh, flags) bytes (VMS_ERR_WORKSPACE
 * otherwise).  [sync]: returns VMS_ERR_INVERTED_ELEMENT if some element has
 * J <= 0 (the outputs are then undefined). */
int vms_assemble(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat,
                 const vms_timeint *ti, const vms_state *st, const double *f_ext,
                 vms_matrix *K, double *R, double *corr, unsigned flags,
                 void *workspace, size_t workspace_bytes);

/* *norm_host = || {R-bar_k, R_p, R_m} ||_2 over non-Dirichlet dofs (section
 * 3.3 step 3), R-bar_k = u-dot_{n+alpha_m} - v_{n+alpha_f}.  [sync]
 * VMS_ERR_NAN if the norm is not finite. */
int vms_residual_norm(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti,
                      const vms_state *st, const double *R, double *norm_host);

/* ---- linear system (section 4) ------------------------------------------ */

/* Dirichlet rows/columns (zeroed, unit diagonal, zero rhs) and symmetric
 * diagonal scaling (section 4.1): W_ii = |K_ii|^(-1/2) if |K_ii| >= eps_diag
 * else 1; K <- W K W in place, rhs_scaled[n][4] = W * (-R + corr) (corr may
 * be NULL), K->W written.  With mirror32 != 0 also writes K->A32..D32.
 * [async] */
int vms_prepare_system(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R,
                       const double *corr, double *rhs_scaled, double eps_diag, int mirror32);

/* y = op * x for one block of K (VMS_OP_A: y[n][3] = A x[n][3]; B: y[n][3] =
 * B x[n]; C: y[n] = C x[n][3]; D: y[n] = D x[n]; FULL: y[n][4] = K x[n][4]).
 * fp32 != 0 uses the FP32 mirrors with float x, y.  [async] */
int vms_spmv(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int op,
             const void *x, void *y, int fp32);

/* S^ = D - C diag(A)^-1 B from the blocks of K -- the approximate Schur
 * complement that preconditions the Schur solve, with diag(A) the point
 * diagonal (section 4.2): off-diagonal part S[n * W2] on shat_col (zero in
 * padding slots), diagonal Sdiag[n], and sdinv[n] = diag(S^)^-1 (1 where
 * S^_ii is 0 or not finite).  The solver forms the same matrix internally.
 * [async] */
int vms_schur_hat(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, double *S, double *Sdiag,
                  double *sdinv);

/* y = S^ x for the S^ of vms_schur_hat (off-diagonal S[n * shat_width] on
 * mesh->shat_col, diagonal Sd[n]; section 4.2), by the product kernel of the
 * Schur preconditioner's CG steps (its first step).  S, Sd, x, y are FP64, or
 * all FP32 when fp32 != 0; x[n] and y[n] must not alias.  Uses the
 * context's small device scratch, so calls on one context must not overlap.
 * [async] */
int vms_shat_spmv(vms_ctx *ctx, const vms_mesh *mesh, const void *S, const void *Sd, const void *x, void *y,
                  int fp32);

/* Workspace bytes needed by vms_solve, vms_solve_scaled, vms_solve_transpose
 * and vms_solve_transpose_scaled for these options (Krylov bases of the four
 * levels, control blocks, temporaries, the scaled right-hand side and
 * solution). */
size_t vms_solve_workspace(const vms_mesh *mesh, const vms_solver_opts *opts);

/* solve(K, R) -> Delta: stage 1 of the Newton iteration (section 3.3 step 5,
 * with the right-hand side of eq. NR_smaller_eqn_1): solve
 *     K Delta = rhs,  rhs = -R + corr  (corr may be NULL: rhs = -R),
 * K = [[A, B], [C, D]] as vms_assemble wrote it, by the symmetric diagonal
 * scaling of section 4.1 and the nested solve of vms_solve_scaled:
 * Dirichlet rows and columns replaced by the identity (Delta = 0 there),
 * W_ii = |K_ii|^(-1/2) (>= eps_diag, else 1), (W K W) x* = W rhs,
 * Delta = W x*.  K is OVERWRITTEN with W K W (the FP32 mirrors too when
 * opts->precision is VMS_MIXED) and K->W with W, as by vms_prepare_system.
 * R, corr, delta: [n][4] (v_x, v_y, v_z, p); delta = (Delta v-dot,
 * Delta p-dot).  Workspace as vms_solve_workspace.  [sync]  Status codes as
 * vms_solve_scaled; with VMS_NOT_CONVERGED delta holds W times the last
 * iterate. */
int vms_solve(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R, const double *corr,
              double *delta, double eps_diag, const vms_solver_opts *opts, void *workspace,
              size_t workspace_bytes, vms_solve_stats *stats);

/* Solve the scaled system K* x* = rhs* by FGMRES (outer level) right-
 * preconditioned by the nested Schur-complement-reduction preconditioner
 * (Algorithm 1 with Algorithm 2 for the Schur products): GMRES on A with
 * 3x3 block-Jacobi, GMRES on S = D - C A^-1 B preconditioned from
 * S^ = D - C diag(A)^-1 B (assembled as by vms_schur_hat): diag(S^)^-1, a
 * Chebyshev polynomial in diag(S^)^-1 S^, or CG steps on S^ (shat_degree,
 * shat_method); CG or GMRES on the A-levels (a_krylov).  x0 = 0; every level stops at
 * ||r|| <= max(rtol ||b||, atol) or maxit.  [sync]
 * Returns VMS_NOT_CONVERGED (x_scaled holds the last iterate) when the outer
 * level hits maxit. */
int vms_solve_scaled(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K,
                     const double *rhs_scaled, double *x_scaled, const vms_solver_opts *opts,
                     void *workspace, size_t workspace_bytes, vms_solve_stats *stats);

/* Stage 2 and update (section 3.3 steps 6-7): Delta = W x* (W = NULL:
 * x_scaled already holds Delta, as vms_solve returns it); Delta u-dot =
 * (alpha_f gamma dt/alpha_m) Delta v-dot - R-bar_k/alpha_m; y-dot += Delta
 * y-dot, y += gamma dt Delta y-dot on the iterate.  Dirichlet components keep
 * v and v-dot; u and u-dot stay fixed there too (dir_lift = 0) or move by
 * Delta u-dot = -R-bar_k/alpha_m (dir_lift = 1).  [async] */
int vms_newton_update(vms_ctx *ctx, const vms_mesh *mesh, const vms_timeint *ti,
                      vms_state *st, const double *W, const double *x_scaled, int dir_lift);

/* Workspace bytes of vms_step: the larger of vms_solve_workspace and the
 * assembly's element buffers (they are used in turn), plus its vectors. */
size_t vms_step_workspace(const vms_mesh *mesh, const vms_solver_opts *opts);

/* One generalized-alpha time step by the predictor multi-corrector algorithm
 * (section 3.3): predictor, then for l = 1..l_max: stage, residual, norm test
 * (||R_(l)|| / ||R_(0)|| <= tol_R or ||R_(l)|| <= tol_A), tangent, scaled
 * nested solve, stage 2 and update.  On return the iterate arrays of `st` hold
 * y_{n+1}, y-dot_{n+1}.  f_ext from vms_nodal_load (or NULL).  K is used as
 * storage for the tangent.  [sync]  VMS_NOT_CONVERGED if l_max is reached. */
int vms_step(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat,
             const vms_timeint *ti, vms_state *st, const double *f_ext, vms_matrix *K,
             const vms_newton_opts *nopts, const vms_solver_opts *sopts,
             void *workspace, size_t workspace_bytes, vms_step_stats *stats);

/* ---- adjoint (implicit differentiation of a converged time step) --------- */

/* Transposed solve, the adjoint counterpart of vms_solve: K^T lam = g with K
 * as vms_assemble wrote it.  Dirichlet rows and columns of K are replaced by
 * the identity (lam = 0 on Dirichlet dofs, g ignored there), W is formed from
 * K's diagonal as in vms_solve, and (W K^T W) lam* = W g is solved by the
 * nested preconditioner built for K^T = [[A^T, C^T], [B^T, D^T]] (Algorithm 1
 * applied to the transposed system; its Schur complement is
 * S^T = D^T - B^T A^-T C^T); lam = W lam*.  K is OVERWRITTEN with W K W and
 * K->W with W; Kt is caller storage with K's layout (FP32 parts needed only
 * for VMS_MIXED), overwritten with the transposed blocks.  g, lam: [n][4].
 * [sync]  Status codes as vms_solve. */
int vms_solve_transpose(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, vms_matrix *Kt, const double *g,
                        double *lam, double eps_diag, const vms_solver_opts *opts, void *workspace,
                        size_t workspace_bytes, vms_solve_stats *stats);

/* Transposed solve of an already scaled system: (W K^T W) lam* = rhs_scaled,
 * with K holding W K W from vms_prepare_system (K->W its scaling), through the
 * nested preconditioner built for the transposed blocks; Kt as in
 * vms_solve_transpose.  [sync]  Same status codes as vms_solve_scaled. */
int vms_solve_transpose_scaled(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, vms_matrix *Kt,
                               const double *rhs_scaled, double *lam_scaled, const vms_solver_opts *opts,
                               void *workspace, size_t workspace_bytes, vms_solve_stats *stats);

/* out[k] (HOST, 5 doubles) = lam^T dR/dtheta_k at the generalized-alpha stages
 * of `st`, theta = (mu, kappa, k1, k2, fibre angle) for the bits set in pmask
 * (1 << k); lam[n][4] = (lam_m, lam_p).  The derivatives differentiate the
 * residual of the consistent-linearization appendix in closed form (tau_M
 * depends on mu and kappa through the wave speed).  dfibre[m][2][3] = d a_i /
 * d angle (needed for bit 4).  Workspace >= vms_adjoint_workspace.  [sync] */
int vms_param_sensitivity(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat,
                          const vms_timeint *ti, const vms_state *st, const double *dfibre,
                          const double *lam, int pmask, double *out, void *workspace,
                          size_t workspace_bytes);

/* Workspace bytes of vms_adjoint_step / vms_param_sensitivity. */
size_t vms_adjoint_workspace(const vms_mesh *mesh, const vms_solver_opts *opts);

/* One backward step of the adjoint through the time history.  st holds y_n,
 * y-dot_n and, as the iterate, the converged y_{n+1}, y-dot_{n+1}.  In:
 * ybar1, ydbar1[n][7] = dJ/d(y_{n+1}), dJ/d(y-dot_{n+1}) as (u 3, p, v 3) and
 * (u-dot 3, p-dot, v-dot 3).  Out: ybar0, ydbar0 = dJ/d(y_n), dJ/d(y-dot_n).
 * Re-assembles the tangent at the converged state into K, solves the
 * transposed reduced system (Kt is its storage), recovers the kinematic
 * multiplier from the block factorisation, back-propagates through the
 * generalized-alpha stage relations and subtracts lam^T dG/dtheta from
 * dJdtheta (HOST, 5 doubles, bits of pmask).  [sync] */
int vms_adjoint_step(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                     const vms_state *st, const double *dfibre, vms_matrix *K, vms_matrix *Kt,
                     const double *ybar1, const double *ydbar1, double *ybar0, double *ydbar0, int pmask,
                     double *dJdtheta, const vms_solver_opts *opts, double eps_diag, void *workspace,
                     size_t workspace_bytes, vms_solve_stats *stats);

/* ---- aggregation multigrid for the A-levels (section 5: the paper uses AMG) */

typedef struct {
  int32_t max_levels;     /* 2 .. VMS_AMG_MAX_LEVELS */
  int32_t min_coarse;     /* a level with at most this many nodes is the coarsest */
  int32_t degree;         /* Chebyshev degree of pre- and post-smoothing on the finest level, and on
                             the levels below it but the coarsest when mid_degree is 0 (1 .. 16) */
  int32_t coarse_degree;  /* Chebyshev degree of the coarsest level's smoothing from zero (1 .. 64) */
  int32_t mid_degree;     /* Chebyshev degree of pre- and post-smoothing on the levels between the
                             finest and the coarsest (1 .. 16); 0 takes degree */
} vms_amg_opts;

typedef struct {
  int32_t n_levels;
  int32_t n[VMS_AMG_MAX_LEVELS];     /* nodes per level (level 0: the mesh) */
  int32_t bs[VMS_AMG_MAX_LEVELS];    /* dofs per node: 3, then 10 */
  int64_t nnzb[VMS_AMG_MAX_LEVELS];  /* blocks per level (level 0: the mesh's slots) */
  size_t device_bytes;               /* bytes vms_amg_upload needs */
} vms_amg_info;

/* Build the mesh-dependent part of a plain-aggregation multigrid hierarchy for
 * the velocity block A (host work, once per mesh): greedy aggregates of the
 * node graph (row_len, col of vms_setup_build, slot width W), the ten
 * conformal motions (translations, rotations, dilation, special conformal
 * fields) per aggregate as near-null space, zero on Dirichlet velocity
 * components (dir_mask), orthonormalised per aggregate by modified
 * Gram-Schmidt into the tentative prolongator, coarse patterns and the block
 * lists of the Galerkin products.  All arrays are HOST arrays.  *out receives
 * the object (free with vms_amg_destroy).  VMS_ERR_ARG on a bad pattern or
 * option.  Each linear solve with a_prec = VMS_APC_AMG forms the coarse
 * operators P^T A P, their block-diagonal inverses and the Chebyshev bounds on
 * the device. */
int vms_amg_create(int32_t n_nodes, int32_t slot_width, const int32_t *row_len, const int32_t *col,
                   const double *X, const uint8_t *dir_mask, const vms_amg_opts *opts, vms_amg **out);
void vms_amg_destroy(vms_amg *amg);
int vms_amg_get_info(const vms_amg *amg, vms_amg_info *info);
/* Bytes of device memory the hierarchy's fixed arrays take (vms_amg_upload). */
size_t vms_amg_device_bytes(const vms_amg *amg);
/* Copy the fixed arrays into caller-owned device memory (at least
 * vms_amg_device_bytes) on ctx's device; the object keeps the device
 * pointers, so the buffer must outlive every solve that uses the hierarchy.
 * [sync] */
int vms_amg_upload(vms_ctx *ctx, vms_amg *amg, void *device_buffer, size_t bytes);
/* HOST views of level `level` (for checks): agg[n] (coarse node of each node)
 * and P[n][bs][10] (the unscaled tentative prolongator) when a coarser level
 * follows, else NULL; for level >= 1 its CSR pattern ptr[n+1], col[] and the
 * dropped-dof mask dropped[n*10]. */
int vms_amg_level_arrays(const vms_amg *amg, int level, const int32_t **agg, const double **P,
                         const int32_t **ptr, const int32_t **col, const uint8_t **dropped);
/* z = one V-cycle of the A-levels' multigrid applied to r ([n][3] velocity
 * vectors, FP64), for the scaled velocity block of K (K->A, K->W as
 * vms_prepare_system left them; symmetrised (A + A^T)/2 when sym = 1): the
 * coarse operators, block inverses and Chebyshev bounds are formed as in a
 * solve, then the cycle is applied.  Workspace at least
 * vms_amg_apply_workspace(mesh, sym).  [sync]  VMS_ERR_BREAKDOWN if a coarse
 * diagonal block is singular. */
size_t vms_amg_apply_workspace(const vms_mesh *mesh, int sym);
int vms_amg_apply(vms_ctx *ctx, const vms_mesh *mesh, const vms_matrix *K, int sym, const double *r, double *z,
                  void *workspace, size_t workspace_bytes);

/* ---- allocation-free time step ------------------------------------------ */

/* vms_step with no workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a static device array of
 * VMS_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, which the library holds from
 * its first use on that GPU until the process ends; vms_ctx_create takes its
 * device address.  Arguments, outputs and status codes as vms_step; the
 * caller still owns the state, K and f_ext.  This call allocates nothing and
 * creates no HIP objects.
 *  - VMS_ERR_WORKSPACE (nothing launched) if vms_step_workspace(mesh, sopts)
 *    exceeds the scratch (with the default solver options: cubes up to about
 *    10^3 hexes, 8 000 tetrahedra);
 *  - VMS_ERR_STATE if launch timing is on (vms_ctx_set_timing creates its
 *    events on demand) or the context has no scratch (device index >= 64).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents; vms_step writes every workspace buffer before reading it, so no
 * part of it has to start at zero.  Calls on one GPU are serialised among the
 * host threads of the process, but calls that overlap on the device (two
 * streams or contexts of one GPU with kernels in flight at once) race on the
 * scratch and give undefined results.  [sync] */
int vms_step_noalloc(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_timeint *ti,
                     vms_state *st, const double *f_ext, vms_matrix *K, const vms_newton_opts *nopts,
                     const vms_solver_opts *sopts, vms_step_stats *stats);
/* VMS_NOALLOC_SCRATCH_BYTES, for bindings that cannot read the macro. */
size_t vms_noalloc_scratch_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* VMS_H */
