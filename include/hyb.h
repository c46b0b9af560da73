/*
 * hyb.h -- C ABI of the MI355X hybridization library (libhyb.so).
 *
 * Algebraic hybridization of the H(div) problem
 *     (alpha u, v) + (beta div u, div v) = (f, v)
 * on Raviart-Thomas RT_k hexahedra, k = 0..3 (Dobrev, Kolev, Lee, Tomov,
 * Vassilevski, "Algebraic hybridization and static condensation with
 * application to scalable H(div) preconditioning", arXiv:1801.08914).
 * Letters: alpha is the mass coefficient and beta the div-div coefficient
 * (the paper's Sec. 3.2 uses the opposite letters).
 *
 * Theorem 2.1: with the block-diagonal broken matrix A_hat = blockdiag(M_T)
 * and a constraint matrix C whose null space is the conforming subspace, the
 * Lagrange multipliers solve H lambda = C A_hat^{-1} f_hat with the SPD matrix
 * H = C A_hat^{-1} C^T, and the broken solution is
 * x_hat = A_hat^{-1} (f_hat - C^T lambda).  H is the sum over elements of
 * H_T = C_T M_T^{-1} C_T^T, the inverse of the element Schur complement on
 * its face dofs with signs (Sec. 3.1 and Sec. 5).
 *
 * Call order: hyb_plan_create (host only, no GPU needed) -> hyb_bind ->
 * hyb_setup -> [hyb_rhs] -> hyb_pcg -> hyb_recover -> hyb_destroy, or
 * hyb_setup -> hyb_solve (rhs + PCG + recovery) for each new load.
 *
 * Conventions (fixed by this library; the paper leaves them to its FE code):
 *   - element vertex v = a + 2b + 4c sits at reference corner (a,b,c) of
 *     [0,1]^3; the geometry is the trilinear map of the 8 vertices and every
 *     element must have det J > 0;
 *   - face f = 2d + s is the face xi_d = s, outward sign eps_f = 2s - 1;
 *     faces on the domain boundary are essential (prescribed normal flux g)
 *     unless hyb_mesh.ess marks them natural;
 *   - local dof order is interior dofs first (3 k (k+1)^2 of them), then the
 *     (k+1)^2 dofs of face 0, ..., face 5; a face dof (j0, j1) has index
 *     n_i + f (k+1)^2 + j0 + (k+1) j1; dofs are nodal normal components at
 *     Gauss-Lobatto (normal direction) x Gauss-Legendre (tangential) nodes;
 *   - interior faces are numbered by increasing (owner, owner's local face),
 *     the owner being the element with the smaller index; multiplier
 *     mu = face (k+1)^2 + j0 + (k+1) j1 in the owner's face frame;
 *   - H is CSR: rows mu ascending, columns ascending, int64 row_ptr, int32
 *     columns, double values.
 *
 * Errors: every call returns HYB_OK (0) or a negative HYB_E_* code; no
 * exception crosses the ABI.  Device-side failures (det J <= 0 at a
 * quadrature point, a non-positive Cholesky pivot) are recorded in the bound
 * status buffer and reported by hyb_status after the stream is synchronised.
 * Device calls are asynchronous on the stream given in hyb_opts.
 *
 * Memory: the caller owns every device buffer (hyb_buffers); the plan owns
 * only host metadata.  Device pointers must stay valid until hyb_destroy.
 */
#ifndef HYB_H
#define HYB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hyb_status_code {
  HYB_OK = 0,
  HYB_E_ARG = -1,       /* bad argument: k outside 0..3, null pointer, size */
  HYB_E_MESH = -2,      /* vertex id out of range, face shared by > 2 elements */
  HYB_E_JACOBIAN = -3,  /* det J <= 0 (host corner check or device qp check) */
  HYB_E_NOT_SPD = -4,   /* non-positive pivot in an element Cholesky */
  HYB_E_STATE = -5,     /* call out of order (e.g. rhs before setup) */
  HYB_E_NOMEM = -6,     /* a bound buffer is missing */
  HYB_E_NOCONV = -7,    /* PCG did not reach rtol within maxit */
  HYB_E_HIP = -8,       /* HIP runtime error; detail holds the hipError_t */
  HYB_E_INTERNAL = -9,  /* the plan broke one of its own invariants (a bug) */
  HYB_E_REFINE = -10    /* reserved (HYB_MIXED elements whose FP32 factor
                           breaks down or whose refinement fails are solved
                           in FP64 instead, see hyb_fallback_count) */
};

enum hyb_precision {
  HYB_FP64 = 0,         /* every step in double precision */
  HYB_MIXED = 1         /* element Cholesky and triangular solves in FP32
                           on the matrix cores (after an exact power-of-two
                           diagonal scaling), refined against the FP64
                           element matrix (residuals on the FP64 matrix
                           cores); the element matrix, the residuals, H, r,
                           the solve and u are FP64.  An element whose FP32
                           factor breaks down or whose refinement fails the
                           backward-error test is solved in FP64 (counted by
                           hyb_fallback_count).  The factor record holds
                           X = M_T^{-1} C_T^T (n x nb, column-major) and
                           recovery is u_T = y_T - X lambda_T (y_T = M_T^{-1}
                           f_hat_T in the y buffer); hyb_rhs re-assembles M_T
                           and re-derives the FP32 factor from the
                           coefficients of the last setup */
};

/* Reduced system a plan assembles (Sec. 3.1 of the paper: hybridization
 * assembles the inverses of the element Schur complements onto the face
 * multipliers, static condensation the complements themselves onto the face
 * dofs, S = [I; W]^T S_hat [I; W] with W = -I for outward-flux copies). */
enum hyb_system {
  HYB_HYBRID = 0,
  HYB_STATIC = 1
};

typedef struct hyb_mesh {
  int64_t nv;             /* number of vertices */
  int64_t ne;             /* number of hexahedra */
  const double* xyz;      /* host, nv x 3, row-major */
  const int32_t* e2v;     /* host, ne x 8, vertex v = a + 2b + 4c */
  const uint8_t* ess;     /* host, ne x 6 (element, local face), or NULL:
                             every boundary face is essential.  For a
                             boundary face, nonzero = essential (normal flux
                             prescribed by g; its dofs are eliminated, Sec. 5)
                             and 0 = natural (its dofs stay unknowns of the
                             element and carry no multiplier).  Entries of
                             interior faces are not read.  Copied by
                             hyb_plan_create. */
} hyb_mesh;

typedef struct hyb_opts {
  int precision;          /* HYB_FP64 or HYB_MIXED */
  void* stream;           /* hipStream_t for every device call; NULL = null stream */
  int kernel_variant;     /* 0: automatic (order- and geometry-specific kernels
                             where they apply), 1: the generic kernels only */
  int refine_sweeps;      /* HYB_MIXED: refinement sweeps after the FP32
                             solve (0: none, the unrefined form; at most 16);
                             < 0: per element while the correction keeps
                             shrinking (stop at ||dx|| <= 2^-53 ||x|| or
                             ||dx|| > ||dx_prev|| / 2; at most 30 sweeps),
                             then the element is solved in FP64 unless
                             ||b - M x|| <= sqrt(n) 2^-53 ||M|| ||x||
                             (inf-norms) */
  int pcg_reduce;         /* where hyb_pcg sums its per-block partials:
                             0 automatic (by size), 1 inside the consuming
                             kernels, 2 in separate one-block kernels; the
                             results are the same bits either way */
  int system;             /* HYB_HYBRID: the multiplier system H lambda = r
                             (default); HYB_STATIC: the static condensation
                             S x = r on the same face dofs (x = the owner's
                             outward flux), with the same CSR pattern, solve
                             and recovery calls (HYB_FP64, generic kernels) */
  int weighted_c;         /* 1: the constraint from the bilinear form
                             (Example 2.3 of the paper), C = M_s C_0 with
                             M_s the face mass matrix of the multiplier
                             space: H' = M_s H M_s, r' = M_s r, lambda' =
                             M_s^{-1} lambda, u unchanged (HYB_HYBRID) */
  int quad_q;             /* Gauss-Legendre points per direction of the
                             element quadrature: 0 or k + 2 (the rule the
                             kernels are built for); any other value is
                             HYB_E_ARG */
} hyb_opts;

/* Sizes of the caller-owned device buffers, filled by hyb_plan_create. */
typedef struct hyb_sizes {
  int64_t ne;             /* elements */
  int32_t k;              /* order */
  int32_t n_local;        /* broken dofs per element, 3 (k+1)^2 (k+2) */
  int32_t n_interior;     /* 3 k (k+1)^2 */
  int32_t n_face_dofs;    /* (k+1)^2 */
  int64_t n_faces;        /* interior faces */
  int64_t n_boundary_faces;
  int64_t m;              /* multipliers = n_faces (k+1)^2 */
  int64_t nnz;            /* nonzeros of H */
  int64_t factor_len;     /* doubles per element in the factor buffer */
  int64_t bytes_maps;     /* device map buffer (topology, geometry, tables) */
  int64_t bytes_factor;   /* factor buffer bytes (ne * factor_len * 8) */
  int64_t bytes_y;        /* cached L^{-1} f_hat buffer bytes (>= ne * n_local * 8) */
  int64_t bytes_work;     /* PCG work vectors and reductions; setup and rhs
                             also use it as scratch (contents not kept) */
} hyb_sizes;

/* Caller-allocated device buffers (e.g. torch tensors' data pointers). */
typedef struct hyb_buffers {
  void* maps;             /* bytes_maps */
  double* factor;         /* bytes_factor */
  double* y;              /* bytes_y */
  int64_t* row_ptr;       /* m + 1 */
  int32_t* col;           /* nnz */
  double* val;            /* nnz */
  double* r;              /* m: the reduced right-hand side */
  double* work;           /* bytes_work */
  int32_t* status;        /* 4 ints: code, first failing element, mixed-form
                             FP64 fallback count, spare */
} hyb_buffers;

typedef struct hyb_solve_info {
  int32_t iters;          /* PCG iterations done */
  int32_t converged;      /* 1 if ||r_k|| <= rtol ||r_0|| */
  double rel_res;         /* ||r_k|| / ||r_0|| (2-norm) */
} hyb_solve_info;

typedef struct hyb_plan hyb_plan_t;

/*
 * Host-only planning (Sec. 2.3 and Sec. 5: the constraint structure).  Copies
 * the mesh, hashes faces, finds owners and the neighbour frame codes, numbers
 * the multipliers, builds the CSR pattern of H and the per-element scatter
 * slots, and checks det J > 0 at the 8 corners of every element.  Needs no
 * GPU.  On success *out owns the plan (free with hyb_destroy).
 * Errors: HYB_E_ARG, HYB_E_MESH, HYB_E_JACOBIAN (detail via hyb_last_detail).
 */
int hyb_plan_create(const hyb_mesh* mesh, int k, const hyb_opts* opt,
                    hyb_plan_t** out, hyb_sizes* sizes);

/*
 * Host copies of the plan's topology, for checks (any pointer may be NULL):
 * elem_face ne x 6 (interior face id or -1), elem_pi ne x 6 (neighbour frame
 * code, 0 for owners and boundary faces), face_owner n_faces x 2 and
 * face_nbr n_faces x 2 (element, local face), row_ptr m + 1, col nnz.
 */
int hyb_plan_topology(const hyb_plan_t* plan, int32_t* elem_face, uint8_t* elem_pi,
                      int32_t* face_owner, int32_t* face_nbr,
                      int64_t* row_ptr, int32_t* col);

/* Element id (or other detail) of the last error on this thread. */
int64_t hyb_last_detail(void);

/*
 * Attach caller-owned device buffers and upload the maps, row_ptr and col
 * (asynchronously on the plan's stream).  Errors: HYB_E_NOMEM if a required
 * pointer is NULL, HYB_E_HIP.
 */
int hyb_bind(hyb_plan_t* plan, const hyb_buffers* buf);

/*
 * Local assembly, factorization and global assembly (Sec. 5):
 * per element, M_T by Gauss quadrature (q = k+2 per direction), boundary-face
 * rows/columns replaced by identity, M_T = L L^T in i-first order, the face
 * block L_bb inverted, H_T = D L_bb^{-T} L_bb^{-1} D (D = diag(eps)) and its
 * scatter into H.val (each entry is a sum of at most two element terms).
 * alpha, beta: device, ne doubles.  If f (device, ne x 3, element-constant
 * load) is non-NULL the right-hand side is formed as in hyb_rhs in the same
 * pass.  g (device, ne x 6 (k+1)^2 boundary normal-flux dofs, NULL = 0) is
 * only read with f.  alpha and beta must stay valid while hyb_rhs is called
 * with boundary data g (the correction -M_re g_e reassembles M_T from them).
 */
int hyb_setup(hyb_plan_t* plan, const double* alpha, const double* beta,
              const double* f, const double* g);

/*
 * Right-hand side for a new load on the current factors (Theorem 2.1):
 * f_hat_T by quadrature (minus M_re g_e), y_T = L^{-1} f_hat_T (kept for
 * recovery), r = sum_T C_T M_T^{-1} f_hat_T into the bound r buffer.
 * Errors: HYB_E_STATE before hyb_setup.
 */
int hyb_rhs(hyb_plan_t* plan, const double* f, const double* g);

/*
 * Jacobi-preconditioned CG on the reduced system H lambda = r (Sec. 6.1 of
 * the paper solves it with PCG and stops on the relative l2 residual; the
 * preconditioner here is the diagonal of H).  Deterministic reductions; stops
 * when ||r_k||_2 <= rtol ||r_0||_2 (tested every 8 iterations) or after maxit
 * iterations.  lambda: device, m doubles (the initial guess is zero; output:
 * the solution).  Needs hyb_setup with f or hyb_rhs.  Returns HYB_E_NOCONV if
 * not converged (lambda then holds the last iterate), HYB_E_STATE before a
 * right-hand side, HYB_E_ARG for a null lambda or maxit < 0.
 */
int hyb_pcg(hyb_plan_t* plan, double rtol, int maxit, double* lambda, hyb_solve_info* info);

/*
 * hyb_pcg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same iteration and the same bits as hyb_pcg, with its work vectors,
 * partial sums and scalars in a 48 MiB array that the library holds on each
 * GPU it runs on until the process ends (the plan's work buffer is not
 * touched).  Calls nothing that allocates.  Plans whose PCG work exceeds the
 * array (about 8 (6 m) bytes, m up to about 1.0e6 multipliers) get HYB_E_ARG
 * with the bytes needed in hyb_last_detail.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind: calls that overlap on one
 * GPU (other streams, other host threads) race.  Other errors as hyb_pcg.
 */
int hyb_pcg_noalloc(hyb_plan_t* plan, double rtol, int maxit, double* lambda, hyb_solve_info* info);

/*
 * The whole solve for a load on the current factors (Theorem 2.1): the
 * right-hand side as hyb_rhs (f: device ne x 3, g: device boundary data or
 * NULL), H lambda = r by hyb_pcg (rtol, maxit), then the recovery of u as
 * hyb_recover.  lambda: device, m doubles; u: device, ne x n_local doubles.
 * Errors: those of the three calls; on HYB_E_NOCONV u is still recovered
 * from the last iterate and info says so.  HYB_E_STATE before hyb_setup.
 */
int hyb_solve(hyb_plan_t* plan, const double* f, const double* g, double rtol, int maxit, double* lambda,
              double* u, hyb_solve_info* info);

/*
 * HYB_MIXED: the number of elements that the last hyb_setup or hyb_rhs (or
 * batch setup) solved in FP64 because their FP32 factor broke down or their
 * refinement failed the backward-error test (0 for HYB_FP64 plans).
 * Synchronises the plan's stream.  Errors: HYB_E_ARG, HYB_E_STATE (not
 * bound), HYB_E_HIP.
 */
int hyb_fallback_count(hyb_plan_t* plan, int64_t* count);

/*
 * Device pointers of the reduced matrix H in the bound buffers (borrowed,
 * valid while the buffers are): row_ptr (m + 1, int64), col (nnz, int32),
 * val (nnz, double; holds H after hyb_setup), and m, nnz.  Any output may be
 * NULL.  Errors: HYB_E_ARG (null plan), HYB_E_STATE (not bound).
 */
int hyb_get_csr(const hyb_plan_t* plan, const int64_t** row_ptr, const int32_t** col, const double** val,
                int64_t* m, int64_t* nnz);

/*
 * Recovery of the broken flux (Theorem 2.1 back substitution):
 * u_T = M_T^{-1} (f_hat_T - C_T^T lambda_T), boundary dofs = g.
 * lambda: device, m doubles; u: device, ne x n_local doubles, local order.
 * Errors: HYB_E_STATE before hyb_rhs / hyb_setup with f.
 */
int hyb_recover(hyb_plan_t* plan, const double* lambda, double* u);

/*
 * Synchronise the plan's stream and read the device status: returns HYB_OK
 * or the first device error (HYB_E_JACOBIAN / HYB_E_NOT_SPD); *detail (may
 * be NULL) receives the failing element.
 */
int hyb_status(hyb_plan_t* plan, int64_t* detail);

/* Launch the plan's later work on stream (a hipStream_t; NULL: the null
 * stream).  The caller orders it after work already queued on the old
 * stream.  Errors: HYB_E_ARG. */
int hyb_set_stream(hyb_plan_t* plan, void* stream);

/* Static text for a status code. */
const char* hyb_strerror(int code);

/*
 * Kernel timing with HIP events recorded on the plan's stream around every
 * launch of the element setup kernel and of the recovery kernel.
 * hyb_timing_enable(plan, 1) starts collecting (and clears earlier pairs);
 * hyb_timing_read synchronises on the last event and returns the summed
 * milliseconds and launch counts of each kernel since enabling (any output
 * pointer may be NULL), then clears them.
 */
int hyb_timing_enable(hyb_plan_t* plan, int on);
int hyb_timing_read(hyb_plan_t* plan, double* ms_setup, int* n_setup, double* ms_recover, int* n_recover);

/* Free the plan's host state (device buffers stay with the caller). */
void hyb_destroy(hyb_plan_t* plan);

/*
 * ---------------------------------------------------------------------------
 * Batches of independent problems of mixed order and mesh (the uneven batch
 * of many small hybridization problems; each problem is a bound plan).  After
 * one launch that clears the same-face blocks of every H, the setup of the
 * FP64 problems runs as a few launches per order present, most expensive
 * order first, and the recovery likewise: up to eight problems per launch,
 * their descriptors in the kernel arguments, one grid range per problem, in
 * the single-plan kernels' teams.
 * Every order uses the generic element routines (Gauss quadrature, packed
 * Cholesky, inverse of the face block), so a batch sets its plans to that
 * record layout; H, r, y and u of each problem equal those of the plan's own
 * calls.  HYB_MIXED plans run the mixed-precision element routines (the
 * same as their own calls, so again the same bits) in one persistent launch
 * per phase, after the FP64 problems' launches, whose work items (problem,
 * run of element blocks) are sorted by cost and taken from a work queue (an
 * atomic counter, most expensive first) by a grid of
 * blocks_per_cu x (compute units) workgroups.
 * With graphs enabled the launch sequences are captured into hipGraphs
 * on the batch's own stream (ordered after and before the plans' stream by
 * events) and replayed; descriptors are copies (device arrays and kernel
 * arguments), so new coefficient values written into the same buffers need
 * no re-capture, and hyb_batch_set with other buffers re-captures.
 * The batch allocates a few small device arrays itself (descriptors, work
 * list); the plans' buffers stay caller-owned and must outlive the batch.
 */
typedef struct hyb_batch hyb_batch_t;

typedef struct {
  int32_t blocks_per_cu;    /* mixed problems' grid = blocks_per_cu x CUs (0: 2) */
  int32_t items_per_block;  /* element blocks per work item (0: 1) */
} hyb_batch_tiles;

/* plans: count bound plans (the batch keeps pointers, it does not own them),
 * launched on plans[0]'s stream; FP64, HYB_MIXED and HYB_STATIC plans may
 * be mixed (a static-condensation plan assembles S and recovers from the
 * face dofs x given as its lambda, as its own calls do).
 * Errors: HYB_E_ARG, HYB_E_STATE (unbound), HYB_E_NOMEM, HYB_E_HIP. */
int hyb_batch_create(hyb_plan_t* const* plans, int32_t count, hyb_batch_t** out);

/* Device inputs of problem p: alpha, beta (ne), f (ne x 3, NULL: matrix
 * only), g (boundary data, read with f, NULL = 0), lambda (m) and u (ne x n)
 * for the recovery (may be NULL until hyb_batch_recover). */
int hyb_batch_set(hyb_batch_t* b, int32_t p, const double* alpha, const double* beta, const double* f,
                  const double* g, const double* lambda, double* u);

/* Setup (as hyb_setup of every plan) / recovery (as hyb_recover) of every
 * problem.  Errors: HYB_E_STATE (inputs missing), HYB_E_HIP; element errors
 * are recorded in each plan's status. */
int hyb_batch_setup(hyb_batch_t* b);
int hyb_batch_recover(hyb_batch_t* b);

/* Work-list tiles (HYB_E_ARG outside 0..64 / 0..1024), and the tiles in use. */
int hyb_batch_set_tiles(hyb_batch_t* b, const hyb_batch_tiles* tiles);
int hyb_batch_get_tiles(const hyb_batch_t* b, hyb_batch_tiles* tiles);

/* Capture and replay the launch sequences as hipGraphs (1) or launch
 * directly (0). */
int hyb_batch_graph(hyb_batch_t* b, int enable);

/* Autotuner: times reps setup + recovery passes for every candidate tile
 * pair (blocks_per_cu in {1,2,4,8} x items_per_block in {1,2,4,8}) on the
 * batch's own inputs (HIP events), keeps the fastest and returns it in best
 * (may be NULL).  The tiles shape the mixed problems' persistent launch; a
 * batch without mixed problems keeps the default pair.  Needs every input
 * of hyb_batch_set; overwrites the outputs. */
int hyb_batch_autotune(hyb_batch_t* b, int reps, hyb_batch_tiles* best);

/*
 * Timing of the batch phases with HIP events recorded on the stream each
 * phase runs on (the batch's own stream on graph replays): one pair around
 * every setup phase (the clearing of the same-face blocks, then the setup
 * launches) and one around every recovery phase.
 * hyb_batch_timing_enable(b, 1) starts collecting (and drops earlier pairs;
 * the autotuner's passes are not timed); hyb_batch_timing_read synchronises
 * and returns the summed milliseconds and counts of each phase since
 * enabling (outputs may be NULL), then clears them.  Errors: HYB_E_ARG,
 * HYB_E_HIP.
 */
int hyb_batch_timing_enable(hyb_batch_t* b, int on);
int hyb_batch_timing_read(hyb_batch_t* b, double* ms_setup, int* n_setup, double* ms_recover, int* n_recover);

void hyb_batch_destroy(hyb_batch_t* b);

#ifdef __cplusplus
}
#endif

#endif /* HYB_H */
