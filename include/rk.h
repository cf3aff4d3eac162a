/*
 * rk.h -- C ABI of the MI355X stage-parallel Radau IIA heat-equation library.
 *
 * Method (Munch, Dravins, Kronbichler, Neytcheva, arXiv:2209.06700):
 *   the finite-element semi-discretisation  M y' + K y = g(t)  of the heat
 *   equation u_t = Delta u + f on the unit cube with homogeneous Dirichlet
 *   conditions, continuous Q_k elements (tensor products of 1D Lagrange
 *   elements on Gauss-Lobatto points, (k+1)^3-point Gauss quadrature,
 *   Sec. 5), advanced by the Q-stage Radau IIA method (Sec. 2).  Each step
 *   solves the premultiplied stage system of eq. (irk:A),
 *       (A_Q^-1 (x) M + tau I_Q (x) K) k = (A_Q^-1 (x) I)(gbar - e (x) K y_n),
 *   with right-preconditioned flexible GMRES and the preconditioner of
 *   eq. (irk:P), P^-1 = (S (x) I)(Lam (x) M + tau I (x) K)^-1 (S^-1 (x) I),
 *   where A_Q^-1 = L U (Crout, unit-diagonal U) and L = S Lam S^-1.  Every
 *   block lam_i M + tau K is approximated by one geometric-multigrid V-cycle
 *   with a Chebyshev-Jacobi smoother and a Chebyshev coarse solve (Sec. 5).
 *   Then y_{n+1} = y_n + tau sum_i b_i k_i (Sec. 1).
 *
 *   The alternative of Sec. 6 (rk_options.method = RK_METHOD_COMPLEX)
 *   diagonalises A_Q^-1 = S Lam S^-1 directly (eq. irk:Ainv; complex S,
 *   Lam) and solves the ceil(Q/2) blocks lam_i M + tau K independently, one
 *   GMRES per block, written as two-by-two real systems
 *   [[K', -M'], [M', K']] with K' = Re(lam) M + tau K, M' = Im(lam) M
 *   (eq. complex:twobytwo) and preconditioned by PRESB (eq. presb:p): two
 *   V-cycles in sequence on H = (Re lam + Im lam) M + tau K.
 *
 * Slot layout of the complex method (RK_OP_CBLOCKS, rk_apply_preconditioner
 *   and rk_vcycle of an RK_METHOD_COMPLEX context): a [Q][N^3] vector of
 *   "slots".  With nb = ceil(Q/2) blocks (the floor(Q/2) conjugate pairs, one
 *   member each with Im lam > 0 in ascending Re lam, then the real
 *   eigenvalue for odd Q), slots 0..nb-1 hold the real parts of the pair
 *   unknowns and the real block, slots nb..Q-1 the imaginary parts: pair j
 *   owns slots j and nb + j.  slots = (T (x) I) k and k = (U (x) I) slots
 *   with the real Q x Q matrices T = U^-1 of rk_info_t.
 *
 * Vector layout (every vector argument):
 *   full grid of N = n_cells*degree + 1 nodes per direction, node (ix,iy,iz)
 *   at offset ix + N*(iy + N*iz) (x fastest); Q-stage vectors are stage-major,
 *   stage i at offset i*N^3.  Boundary nodes are part of the layout; on input
 *   they are ignored (treated as 0), on output they are written as 0.
 *   All vector pointers are DEVICE pointers owned by the caller.  The library
 *   keeps no pointer to a caller vector after a call returns.
 *
 * Memory: the caller allocates one device workspace of rk_workspace_bytes()
 *   bytes and passes it to rk_create(); the library never allocates device
 *   memory itself.  The workspace must stay alive until rk_destroy().
 *
 * Streams: all device work of a context is ordered on the HIP stream given
 *   to rk_create() (NULL = the default stream).  A batched V-cycle forks the
 *   V-cycles of some blocks onto private streams of the context (see
 *   rk_options.vc_streams) after the work already on that stream, and joins
 *   them back before any later work on it.  rk_apply_operator(),
 *   rk_vcycle() and rk_apply_preconditioner() are asynchronous; rk_create()
 *   and rk_step() return after their device work has finished.
 *
 * Errors: every function returns RK_OK (0) or a negative code; no C++
 *   exception crosses the ABI.  rk_last_error() returns a message for the
 *   last failure of a context.  One context must not be used by two host
 *   threads at the same time.
 */
#ifndef RK_H
#define RK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define RK_OK          0
#define RK_EINVAL     -1   /* bad argument: NULL pointer, size or enum out of range */
#define RK_EWORKSPACE -2   /* workspace NULL or smaller than rk_workspace_bytes() */
#define RK_EHIP       -3   /* a HIP runtime call failed; see rk_last_error() */
#define RK_ENOCONV    -4   /* FGMRES hit max_iter; y is left unchanged */

/* vector element types */
#define RK_FP64 0
#define RK_FP32 1

/* preconditioner precision (rk_options.precision) */
#define RK_PREC_FP64  0    /* V-cycles in fp64 */
#define RK_PREC_MIXED 1    /* V-cycles, smoother, transfers in fp32 with fp32
                              accumulation; FGMRES, orthogonalisation, residuals
                              and the stage combination stay fp64 */

/* block-solve mode (rk_options.mode) */
#define RK_BATCHED   0     /* all Q blocks in every kernel launch (Sec. 3, batching) */
#define RK_PER_STAGE 1     /* one block after the other (the paper's sequential IRK) */

/* stage-system solver (rk_options.method) */
#define RK_METHOD_CROUT   0   /* FGMRES on eq. (irk:A) with the preconditioner of eq. (irk:P) */
#define RK_METHOD_COMPLEX 1   /* direct diagonalisation, per-block GMRES with PRESB (Sec. 6)  */

/* operator forms for rk_apply_operator */
#define RK_OP_CALA   0     /* v = (A^-1 (x) M + tau I (x) K) u, Q stages, eq. (irk:A) */
#define RK_OP_STAGE  1     /* v = (I (x) M + tau A (x) K) u,    Q stages (stage system, Sec. 2) */
#define RK_OP_BLOCKS 2     /* v_i = (lam_i M + tau K) u_i,      Q stages, blocks of eq. (irk:P) */
#define RK_OP_K      3     /* v = K u, one vector */
#define RK_OP_M      4     /* v = M u, one vector */
#define RK_OP_CBLOCKS 5    /* v = (Lam_r (x) M + tau I (x) K) u on slot vectors: per pair
                              [[K', -M'], [M', K']], the real block lam M + tau K (Sec. 6) */

#define RK_MAX_Q      9
#define RK_MAX_DEGREE 6
#define RK_MAX_LEVELS 16

typedef struct rk_ctx rk_ctx;

/* Uniform mesh of the cube [0,length]^3 with n_cells^3 hexahedra (Sec. 5: the
   unit cube, n_cells = 2^L; here any length > 0, cell size h = length/n_cells,
   so M scales with h^3 and K with h; the deformed-mesh calls and contexts with
   deform != 0 take length = 1, the cube their mapping is defined on).  Any
   n_cells >= 1, with N = n_cells*degree + 1 <= 16384 and N*Q <= 65535.  Multigrid
   levels halve n_cells while it is even, down to the odd part of n_cells
   (rk_info_t.n_levels, rk_info_t.level_cells).  An odd n_cells therefore has a
   single level: the "V-cycle" is then the Chebyshev-Jacobi coarse solve on
   the fine grid alone, with no coarse-grid correction, and the FGMRES
   iteration count grows with n_cells*degree (tests/test_gpu_step.py pins it
   for n_cells = 15 against 16).  Use n_cells = m 2^L with a small odd m. */
typedef struct {
    int32_t n_cells;
    double  length;             /* edge of the cube, > 0 */
} rk_mesh;

typedef struct {
    int32_t precision;          /* RK_PREC_FP64 | RK_PREC_MIXED                     */
    int32_t mode;               /* RK_BATCHED | RK_PER_STAGE                        */
    double  rtol;               /* FGMRES: stop when ||rhs - A k||_2 <= rtol ||rhs||_2 */
    int32_t max_iter;           /* FGMRES iterations per step (all restarts)        */
    int32_t restart;            /* Krylov basis length before a restart             */
    int32_t cheb_degree;        /* smoother: V(nu,nu) with Chebyshev degree nu      */
    int32_t coarse_cheb_degree; /* Chebyshev degree of the coarsest-level solve     */
    double  cheb_range;         /* interval [upper/cheb_range, upper] for D^-1 A     */
    double  eig_safety;         /* upper = eig_safety * estimated lambda_max         */
    int32_t eig_iterations;     /* power iterations of that estimate                */
    const double* eig_max;      /* host [n_levels]: explicit upper bounds (fine to
                                   coarse), used as given; NULL = estimate at create */
    int32_t timing;             /* 1: fill the per-component times of rk_stats     */
    int32_t method;             /* RK_METHOD_CROUT | RK_METHOD_COMPLEX              */
    double  deform;             /* 0: the affine mesh.  Otherwise the Krylov operator
                                   and K y_n live on the deformed mesh with this eps
                                   (|eps| <= RK_MAX_DEFORM, see rk_deformed_apply);
                                   the V-cycles as selected by deform_mg             */
    int32_t autotune;           /* 1: at create, time the operator kernel's z-chunk
                                   length (1, 2, 4, 8, 16 elements) and, for an fp32
                                   preconditioner, its x-y tile shape (about 32 or 64
                                   x-nodes) on every level, separately for the V-cycle
                                   epilogues and the plain operator, and the z-chunk
                                   of the fp64 Krylov operator; keep the fastest.
                                   0: a size heuristic, the narrow tiles             */
    int32_t deform_mg;          /* deform != 0 only.  1: V-cycles on the deformed
                                   levels (each level rediscretised on its mapped mesh,
                                   stored Jacobi diagonals, Chebyshev updates as
                                   separate passes); 0: affine-mesh V-cycles          */
    int32_t vc_streams;         /* batched mode: the stage blocks of a V-cycle are
                                   split into this many groups (1..RK_MAX_Q, capped at
                                   the block count), each group on its own stream
                                   (forked from and joined back into the context's
                                   stream), so that the latency-bound coarse levels
                                   of one group overlap the fine levels of another.
                                   Applies to V-cycles of at least 2^23 fine-level
                                   stage-DoFs; smaller ones run on one stream.
                                   Results do not depend on it.  Contexts stepped
                                   concurrently (rk_step_batch) already fill the
                                   GPU; there 1 is faster.                           */
    int32_t z_chunk;            /* 0: z-chunk of the operator kernel from the
                                   autotuner (autotune = 1) or a size heuristic;
                                   1..64: this many elements per z-chunk for every
                                   operator launch of the context (no tuning).
                                   Results do not depend on it.                       */
    int32_t tile_shape;         /* with z_chunk > 0: the x-y tile shape of the fp32
                                   diagonal-mix kernels, 0 (about 32 x-nodes) or 1
                                   (about 64).  Results do not depend on it.           */
    int32_t tail_nodes;         /* affine-mesh V-cycles: the levels of at most this
                                   many nodes per stage (N^3), down to the coarsest,
                                   run in one launch with one workgroup per stage
                                   block (rk_info_t.tail_level); 0: every level
                                   launches its own kernels.  Results agree with the
                                   multi-launch V-cycle up to rounding.              */
} rk_options;

typedef struct {
    int32_t iterations;         /* FGMRES iterations of the step (complex method:
                                   lock-step iterations, the maximum over blocks)   */
    int32_t vcycles;            /* V-cycles (counted per block solve when per-stage,
                                   per batched launch sequence when batched)         */
    double  rel_residual;       /* true ||rhs - A k||_2 / ||rhs||_2 at the end (complex
                                   method: the largest block's relative residual)   */
    double  t_rhs, t_vmult, t_basis, t_blocks, t_rest;   /* seconds (timing = 1)     */
    int32_t block_iterations[RK_MAX_Q];   /* complex method: GMRES iterations of
                                   block j (j < n_blocks); zero otherwise            */
} rk_stats;

typedef struct {
    int32_t N;                  /* nodes per direction, n_cells*degree + 1          */
    int32_t n_cells, degree, Q, n_levels;
    int32_t level_cells[RK_MAX_LEVELS];   /* cells per direction, fine to coarse   */
    double  tau, h;
    double  A[RK_MAX_Q * RK_MAX_Q], b[RK_MAX_Q], c[RK_MAX_Q];   /* Butcher tableau */
    double  Ainv[RK_MAX_Q * RK_MAX_Q];
    double  L[RK_MAX_Q * RK_MAX_Q];       /* Crout factor of A^-1 (lower)           */
    double  S[RK_MAX_Q * RK_MAX_Q], Sinv[RK_MAX_Q * RK_MAX_Q];  /* L = S Lam S^-1  */
    double  lambda[RK_MAX_Q];             /* Lam = diag(L)                          */
    double  eig_max[RK_MAX_LEVELS];       /* Chebyshev upper bounds in use          */
    double  nodes[RK_MAX_DEGREE + 1];     /* Gauss-Lobatto nodes on [0,1]           */
    /* direct diagonalisation of A^-1 (eq. irk:Ainv) in the slot layout above   */
    int32_t n_blocks, n_pairs;            /* ceil(Q/2), floor(Q/2)                  */
    double  clam_re[RK_MAX_Q], clam_im[RK_MAX_Q];   /* lam of block j (Im >= 0)     */
    double  T[RK_MAX_Q * RK_MAX_Q], U[RK_MAX_Q * RK_MAX_Q];   /* row-major, T = U^-1 */
    int32_t level_cz[RK_MAX_LEVELS];      /* z-chunk of the level's block operator
                                             in the V-cycle epilogues (smoother,
                                             residual; 0: size heuristic)         */
    int32_t krylov_cz;                    /* same for the fp64 Krylov operator     */
    int32_t level_ts[RK_MAX_LEVELS];      /* tile shape of the V-cycle epilogues:
                                             0 about 32 x-nodes, 1 about 64 (fp32
                                             preconditioner only)                 */
    int32_t level_cz_store[RK_MAX_LEVELS];/* z-chunk and tile shape of the level's */
    int32_t level_ts_store[RK_MAX_LEVELS];/* plain block operator (RK_OP_BLOCKS)   */
    int32_t tail_level;                   /* first level of the one-launch coarse
                                             end of the V-cycle (-1: none)        */
} rk_info_t;

/* Fills *opt with the defaults: RK_PREC_FP64, RK_BATCHED, rtol 1e-10,
   max_iter 200, restart 30, cheb_degree 3, coarse_cheb_degree 3,
   cheb_range 15, eig_safety 1.2, eig_iterations 30, eig_max NULL, timing 0,
   RK_METHOD_CROUT, deform 0, autotune 1, deform_mg 1, vc_streams 2, z_chunk 0,
   tile_shape 0, tail_nodes 4913 (17^3). */
void rk_default_options(rk_options* opt);

/* Bytes of device workspace needed for the given mesh, degree (1..6),
   Q (1..9) and options (opt may be NULL for the defaults). */
int rk_workspace_bytes(const rk_mesh* mesh, int degree, int Q, const rk_options* opt,
                       size_t* bytes);

/* Sets up a context: Radau IIA tableau (Sec. 2), A^-1 = L U, L = S Lam S^-1
   (eq. irk:P), the direct diagonalisation of A^-1 (eq. irk:Ainv), 1D element
   data, the level hierarchy, and the Chebyshev bounds (estimated by power
   iteration on D^-1 A of every multigrid block -- lam_i M + tau K, or for
   RK_METHOD_COMPLEX the PRESB matrices H of every slot -- unless
   opt->eig_max is given; batched and per-stage runs share the largest bound
   over the blocks of a level, as in the paper's batched runs).  d_workspace:
   device memory of at least rk_workspace_bytes() bytes, 256-byte aligned.
   hip_stream: a hipStream_t or NULL.  Blocks until set-up has finished. */
int rk_create(const rk_mesh* mesh, int degree, int Q, double tau, const rk_options* opt,
              void* d_workspace, size_t workspace_bytes, void* hip_stream, rk_ctx** out);

int rk_destroy(rk_ctx* ctx);

/* Host copy of the context's sizes and Q x Q data. */
int rk_info(const rk_ctx* ctx, rk_info_t* out);

/* One Radau IIA step from t_n (Sec. 2).  d_y: fp64 [N^3], y_n on input,
   y_{n+1} on output.  The source is g(t) = gamma(t) G: d_G is an fp64 [N^3]
   load vector (int f phi_i; NULL means g = 0) and h_gamma a host array of Q
   values gamma(t_n + c_i tau) (ignored when d_G is NULL).  h_stats may be NULL.
   Returns RK_ENOCONV (y unchanged, stats filled) when max_iter is reached.
   RK_METHOD_COMPLEX: the right-hand side of eq. (irk:A) goes to the slots
   (T (x) I), every block runs its own right-preconditioned GMRES with PRESB
   until ||w_j - B_j u_j||_2 <= rtol ||w_j||_2 (all blocks advance in lock
   step, in the same kernel launches; a converged block stops contributing),
   and k = (U (x) I) u. */
int rk_step(rk_ctx* ctx, double t_n, double* d_y, const double* d_G, const double* h_gamma,
            rk_stats* h_stats);

/* One step of each of `count` independent contexts: the uneven batch of heat
   problems with different meshes, degrees, Q and tau (one context each).
   Entry i is rk_step(ctx[i], t_n[i], d_y[i], d_G[i], h_gamma + i*RK_MAX_Q,
   h_stats + i); d_G may be NULL or hold NULL entries, h_stats and h_codes may
   be NULL.  The entries run concurrently on `threads` host threads (0: one
   per entry; at most 16), each on its context's own stream, so entries on
   different streams overlap on the GPU.  Entries whose contexts share a
   stream run on one thread, in input order; the streams are handed to the
   threads largest first, each to the least loaded thread, by the sum over
   their contexts of max(N^3 Q, 2^23): below about 8M stage-DoFs a step costs
   its launch and synchronisation latency more than its size.  A context must
   appear at most once.  Every entry is attempted; per-entry codes
   go to h_codes, and the return value is the first failing entry's code
   (RK_OK if all succeeded).  Errors of an entry are reported by
   rk_last_error(ctx[i]). */
int rk_step_batch(rk_ctx* const* ctx, int count, const double* t_n, double* const* d_y,
                  const double* const* d_G, const double* h_gamma, rk_stats* h_stats, int* h_codes,
                  int threads);

/* v = op(u) for one of the RK_OP_* forms, with dtype RK_FP64 or RK_FP32 for
   both vectors.  Q-stage forms take [Q][N^3] vectors, RK_OP_K / RK_OP_M one
   [N^3] vector.  u and v must not overlap.  Asynchronous.  A context with
   deform != 0 applies RK_OP_CALA, RK_OP_CBLOCKS, RK_OP_K and RK_OP_M on the
   deformed mesh, in fp64 only; other forms return RK_EINVAL there. */
int rk_apply_operator(rk_ctx* ctx, int form, int dtype, const void* d_u, void* d_v);

/* v_i = op_i(u_i) for count contexts at once (the uneven batch of Sec. 5.4:
   problems of different meshes, degrees, Q and tau), for the diagonal-mix
   forms RK_OP_BLOCKS, RK_OP_K and RK_OP_M with each context's own
   coefficients (Sec. 3.4: all Q stage blocks of a problem in one launch).
   d_u[i], d_v[i] are device vectors of ctx[i] as rk_apply_operator() takes
   them, all in dtype (RK_FP64 or RK_FP32); no output may overlap an input or
   another output.  The (tile, z-chunk, stage) items of all problems of one
   degree go through one persistent kernel that walks them as a work list (up
   to 12 problems per launch; one launch per degree and group of 12); a
   problem of 2^23 stage-DoFs or more fills the GPU alone and takes its
   context's own tuned launch instead.
   Results equal rk_apply_operator()'s bitwise.  Asynchronous on hip_stream
   (NULL = the default stream); the caller orders it against work queued on
   the contexts' own streams.  Affine-mesh contexts only.  Errors (reported
   by rk_last_error(NULL)): RK_EINVAL for count < 1, NULL arrays, contexts
   or vectors, a deformed-mesh context, another form or dtype, overlapping
   vectors; RK_EHIP for a failed launch. */
int rk_apply_operator_batch(rk_ctx* const* ctx, int count, int form, int dtype, const void* const* d_u,
                            void* const* d_v, void* hip_stream);

/* x_i = one V-cycle for the block lam_i M + tau K applied to b_i, i = 1..Q,
   on [Q][N^3] vectors (RK_METHOD_COMPLEX: for the PRESB matrix H of slot i):
   the geometric multigrid of Sec. 5 (levels halve n_cells, transfer by the
   nested-space embedding and its transpose), V(nu,nu) with Chebyshev-Jacobi
   smoothing of degree nu = cheb_degree and a Chebyshev-Jacobi coarse solve of
   degree coarse_cheb_degree, one Chebyshev interval for all blocks (Sec. 5.4).
   dtype must be RK_FP32 for RK_PREC_MIXED contexts and RK_FP64 otherwise.
   Batched (all blocks in each launch, Sec. 3.4) or per-stage as set in the
   options.  b's boundary entries must be 0; x's are written 0.  b and x must
   not overlap.  Asynchronous. */
int rk_vcycle(rk_ctx* ctx, int dtype, const void* d_b, void* d_x);

/* z = P^-1 r (eq. irk:P) on fp64 [Q][N^3] vectors: basis change S^-1 (with
   the cast to fp32 in mixed precision), the Q block V-cycles, basis change S.
   RK_METHOD_COMPLEX: z = PRESB^-1 r on slot vectors (eq. presb:p), per pair
   g1 = V(H)(r_re + r_im), g2 = V(H)(r_im - Im(lam) M g1), z = (g1 - g2, g2),
   the real block z = V(lam M + tau K) r.
   r and z must not overlap.  Asynchronous. */
int rk_apply_preconditioner(rk_ctx* ctx, const double* d_r, double* d_z);

/* ---------------------------------------------------------------------------
 * Deformed (non-affine) meshes: the operator only (no solver).  The paper
 * works on affine meshes; Sec. 3.4 gives per-quadrature-point geometry as the
 * data that batching the stages amortises.  The mesh here is the uniform
 * n_cells^3 mesh of the unit cube mapped by
 *     Phi(x) = x + eps sin(pi x1) sin(pi x2) sin(pi x3) (1, 1, 1),
 * the identity on the boundary, with the same Q_k reference element and
 * (k+1)^3-point Gauss rule as the affine mesh; Dirichlet conditions and the
 * vector layout as above (node (ix,iy,iz) is the image of the affine node).
 * Errors of these context-free calls are reported by rk_last_error(NULL).
 * ------------------------------------------------------------------------- */
#define RK_MAX_DEFORM 0.1   /* |eps| <= 0.1 keeps det Phi' >= 0.05 */

/* Bytes of the geometry array (dtype RK_FP64 or RK_FP32): per cell and
   Gauss point 7 values, w det J and the symmetric w det J J^-1 J^-T. */
int rk_deformed_geometry_bytes(const rk_mesh* mesh, int degree, int dtype, size_t* bytes);

/* Fills the caller's device array d_geometry (rk_deformed_geometry_bytes
   bytes) for the map with amplitude eps (|eps| <= RK_MAX_DEFORM), computed
   in fp64 and stored in dtype.  Asynchronous on hip_stream (NULL = default). */
int rk_deformed_geometry(const rk_mesh* mesh, int degree, double eps, int dtype, void* d_geometry,
                         void* hip_stream);

/* v_s = h_alpha[s] M u_s + h_beta[s] K u_s for s < Q on [Q][N^3] device
   vectors of dtype (the geometry must have the same dtype), with M and K the
   deformed-mesh mass and stiffness matrices.  Cell-based sum factorisation:
   each cell's geometry is read once and applied to all Q stages.  v is
   overwritten; u and v must not overlap.  Asynchronous on hip_stream. */
int rk_deformed_apply(const rk_mesh* mesh, int degree, int Q, const double* h_alpha, const double* h_beta,
                      int dtype, const void* d_geometry, const void* d_u, void* d_v, void* hip_stream);

/* ---------------------------------------------------------------------------
 * No allocation at all: for callers that cannot allocate device memory or
 * create a context (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).
 * ------------------------------------------------------------------------- */
#define RK_STATIC_SCRATCH_BYTES (64u << 20)   /* per GPU, held until the process ends */

/* v = op(u) as rk_apply_operator() computes it on a context created with
   the same mesh, degree, Q and tau (Crout forms RK_OP_CALA, RK_OP_STAGE,
   RK_OP_BLOCKS, RK_OP_K, RK_OP_M; affine mesh), but without a context: no
   workspace, no allocation of any kind.  RK_OP_CALA and RK_OP_STAGE mix the
   input stages first; the mixed input and the Q x Q table go to a static
   device array of RK_STATIC_SCRATCH_BYTES (+ 4 KiB) that each GPU holds from
   the first such call until the process ends, so those two forms need
   Q * N^3 * sizeof(dtype) <= RK_STATIC_SCRATCH_BYTES and return RK_EINVAL
   beyond it.  All calls on one GPU share that array: calls that overlap in
   time on one GPU (two streams or two host threads) race and must be
   serialised by the caller.  u and v are the caller's device vectors and must
   not overlap.  Asynchronous on hip_stream (NULL = the default stream);
   errors are reported by rk_last_error(NULL). */
int rk_apply_operator_static(const rk_mesh* mesh, int degree, int Q, double tau, int form, int dtype,
                             const void* d_u, void* d_v, void* hip_stream);

/* Message of the last failed call on ctx (or of the last failed rk_create or
   context-free call when ctx is NULL).  The pointer stays valid until the
   next call. */
const char* rk_last_error(const rk_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RK_H */
