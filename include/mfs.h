/* mfs.h -- C ABI of libmfs: the hot path of the multibody MFS scattering method
 * (Cai, Bagge, Martinsson, "A stable and fast method for solving multibody scattering problems
 * via the method of fundamental solutions") on AMD Instinct MI355X (gfx950).
 *
 * Conventions for every entry point
 *   - Every call returns an mfs_status: 0 on success, a negative code on failure.  No call
 *     throws, aborts or exits.  On failure mfs_last_error() returns a thread-local message.
 *   - Arguments are validated before any work is enqueued; a rejected call leaves outputs
 *     untouched.  HIP runtime failures map to MFS_ERR_HIP with the HIP error string.
 *   - "device" pointers are HIP device memory owned by the caller; the library never frees
 *     them.  "host" pointers are ordinary host memory, read during the call only.
 *   - Complex numbers are interleaved (re, im): complex128 = 2 x double, complex64 = 2 x float.
 *   - Multi-right-hand-side vectors are RHS-major, [R][N]: element (r, i) at r * N + i.
 *   - The global unknowns are ordered body by body: body tau owns the k_tau consecutive
 *     entries starting at the prefix sum of k over bodies 0..tau-1 (its equivalent points
 *     x_hat in the order of its shape template).
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).  Calls marked
 *     "asynchronous" only enqueue work on that stream; calls marked "synchronous" return
 *     after their work has finished.
 *   - All memory the library allocates for itself (scene tables, workspaces, Krylov bases)
 *     is owned by the scene or freed before return.
 */
#ifndef MFS_H_
#define MFS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFS_OK = 0,
  MFS_ERR_ARG = -1,    /* invalid argument: null pointer, bad size, bad enum, unsupported combination */
  MFS_ERR_NOMEM = -2,  /* device allocation failed */
  MFS_ERR_HIP = -3,    /* HIP runtime error (message in mfs_last_error) */
  MFS_ERR_GEOM = -4,   /* geometry not admissible (points coincide, body outside its proxy surface) */
  MFS_ERR_RANK = -5,   /* a least-squares factorisation has rank zero */
  MFS_ERR_NOCONV = -6  /* iteration limit reached before the tolerance; outputs hold the last iterate */
} mfs_status;

typedef enum {
  MFS_FP64 = 0,  /* all arithmetic in double precision */
  MFS_FP32 = 1,  /* pair sums and S products in single precision */
  MFS_MIXED = 2  /* solve only: FP32 operator inside FP64 GMRES, FP64 iterative refinement */
} mfs_prec;

/* Message for the last failure on this thread ("" if none).  Valid until the next call. */
const char* mfs_last_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int mfs_version(void);

/* ------------------------------------------------------------------------------------------
 * Scattering matrix of one shape (Sec. 4 of the paper, eq. scattering-matrix).
 *
 * Point sets are host FP64 arrays, point-major [count][dim], in the body frame:
 *   colloc  m collocation points x_i on the boundary Gamma           (Sec. 3.1)
 *   src     n MFS sources y_j inside Gamma                            (Sec. 3.1-3.2)
 *   proxy   p proxy points z_i on a surface Psi enclosing Gamma       (Sec. 4.1-4.2)
 *   eqpts   k equivalent points x_hat where incoming fields are sampled and outgoing fields
 *           are represented.  NULL selects paper mode: x_hat is the skeleton of the
 *           collocation points found by column-pivoted QR of B (Sec. 4.2), stopped at relative
 *           precision eps_skel and capped at k_cap points.
 * Matrices (all phi_kappa): A = phi(x - y) m x n, B = phi(z - x) p x m, D = phi(z - y) p x n,
 * B_hat = phi(z - x_hat) p x k.
 *   paper mode:  S = Z* C A^+ U with B ~= B(:, I) Z*, U = conj(Z), B C = D        (Sec. 4.2-4.5)
 *   given x_hat: S = (B_hat^+ D) A^+ (B_hat^+ B)^T (the same steps with B_hat in place of
 *                B(:, I); it equals the paper-mode formula when x_hat is a skeleton)
 * Least-squares solves use Householder QR with column pivoting in FP64, truncated where the
 * pivot's remaining column norm falls to eps_ls times the first pivot's (basic solution).
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t dim;          /* 2 or 3 */
  double kappa;         /* wavenumber > 0 */
  const double* colloc; /* host, [m][dim] */
  int64_t m;
  const double* src;    /* host, [n][dim], n <= m */
  int64_t n;
  const double* proxy;  /* host, [p][dim] */
  int64_t p;
  const double* eqpts;  /* host, [k][dim], or NULL for paper mode */
  int64_t k;            /* given mode: number of equivalent points (k <= p) */
  double eps_skel;      /* paper mode: relative CPQR stopping precision (e.g. 1e-10) */
  double eps_ls;        /* relative truncation of the least-squares solves (e.g. 1e-13) */
  int64_t k_cap;        /* paper mode: maximum skeleton size (<= min(p, m)) */
} mfs_shape_desc;

/* Build S for one shape.  Synchronous.
 *   S64_dev       device, complex128, column-major k x k (S(i,j) at i + j*k); capacity k*k
 *                 (paper mode: k_cap*k_cap).  Required.
 *   S32_dev       device, complex64 copy of S in the same layout, or NULL.
 *   k_out         host, receives k (paper mode: the skeleton size).  Required.
 *   skel_idx_out  host, int64[k_cap]: paper mode receives the skeleton indices into colloc
 *                 (the equivalent points are colloc[skel_idx]); ignored in given mode; may be NULL.
 *   diag_out      host, double[4] or NULL: {numerical rank of A, numerical rank of B_hat (or of B
 *                 in paper mode), |R_11|/|R_rr| of the B_hat (B) factorisation, ||S - S^T||_F/||S||_F}.
 * Errors: MFS_ERR_ARG (sizes, dim, null), MFS_ERR_RANK (a factorisation of rank 0),
 *         MFS_ERR_NOMEM, MFS_ERR_HIP. */
mfs_status mfs_build_S(const mfs_shape_desc* desc, void* S64_dev, void* S32_dev, int64_t* k_out,
                       int64_t* skel_idx_out, double* diag_out, void* stream);

/* ------------------------------------------------------------------------------------------
 * Scene: T bodies, each a translated copy of one of n_shapes shapes (bodies of one shape share
 * one S; Sec. 5.1 Example 4).  The scene packs the global equivalent points
 * x_hat = template[shape_of[tau]] + centres[tau] on the device in FP64 (absolute) and in FP32
 * (relative to the middle of the bounding box of the centres), with body tables.
 * ------------------------------------------------------------------------------------------ */
typedef struct mfs_scene mfs_scene;

/* Create a scene.  Synchronous; packing runs on a private stream of the calling thread and does
 * not wait for work on other streams.
 *   dim, kappa      2 or 3; wavenumber > 0
 *   T               number of bodies >= 1
 *   shape_of        host int32[T], values in [0, n_shapes)
 *   centres         host double[T][dim]
 *   rotations       host double[T][dim][dim] (row-major), the orientation R_tau of each body, or
 *                   NULL for none: body tau's points are R_tau p + c_tau for every point p of its
 *                   shape.  A body's S, A and U depend only on distances, so turned copies share
 *                   their shape's matrices (Sec. 5.1, Example 4).  Each must be a proper rotation.
 *   k_of_shape      host int64[n_shapes], equivalent points per shape (1..4096)
 *   eq_template     host array of n_shapes pointers to double[k_s][dim] (body frame)
 *   S64_dev         host array of n_shapes device pointers to complex128 k_s x k_s column-major
 *   S32_dev         host array of n_shapes device pointers to complex64 copies, or NULL
 *                   (then FP32 and mixed operations return MFS_ERR_ARG)
 * The S buffers stay owned by the caller and must outlive the scene.  Total N = sum k <= 2^31-1.
 * Errors: MFS_ERR_ARG, MFS_ERR_NOMEM, MFS_ERR_HIP. */
mfs_status mfs_scene_create(int32_t dim, double kappa, int64_t T, const int32_t* shape_of,
                            const double* centres, const double* rotations, int32_t n_shapes, const int64_t* k_of_shape,
                            const double* const* eq_template, const void* const* S64_dev,
                            const void* const* S32_dev, mfs_scene** out);

/* Destroy a scene.  Its device blocks go back to the library's allocation cache, ordered after
 * the work enqueued on the stream of the scene's latest call, so the call returns at once and
 * does not wait for other streams.  Work on a different stream that still reads the scene must be
 * complete before this call. */
mfs_status mfs_scene_destroy(mfs_scene* scene);

/* N (global unknowns), T, and device bytes the scene holds now.  Host outputs may be NULL. */
mfs_status mfs_scene_size(const mfs_scene* scene, int64_t* N_out, int64_t* T_out, size_t* bytes_out);

/* Copy the packed FP64 equivalent points x_hat (absolute coordinates) to host double[N][dim].
 * Synchronous. */
mfs_status mfs_scene_points(const mfs_scene* scene, double* xhat_host);

/* ------------------------------------------------------------------------------------------
 * Hot path.
 * ------------------------------------------------------------------------------------------ */

/* Sound-soft plane-wave data at the equivalent points: vhat[r][i] = -exp(i kappa d_r . x_hat_i)
 * (v = -u_inc, footnote to eq. BVP).  Asynchronous.
 *   dirs_host  host double[R][dim], unit directions d_r
 *   vhat_dev   device complex128 [R][N] (output) */
mfs_status mfs_plane_wave(const mfs_scene* scene, const double* dirs_host, int32_t R, void* vhat_dev,
                          void* stream);

/* Off-body pair sum t = G_hat q, G_hat(i,j) = phi_kappa(x_hat_i - x_hat_j) for points on different
 * bodies and 0 on the diagonal blocks (eq. Gmtx-entries, eq. mbody2).  Asynchronous.
 *   q_dev, t_dev  device [R][N]; complex128 for MFS_FP64, complex64 for MFS_FP32; t != q. */
mfs_status mfs_ghat_apply(const mfs_scene* scene, const void* q_dev, void* t_dev, int32_t R,
                          mfs_prec prec, void* stream);

/* Block-diagonal scattering matrices: y = beta * q + S t, y_tau = beta q_tau + S_shape(tau) t_tau
 * (eq. mbody1).  beta = 0 gives the right-hand side b = S vhat (eq. mbody2) with t = vhat.
 * Asynchronous.  q_dev may be NULL when beta = 0.  Types as for mfs_ghat_apply. */
mfs_status mfs_s_apply(const mfs_scene* scene, const void* q_dev, const void* t_dev, void* y_dev,
                       double beta, int32_t R, mfs_prec prec, void* stream);

/* The operator of eq. mbody2: y = q + S G_hat q.  Asynchronous.
 *   q_dev, y_dev  device [R][N]; complex128 (MFS_FP64) or complex64 (MFS_FP32); y != q. */
mfs_status mfs_apply(const mfs_scene* scene, const void* q_dev, void* y_dev, int32_t R, mfs_prec prec,
                     void* stream);

/* GMRES solve of (I + S G_hat) qhat = S vhat (eq. mbody2, Sec. 2.3), from x0 = 0 or a given x0.
 *   MFS_FP64:  restarted GMRES(restart) with the FP64 operator.
 *   MFS_MIXED: iterative refinement: r = b - A x with the FP64 operator, then GMRES with the FP32
 *              operator and FP64 Krylov vectors on A d = r to relative tolerance inner_tol,
 *              x += d; repeated until ||b - A x|| / ||b|| <= tol (FP64 residual) or max_refine.
 *              With deflate = 1 the correction solves after the first run on the operator
 *              deflated by the first inner solve's Krylov space (GCRO) instead of afresh.
 * Each right-hand side has its own Krylov space (unless block = 1, below); the R operator
 * applications of one iteration share one pair-kernel launch.  Orthogonalisation is classical Gram-Schmidt with a second pass
 * where the first one cancelled (||w'|| < 0.1 ||w||).  The stopping test is
 * ||b - A x||_2 / ||b||_2 <= tol per column, checked with the FP64 operator before returning.
 * Synchronous.
 *   vhat_dev  device complex128 [R][N]: Dirichlet data at x_hat (b = S vhat is formed inside)
 *   qhat_dev  device complex128 [R][N]: solution (output; input too when use_x0 = 1)
 *   info      host, may be NULL. */
typedef struct {
  double tol;        /* relative residual target, e.g. 1e-8 */
  int32_t maxit;     /* total inner iterations (operator applications) allowed */
  int32_t restart;   /* Krylov basis size before a restart (1..32768); the basis takes
                        (restart+1) * R * N * 16 bytes of device memory (8 with basis32) */
  int32_t max_refine;/* MFS_MIXED: outer refinement steps allowed */
  double inner_tol;  /* MFS_MIXED: smallest relative residual reduction asked of an inner solve; the
                        last steps ask only for the reduction the outer tolerance still needs */
  mfs_prec prec;     /* MFS_FP64 or MFS_MIXED */
  int32_t verbose;   /* >0: one line per restart/refinement on stderr; >1: also every 250 steps */
  double fp64_until; /* MFS_MIXED: within a cycle, apply the FP64 operator while the residual
                        estimate is above this value and the FP32 one below it (inexact Krylov:
                        early steps need the accurate operator); 0 = FP32 throughout */
  int32_t use_x0;    /* 1: qhat_dev holds an initial guess (warm start, or resuming a checkpointed
                        solve: the FP64 residual is recomputed first); 0: x0 = 0 */
  int32_t use_graph; /* 1: replay the Gram-Schmidt, Givens and basis-update launches of each Arnoldi
                        step from HIP graphs (one captured per 64 steps, the step index read from
                        device memory); the operator application stays a direct launch.  Same
                        arithmetic as 0, fewer launches: for small systems, where launch cost
                        dominates.  0: direct launches */
  int32_t basis32;   /* MFS_MIXED with fp64_until = 0: 1 stores the Krylov basis in complex64
                        (half the memory and basis traffic; inner products, the Hessenberg matrix,
                        rotations and the solution update stay FP64).  0: complex128 basis */
  int32_t deflate;   /* MFS_MIXED: 1 keeps the first inner solve's Krylov space (its basis,
                        rotations and triangular factor stay in the basis workspace; each column
                        keeps its own) and runs every later correction solve on the operator
                        deflated by it (GCRO): the new Arnoldi vectors follow the longest kept
                        space in the same workspace, each step's Gram-Schmidt runs over both, and
                        one more FP32 operator application per correction adds the component in
                        the kept space.  Needs room for 64 new steps after the kept ones
                        (restart >= longest kept space + 65), else plain restarts.  Ignored for
                        MFS_FP64.  0: each correction solve starts afresh */
  int32_t block;     /* 1 with 2 <= R <= 64: block GMRES, one Krylov space shared by the R right-hand
                        sides (each step applies the operator to a block of R basis vectors and
                        extends the space by R; every column is the best combination of the whole
                        space).  restart then counts block steps: the basis takes
                        (restart+1) * R * N * 8 bytes with basis32 (16 otherwise) and the block
                        Hessenberg matrix R^2 restart (restart+3) / 2 * 16 bytes.  Orthogonalisation
                        is block classical Gram-Schmidt with two passes and shifted CholeskyQR3 of each
                        new block, inner products and the least-squares problem in FP64.  MFS_MIXED:
                        each cycle runs on the FP32 operator and is followed by the FP64 residual, as
                        above; MFS_FP64: restarted block GMRES with the FP64 operator.  Not combined
                        with fp64_until, use_graph or deflate.  0: one Krylov space per column */
} mfs_solve_opts;

typedef struct {
  int32_t n_matvec32;   /* FP32 operator applications (per right-hand side) */
  int32_t n_matvec64;   /* FP64 operator applications, including residual checks */
  int32_t n_refine;     /* refinement steps taken (MFS_MIXED) */
  int32_t n_restart;    /* GMRES restarts */
  double relres_max;    /* max over columns of the final FP64 relative residual */
  double t_total_s;     /* wall time of the call */
  int32_t n_reorth;     /* Arnoldi steps that took the second Gram-Schmidt pass (max over columns) */
} mfs_solve_info;

mfs_status mfs_solve(const mfs_scene* scene, const void* vhat_dev, int32_t R, const mfs_solve_opts* opts,
                     void* qhat_dev, mfs_solve_info* info, void* stream);

/* Device bytes a scene of this layout holds after mfs_solve with these options and R right-hand
 * sides, followed by an FP64 mfs_eval_field at n_targets points (0: none): its tables and its
 * grow-only workspaces (pair partial sums, padded and split charges, the Krylov basis and
 * coefficients of the per-column or the block solve, solver vectors), each as the block the
 * allocation cache takes for it, with the launch shapes the scene would use now (its process-wide
 * table, else the heuristic).  The split charges of the FP16 matrix-core pair sum are counted
 * wherever it may run, so this is an upper bound where its use depends on the geometry.  Not
 * counted: the caller's S matrices and vectors (vhat, qhat, targets, field), and blocks the cache
 * keeps for reuse.  For admission control by device memory.  Host only; no device is touched.
 *   dim, T, shape_of, n_shapes, k_of_shape: as for mfs_scene_create; rotations: 1 if the scene
 *   will carry rotations.  opts: prec, restart, block, basis32 and fp64_until are read.
 * Errors: MFS_ERR_ARG. */
mfs_status mfs_solve_footprint(int32_t dim, int64_t T, const int32_t* shape_of, int32_t n_shapes,
                               const int64_t* k_of_shape, int32_t rotations, int32_t R,
                               const mfs_solve_opts* opts, int64_t n_targets, size_t* bytes_out);

/* ------------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.
 *
 * mfs_apply_static computes the same operator as mfs_apply, y = q + S G_hat q, with the same
 * kernels, but keeps every intermediate (the pair sum's partial slices, and for the symmetric
 * kernel on bodies padded to whole tiles the padded copy of the charges) in a fixed array of
 * MFS_STATIC_SCRATCH_BYTES that the library holds on each device it runs on until the process ends.
 * The call allocates nothing: no hipMalloc, no hipFree, no allocating library routine, no scene
 * workspace.  The array's device address is looked up once per device, when the first scene is
 * created there (mfs_scene_create), so the scene passed in fixes the device.
 *   q_dev, y_dev  device [R][N]; complex128 (MFS_FP64) or complex64 (MFS_FP32); y != q.
 * Launch shape: the scene's, cut to what fits in the array (fewer source slices; the plain kernel
 * when the symmetric kernel's slices do not fit), so the last bits of FP32 results may differ from
 * mfs_apply's; the operator is the same.  Limit: one partial slice, R x N x 8 bytes (FP32) or
 * R x N x 16 bytes (FP64), must fit in the array; larger calls return MFS_ERR_ARG and enqueue nothing.
 * Every call on a device shares that device's array and overwrites it; no call reads what an
 * earlier call left there (each slice is written before it is read), so nothing needs clearing.
 * Calls that overlap on one device race on the array: serialise them (one stream, or events).
 * Asynchronous. */
#define MFS_STATIC_SCRATCH_BYTES (64ull << 20)
mfs_status mfs_apply_static(const mfs_scene* scene, const void* q_dev, void* y_dev, int32_t R, mfs_prec prec,
                            void* stream);

/* Scattered field u(x) = sum_j phi_kappa(x - x_hat_j) qhat_j at M targets (eq. out_skel), valid for
 * targets on or outside every body's proxy surface (Sec. 2.3, Sec. 4.1).  Asynchronous.
 *   qhat_dev     device [R][N] complex128 (MFS_FP64) or complex64 (MFS_FP32)
 *   targets_dev  device double[M][dim], absolute coordinates
 *   u_dev        device [R][M], complex128 (MFS_FP64) or complex64 (MFS_FP32) */
mfs_status mfs_eval_field(const mfs_scene* scene, const void* qhat_dev, int32_t R, const double* targets_dev,
                          int64_t M, void* u_dev, mfs_prec prec, void* stream);

/* ------------------------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).
 * While enabled, every pair-sum launch (G_hat and field evaluation) is bracketed by HIP events
 * recorded on the stream it runs on, and the algorithmic pair count of the launch is recorded.
 * ------------------------------------------------------------------------------------------ */
typedef enum { MFS_KERNEL_PAIR_F32 = 0, MFS_KERNEL_PAIR_F64 = 1 } mfs_kernel_kind;

/* Start (on != 0) or stop recording.  Starting clears earlier records.  Not thread-safe. */
mfs_status mfs_timing_enable(int32_t on);

/* Totals over the recorded launches of one kind: summed kernel time in milliseconds, number of
 * launches, and algorithmic pair evaluations (off-body pairs times right-hand sides).  Waits for
 * the recorded events.  Host outputs may be NULL. */
mfs_status mfs_timing_read(mfs_kernel_kind kind, double* total_ms, int64_t* launches, double* pairs);

/* ------------------------------------------------------------------------------------------
 * Full MFS sources and the field near the bodies (Sec. 4.6).
 *
 * The equivalent sources q_hat of body tau represent its scattered field only outside its proxy
 * surface Psi_tau.  Its own MFS sources (the points y_j of Sec. 3) are reconstructed as
 *     q_tau^mfs = A_tau^+ ( v_tau - U_tau (G_hat q_hat)_tau ),
 * v_tau being the Dirichlet data at the collocation points of Gamma_tau and U_tau the map from
 * values at the equivalent points to values at the collocation points (the one inside S).  Their
 * field sum_j phi(x - y_j) q_j^mfs is valid everywhere outside the source curve or surface, so the
 * scattered field can be evaluated up to and on the boundaries.  The calls below that take a
 * scene accept at most 65535 bodies.
 * ------------------------------------------------------------------------------------------ */
typedef struct mfs_recon mfs_recon;    /* per shape: pivoted QR of A, A^+ U, points, proxy radius */

/* Reconstruction factors of one shape, FP64 on the device: the column-pivoted Householder QR of
 * A = phi(x_i - y_j) (truncated at eps_ls like the solves inside mfs_build_S) and Y = A^+ U.
 *   desc        as for mfs_build_S (given equivalent points, or paper mode with eqpts = NULL)
 *   psi_radius  radius of the proxy surface about the body centre: a target x is inside Psi_tau
 *               when |x - c_tau| < psi_radius
 * Synchronous.  Errors: MFS_ERR_ARG, MFS_ERR_RANK, MFS_ERR_NOMEM, MFS_ERR_HIP. */
mfs_status mfs_recon_create(const mfs_shape_desc* desc, double psi_radius, mfs_recon** out, void* stream);

/* Free the factors.  Waits for the device (kernels on any stream may still read them). */
mfs_status mfs_recon_destroy(mfs_recon* recon);

/* Collocation points m, MFS sources n, equivalent points k, numerical rank of A.  Host outputs may
 * be NULL. */
mfs_status mfs_recon_size(const mfs_recon* recon, int64_t* m, int64_t* n, int64_t* k, int64_t* rank);

/* Totals over the scene's bodies: collocation points (sum m_tau) and MFS sources (sum n_tau), the
 * lengths of the per-body arrays below.  recon: host array [n_shapes] of factors, one per shape of
 * the scene, with the scene's k and kappa.  Synchronous on the first call with a new set. */
mfs_status mfs_near_sizes(const mfs_scene* scene, const mfs_recon* const* recon, int64_t* colloc_total,
                          int64_t* src_total);

/* v = -exp(i kappa d_r . x) at every body's collocation points, device complex128
 * [R][colloc_total], bodies in order (footnote to eq. BVP).  Asynchronous. */
mfs_status mfs_plane_wave_colloc(const mfs_scene* scene, const mfs_recon* const* recon, const double* dirs_host,
                                 int32_t R, void* v_dev, void* stream);

/* q^mfs of every body (Sec. 4.6), FP64.
 *   v_colloc_dev  device complex128 [R][colloc_total]: Dirichlet data at the collocation points
 *   qhat_dev      device complex128 [R][N]: solved equivalent sources
 *   qmfs_dev      device complex128 [R][src_total] output, bodies in order
 * Asynchronous. */
mfs_status mfs_reconstruct(const mfs_scene* scene, const mfs_recon* const* recon, const void* v_colloc_dev,
                           const void* qhat_dev, int32_t R, void* qmfs_dev, void* stream);

/* Scattered field at M targets anywhere outside the MFS source curves or surfaces, FP64: body tau
 * contributes through its MFS sources where |x - c_tau| < psi_radius and through its equivalent
 * points elsewhere.  A target on an MFS source gives an infinite value.
 *   targets_dev  device double [M][dim]; u_dev device complex128 [R][M]
 * Asynchronous. */
mfs_status mfs_eval_field_near(const mfs_scene* scene, const mfs_recon* const* recon, const void* qhat_dev,
                               const void* qmfs_dev, int32_t R, const double* targets_dev, int64_t M, void* u_dev,
                               void* stream);

/* ------------------------------------------------------------------------------------------
 * Device allocation cache.  Scene tables, pair partial sums and Krylov bases are drawn from a
 * process-wide cache of device blocks: a freed block stays on its device and is reused by the next
 * request whose size it fits (at most twice the size asked for), with the new owner's stream
 * ordered after the previous owner's last use.  A request loop therefore keeps its Krylov bases
 * resident instead of calling hipMalloc and hipFree (which waits for the device) per request.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int64_t hits;          /* allocations served from the cache */
  int64_t misses;        /* allocations that called hipMalloc */
  int64_t cached_bytes;  /* bytes held in the cache, free for reuse */
  int64_t live_bytes;    /* bytes handed out and not yet returned */
  int64_t limit_bytes;   /* cap on cached_bytes; blocks beyond it are freed when returned */
} mfs_pool_stats;

/* Counters of the cache (all devices).  Host output. */
mfs_status mfs_pool_query(mfs_pool_stats* out);

/* Set the cap on cached bytes (>= 0); cached blocks are released if the cache exceeds it. */
mfs_status mfs_pool_set_limit(int64_t max_cached_bytes);

/* Budget for the partial sums of the symmetric pair kernel, process-wide (runtime only).  The
 * kernel writes its source-side sums as partial slices of N entries per right-hand side: one per
 * group distance where each wave stores its own (the fastest form), or about 8 times fewer where
 * the 8 waves of a block share each staged source tile and store its sums once (a barrier per
 * tile: a few percent more time, and 4 to 8 times fewer HBM writes).  The shared form runs when
 * the one-wave form's slices for the call's right-hand sides would exceed `bytes`; bytes <= 0
 * restores the default, 4 GiB.  *previous (may be null) receives the budget in force before the
 * call.  Takes effect for pair sums launched afterwards; a solve's footprint follows it, so set it
 * before mfs_solve_footprint and the solves it sizes.  Never fails. */
mfs_status mfs_sym_slice_budget(int64_t bytes, int64_t* previous);

/* Release every cached block to the device (waits for each block's last use).  Blocks held by live
 * scenes are not affected. */
mfs_status mfs_pool_trim(void);

/* ------------------------------------------------------------------------------------------
 * Launch-shape autotuner.  Not part of the method: it picks how the off-body pair sum of the
 * operator (eq. Gmtx-entries, eq. mbody2) is spread over the device, never what it computes.
 *
 * The pair sum splits the sources seen by every block of targets into `nchunks` slices (more
 * slices: more blocks in flight on a small system, but more partial sums for the S product to
 * read back), and on the VALU kernel each thread carries `rhs_per_thread` right-hand sides (1, 2
 * or 4; the matrix-core kernel, for 8 or more right-hand sides, has no such knob).  With 1 to 32
 * right-hand sides in FP32, a symmetric kernel can run instead: G_hat is symmetric, so it
 * evaluates phi once per unordered pair of points and adds it into both sums.  It works on tiles of
 * 64 points of one body; bodies whose point count is not a multiple of 64 are padded with
 * zero-charge points where that adds at most 40% to the pair count.  There `nchunks` counts the
 * chunks of group distances per target group, and the kernel leaves about N / 512 further partial
 * slices per right-hand side (at most 8 GiB of them, else another kernel runs).  A scene uses, in
 * this order: its own tuned shape for (precision, R); the process-wide table, keyed by
 * (dim, kernel, R, floor(log2 N)); the heuristic (the symmetric kernel where it applies and
 * R <= 24).  Slices are summed in a fixed order, so a given shape gives reproducible results;
 * another shape may change the last bits of the sums.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t nchunks;         /* chosen source slices (distance chunks if symmetric) */
  int32_t rhs_per_thread;  /* chosen right-hand sides per thread (VALU kernels), 0 otherwise */
  double ms;               /* time of one operator application with the chosen shape */
  double ms_heuristic;     /* the same with the untuned shape */
  int32_t n_tried;         /* shapes timed */
  int32_t uses_mfma;       /* 1 when the matrix-core kernel won (R >= 8) */
  int32_t symmetric;       /* 1 when the symmetric kernel won */
  double ms_plain;         /* time with the plain kernel's heuristic shape (-1 if not timed) */
} mfs_tune_result;

/* Time the operator y = q + S G_hat q (mfs_apply for MFS_FP64 / MFS_FP32, the complex128-vector
 * form with an FP32 pair sum for MFS_MIXED) on this scene with R right-hand sides for a set of
 * launch shapes around the heuristic, `reps` applications each after one warm-up, and keep the
 * fastest: in the scene and in the process-wide table.  Uses synthetic charges in scratch device
 * memory; the caller's data is not touched.  Another shape replaces the untuned one only when it
 * is at least 2% faster, so that timing noise does not move the choice between runs.
 * Synchronous.  Pair-sum launches made while kernel timing is enabled are recorded like any
 * other.  out may be NULL. */
mfs_status mfs_autotune(mfs_scene* scene, int32_t R, mfs_prec prec, int32_t reps, mfs_tune_result* out,
                        void* stream);

/* The launch shape the scene will use for (R, prec): nchunks, rhs_per_thread (0 for the FP64 and
 * matrix-core kernels), symmetric (1 if the symmetric kernel runs) and where the
 * shape comes from (2 = the scene's own, 1 = the process-wide table, 0 = the heuristic).  Host
 * outputs may be NULL. */
mfs_status mfs_tune_get(const mfs_scene* scene, int32_t R, mfs_prec prec, int32_t* nchunks,
                        int32_t* rhs_per_thread, int32_t* symmetric, int32_t* source);

/* Which pair kernel the pair sum G_hat q runs for (R, prec) on this scene, as the launch shape
 * stands now (mfs_tune_set and mfs_autotune may change it). */
typedef enum {
  MFS_PAIR_F64 = 0,         /* FP64, plain */
  MFS_PAIR_F32 = 1,         /* FP32 vector units, body-centre phase split */
  MFS_PAIR_F32_SYM = 2,     /* FP32 vector units, phi once per unordered pair */
  MFS_PAIR_F32_SYM16 = 3,   /* the same on 16-point sub-blocks (3D, bodies of multiples of 16) */
  MFS_PAIR_MC_F32 = 4,      /* matrix cores, FP32 products (R >= 8) */
  MFS_PAIR_MC_F16X3 = 5,    /* matrix cores, FP16 products of split operands (R >= 8) */
  MFS_PAIR_MC_F64 = 6,      /* FP64 on the FP64 matrix cores (R >= 8) */
  MFS_PAIR_F32_SYM_SHARED = 7,   /* MFS_PAIR_F32_SYM with 8 waves per block sharing each source
                                    tile (the slices of the one-wave form would pass the budget of
                                    mfs_sym_slice_budget) */
  MFS_PAIR_F32_SYM16_SHARED = 8  /* the same for MFS_PAIR_F32_SYM16 */
} mfs_pair_kernel_kind;
mfs_status mfs_pair_kernel(const mfs_scene* scene, int32_t R, mfs_prec prec, int32_t* kind);

/* Matrix-core form of the FP32 pair sum with 8 or more right-hand sides (bodies of multiples of 16
 * points).  enable = 1 (the default where the scene allows it): FP16 products of split operands,
 * each FP32 operand carried as a high and a low FP16 part, three products per real product,
 * accumulated in FP32 (~2^-21 relative per product; Ootomo and Yokota 2022); it needs |phi| bounded
 * over the scene's off-body pairs (always in 2D; in 3D from the closest pair of body centres less
 * twice the largest body radius) and MFS_ERR_ARG is returned when no bound is known.  enable = 0:
 * FP32 products.  Host only. */
mfs_status mfs_scene_set_split_fp16(mfs_scene* scene, int32_t enable);

/* Set the scene's own shape for (R, prec): 1 <= nchunks <= 1024; rhs_per_thread 0 = by R, or 1, 2,
 * 4; symmetric 1 = the symmetric kernel where it applies (up to 32 right-hand sides), -1 = as the
 * heuristic (up to 24), 0 = never.  nchunks = 0 removes the scene's entry. */
mfs_status mfs_tune_set(mfs_scene* scene, int32_t R, mfs_prec prec, int32_t nchunks, int32_t rhs_per_thread,
                        int32_t symmetric);

/* The process-wide table as a text file: a header line, then one entry per line
 * ("dim kernel R log2N nchunks rhs_per_thread symmetric").  Loading merges into the table and is
 * all or nothing: a malformed file is rejected (MFS_ERR_ARG) and leaves the table unchanged.  Host
 * only; no device is touched. */
mfs_status mfs_tune_save(const char* path);
mfs_status mfs_tune_load(const char* path);
mfs_status mfs_tune_clear(void);
mfs_status mfs_tune_table_size(int64_t* entries);

#ifdef __cplusplus
}
#endif

#endif /* MFS_H_ */
