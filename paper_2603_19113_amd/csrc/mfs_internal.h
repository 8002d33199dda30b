// Internal declarations shared by the translation units of libmfs.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mfs.h"

namespace mfs {

// ------------------------------------------------------------------ errors ---
void set_error(const std::string& msg);
mfs_status fail(mfs_status code, const std::string& msg);

#define MFS_HIP_TRY(expr)                                                                   \
  do {                                                                                      \
    hipError_t e__ = (expr);                                                                \
    if (e__ != hipSuccess)                                                                  \
      return ::mfs::fail(MFS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

// --------------------------------------------------------------- complex ----
template <typename T>
struct Cplx {
  T re, im;
};
using c64 = Cplx<float>;
using c128 = Cplx<double>;

// ------------------------------------------------------------- scene view ---
// Device-side description of the packed scene, passed by value to kernels.
struct SceneDev {
  int32_t dim;
  int64_t N;
  int64_t T;
  double kappa;
  double origin[3];       // FP32 coordinates are relative to this point
  const double* x64[3];   // absolute FP64 coordinates, SoA
  const float* x32[3];    // FP32 coordinates relative to origin, SoA
  const float* l32[3];    // FP32 body-local offsets x_hat - c_body (the shape template), SoA
  const float* lsq32;     // [N] |l|^2 of the FP32 offsets
  const double* centres;  // [T][dim] body centres, FP64
  const int32_t* body_of; // [N]
  const int64_t* body_ptr;// [T+1]
  const int32_t* shape_of;// [T]
  const int64_t* k_of_shape;      // [n_shapes]
  const void* const* S64;         // [n_shapes] device pointers (complex128, col-major)
  const void* const* S32;         // [n_shapes] device pointers (complex64) or null
  double offbody_pairs;           // N^2 - sum_tau k_tau^2
  bool all_k_mult16;              // every shape has a multiple of 16 points (matrix-core path)
  bool all_k_mult64;              // every shape has a multiple of 64 points (symmetric pair kernel)
  bool sym16;                     // 3D, every shape a multiple of 16 points but not all of 64: the
                                  // symmetric kernel works on 16-point sub-blocks, no padded layout
  // Padded layout for the symmetric kernel when some shape's point count is not a multiple of 64:
  // body b occupies [pad_ptr[b], pad_ptr[b+1]) with its points first and zero-charge fillers at its
  // centre after them.  Npad = N and null tables when every count is a multiple of 64 (or no
  // padding was made).
  int64_t Npad;
  const int64_t* pad_ptr;         // [T+1]
  const int32_t* body_of_pad;     // [Npad]
  const float* l32p[3];           // [Npad] body-local offsets, 0 for fillers
  const float* lsqp;              // [Npad]
  double rho_max;                 // largest |x_hat - c_body| over all shapes
  int phi16_shift;                // sA with 2^sA |phi| < 2^13 for every off-body pair (the FP16
                                  // matrix-core kernel), or -1 where no such bound is known
  const double* rot;              // [T][dim][dim] body orientations (row-major), or null: identity
};

// ------------------------------------------------------- kernel launchers ---
// Pair sums (pair_kernels.hip).  Targets are either the scene's own points (G_hat, with
// same-body exclusion) or arbitrary FP64 targets (field evaluation, no exclusion).  Results
// are per-source-chunk partial sums, partial[c][r][M], which the consumer adds in chunk order.
int pair_chunks_for(int64_t n_sources, int64_t n_targets, int tpt);
bool ghat_uses_mfma(const SceneDev& s, int R);

// rt: right-hand sides per thread of the VALU kernel (1, 2 or 4; anything else picks by R);
// ignored where the matrix-core kernel runs.
int ghat_default_rt(int R);
// Symmetric pair kernels (1 to kSymMaxRhs right-hand sides): groups of 256 points (G0 of them,
// padded with empty groups to G, a multiple of the W waves of a block), distances 0..Dmax, block
// offsets 0..HH-1 in nchunks_d chunks of dpc each; they write `slices` partial slices (nchunks_d
// target-side, HH / W source-side).  nchunks_d <= 0 picks the heuristic.  W = 1 (each wave stores
// its own source-side sums: the fastest) unless those slices would pass the slice budget, then
// kSymW (the block's waves share each source tile and store its sums once: ~kSymW times fewer
// slices and HBM writes, at a few percent more time for the barrier per tile).
constexpr int kSymMaxRhs = 32;         // the symmetric kernel may run up to this many right-hand sides
constexpr int kSymDefaultMaxRhs = 24;  // and does by default up to this many
constexpr int kSymW = 8;               // waves per block where the source tiles are shared
constexpr int64_t kSymSliceBudget = 4ll << 30;  // default slice budget (bytes)
struct SymPlan {
  int64_t G;
  int W, Dmax, HH, dpc, nchunks_d, slices;
  bool even;
};
SymPlan sym_plan(int64_t N, int nchunks_d, int W);
int sym_block_waves(int64_t NP, int R);   // W for R right-hand sides on NP points
int64_t sym_slice_budget(int64_t bytes);  // set the budget (<= 0: the default); returns the previous
bool ghat_sym_possible(const SceneDev& s, int R);
hipError_t launch_ghat_f32_sym(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks_d, int rt,
                               hipStream_t st);
// The symmetric kernel's view of a scene: the scene itself, or its padded layout (N = Npad).
SceneDev sym_view(const SceneDev& s);
// True when the symmetric kernel runs on the padded layout (bodies padded to whole 64-point tiles).
bool sym_padded(const SceneDev& s);
// t[r][i] = sum_c partial[c][r][pad(i)] for the padded layout.
hipError_t launch_reduce_partials_padded(const SceneDev& s, const c64* partial, int nchunks, int R, c64* out,
                                         hipStream_t st);
// split: device workspace of ghat_split_bytes(s, R) bytes for the FP16 matrix-core kernel (the
// split charges), or null: then the FP32 matrix-core kernel runs where the matrix cores are used.
hipError_t launch_ghat_f32(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks,
                           hipStream_t st, int rt = 0, void* split = nullptr);
// The FP16 matrix-core kernel (split operands) applies: many right-hand sides, bodies of multiples of
// 16 points, and a scale 2^sA with 2^sA |phi| < 2^13 known for the scene (phi16_shift >= 0).
bool ghat_uses_mfma16(const SceneDev& s, int R);
size_t ghat_split_bytes(const SceneDev& s, int R);
// The matrix-core pair sum (mc_kernels.hip): the split FP16 form where split is given and the scene
// allows it, else the FP32 form.
hipError_t launch_ghat_mc(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks, void* split,
                          hipStream_t st);
// The FP64 pair sum on the FP64 matrix cores (mc_kernels.hip), where ghat_uses_mfma holds.
hipError_t launch_ghat_mc64(const SceneDev& s, const c128* q, int R, c128* partial, int nchunks, hipStream_t st);
// FP64 pair sum: the matrix cores from 8 right-hand sides, the symmetric kernel (its own plan, four
// waves per block sharing each source tile) for one unless allow_sym is false, else the plain kernel in nchunks slices.
// ghat_f64_slices gives the number of partial slices it writes.
bool ghat_f64_sym(const SceneDev& s, int R);
int ghat_f64_slices(const SceneDev& s, int R, int nchunks);
hipError_t launch_ghat_f64(const SceneDev& s, const c128* q, int R, c128* partial, int nchunks,
                           hipStream_t st, bool allow_sym = true);
hipError_t launch_eval_f32(const SceneDev& s, const c64* q, int R, const double* targets, int64_t M,
                           c64* partial, int nchunks, hipStream_t st);
hipError_t launch_eval_f64(const SceneDev& s, const c128* q, int R, const double* targets, int64_t M,
                           c128* partial, int nchunks, hipStream_t st);

// Sum partial[c][r][M] over c into out[r][M] (field evaluation, plain G_hat output).
hipError_t launch_reduce_partials_f32(const c64* partial, int nchunks, int64_t M, int R, c64* out,
                                      hipStream_t st);
hipError_t launch_reduce_partials_f64(const c128* partial, int nchunks, int64_t M, int R, c128* out,
                                      hipStream_t st);

// Block-diagonal S (sapply.hip): y = beta q + S t, t = sum over chunks of partial.
// TQ is the type of q and y; the S factors and partials are in the operator precision.
// The S products read the pair sums at partial[c][r][pptr[body] + j] (rows of NP entries);
// pptr = null means the packed layout (body_ptr, N).
hipError_t launch_sapply_f64(const SceneDev& s, const c128* partial, int nchunks, const c128* q, double beta,
                             c128* y, int R, int kmax, hipStream_t st);
hipError_t launch_sapply_f32(const SceneDev& s, const c64* partial, int nchunks, const c64* q, float beta,
                             c64* y, int R, int kmax, hipStream_t st, const int64_t* pptr = nullptr, int64_t NP = 0);
hipError_t launch_sapply_mixed(const SceneDev& s, const c64* partial, int nchunks, const c128* q, double beta,
                               c128* y, int R, int kmax, hipStream_t st, const int64_t* pptr = nullptr,
                               int64_t NP = 0);
// Padded layout: fill the padded offsets (pad_scene) and gather charges into it (zero for fillers).
hipError_t launch_pad_scene(const SceneDev& s, float* l32p, float* lsqp, hipStream_t st);
hipError_t launch_gather_pad(const SceneDev& s, const c64* q, int R, c64* qp, hipStream_t st);

// Elementwise helpers (sapply.hip).
hipError_t launch_to_c64(const c128* in, c64* out, int64_t n, hipStream_t st);
hipError_t launch_plane_wave(const SceneDev& s, const double* dirs_dev, int R, c128* vhat, hipStream_t st);
hipError_t launch_pack_scene(int dim, int64_t T, const int32_t* shape_of, const double* centres,
                             const double* rot, const int64_t* tmpl_ptr, const double* tmpl_pts, const int64_t* body_ptr,
                             const double* origin, double* x64_soa, float* x32_soa, float* l32_soa,
                             float* lsq, int32_t* body_of, int64_t N, hipStream_t st);

// Krylov kernels (krylov.hip).  One Arnoldi/GMRES state per right-hand side; vectors [R][N].
struct KrylovDev {
  int64_t N;
  int R;
  int m;              // restart length
  void* V;            // [(m+1)][R][N], complex128, or complex64 when v32
  bool v32;           // basis stored in single precision (inner solves with the FP32 operator)
  c128* H;            // [R][m][m+1]: column j of rhs r at H + (r*m + j)*(m+1)
  c128* cs;           // [R][m]
  c128* sn;           // [R][m]
  c128* g;            // [R][m+1]
  c128* hcol;         // [R][m+1] first Gram-Schmidt coefficients
  c128* h2;           // [R][m+1] second-pass coefficients
  c128* y;            // [R][m]   least-squares coefficients
  double* beta;       // [R] norms of the cycle's starting residuals
  double* bnorm;      // [R] norms the relative estimate refers to
  double* res;        // [R] |g_{j+1}| / bnorm
  double* hnorm;      // [R] ||w|| of the current step
  int32_t* active;    // [R] 1 while the column iterates in this cycle
  int32_t* jlen;      // [R] Arnoldi steps taken by the column in this cycle
  double* wn;         // [R] ||w|| before orthogonalisation
  int32_t* reorth;    // [R] 1 if the current step takes the second Gram-Schmidt pass
  int32_t* n_reorth;  // [R] number of second passes taken (diagnostics)
  double reorth_eta;  // second pass when ||w'|| < eta ||w||
  double* ratio_log;  // optional [R][2m] log of ||w'|| / ||w|| per step (diagnostics), or null
  double* part;       // [R][m+1][nblk][2] partial sums
  int nblk;
  // Graph replay: the step index and the cycle's tolerance live on the device (set by the cycle
  // start, advanced by each step), so one captured step serves every step of its bucket.  Null
  // for eager launches, which pass the step as an argument.
  int32_t* jdev;
  double* tol_dev;
  double tol;         // tolerance written to tol_dev at the cycle start
  // Deflated correction solves (GCRO): the process starts at basis slot joff, after the vectors
  // of an earlier process that are kept (kold[r] + 1 <= joff of them for column r; the slots
  // between are vectors of steps after that column had converged); its Hessenberg column,
  // rotation, g and y entries sit at index joff + j of their arrays.  Each step's Gram-Schmidt
  // runs over all joff + j + 1 vectors and replaces the coefficients a on the kept vectors by
  // a - qdef (qdef^H a), which removes only the part along C = V_old Q (Q^H qdef = 0, the columns
  // of Q spanning the range of the kept process's Hessenberg matrix), and zeroes those on the
  // slots between.  Eager launches only (jdev null).  joff = 0 and qdef null otherwise.
  int joff;
  const c128* qdef;
  const int32_t* kold;  // [R] steps of the kept process per column
};

// Steps per captured graph: the graph of bucket b serves steps b*kStepBucket ... (b+1)*kStepBucket-1.
constexpr int kStepBucket = 64;

int krylov_nblk(int64_t N);
int krylov_part_blocks(int64_t N);  // blocks per vector of the widest inner-product launch
hipError_t launch_norms(const c128* v, int64_t N, int R, double* part, int nblk, double* out_norm,
                        hipStream_t st);
hipError_t launch_start_cycle(KrylovDev k, const c128* r0, hipStream_t st);
hipError_t launch_arnoldi_orth(KrylovDev k, int j, c128* w, hipStream_t st);
hipError_t launch_arnoldi_finish(KrylovDev k, int j, c128* w, double tol, hipStream_t st);
hipError_t launch_gmres_update_x(KrylovDev k, c128* x, hipStream_t st);
// Deflation helpers (one right-hand side):
//   out = V_{0..count-1}^H w;  w -= V_{0..count-1} h;  x += sum_{i<jlen} y_{joff+i} V_{joff+i}
//   q = G^H e_kold and e = G e (rotations 0..kold[r]-1 of the process that built the kept vectors)
//   h -= q (q^H h) over the first kold[r] + 1 entries, zero on the rest of the first o (all o
//   where keep[r] == 0; keep may be null)
hipError_t launch_basis_dots(KrylovDev k, const c128* w, int count, c128* out, hipStream_t st);
hipError_t launch_basis_axpy(KrylovDev k, const c128* h, int count, c128* w, hipStream_t st);
hipError_t launch_update_from_y(KrylovDev k, c128* x, hipStream_t st);
hipError_t launch_givens_last_column(KrylovDev k, const int32_t* kold, c128* q, hipStream_t st);
hipError_t launch_givens_apply(KrylovDev k, const int32_t* kold, c128* e, hipStream_t st);
hipError_t launch_deflate_coeffs(const c128* q, int o, const int32_t* kold, c128* h, int R, int ld,
                                 const int32_t* keep, hipStream_t st);
hipError_t launch_axpby(const c128* a, const c128* b, c128* out, double alpha, double beta, int64_t n,
                        hipStream_t st);

// Block GMRES (bkrylov.hip): one Krylov space for all R <= 64 right-hand sides.  Matrices are
// column-major complex128 unless a32 (then A is complex64); see bkrylov.hip for the layouts.
//   bdots:     part[s][c][k] = sum over row slice s of conj(A[k][n]) B[c][n], k < K, c < R
//   breduce:   out[k + c ldo] (= or +=) sum_s part[s][c][k]; copy gets the sum too when not null
//   bgemm_nk:  out[c ldo + n] = beta in[c ldi + n] + alpha sum_k A[k lda + n] C[k + c ldc], n < M
//   chol:      one shifted CholeskyQR step on an R x R Gram matrix (F, Finv, Rtot = F Rtot)
//   bhess_*:   Householder QR of the block Hessenberg matrix (reflector rho on rows rho..rho+R)
constexpr int64_t kBdotsPartMax = 131072;  // bound on nsplit * K of one bdots launch
int bdots_splits(int64_t N, int K);
// fp32: the FP32 matrix-core form (operands rounded to FP32, each 32-long slab of the reduction
// summed in FP32 and added into FP64), for the Gram-Schmidt passes of the mixed solve
hipError_t launch_bdots(const void* A, bool a32, int64_t lda, int K, const c128* B, int64_t ldb, int R, int64_t N,
                        c128* part, int nsplit, hipStream_t st, bool fp32 = false);
// FP32 forms with complex64 right operands (converted once per pass: half the bytes re-read per tile)
hipError_t launch_bdots32_b64(const c64* A, int64_t lda, int K, const c64* B, int64_t ldb, int R, int64_t N, c128* part,
                              int nsplit, hipStream_t st);
hipError_t launch_bgemm32_c64(const c64* A, int64_t lda, int64_t M, int K, const c64* C, int64_t ldc, int R,
                              double alpha, double beta, const c128* in, int64_t ldi, c128* out, int64_t ldo,
                              hipStream_t st);
hipError_t launch_to_c64_2d(const c128* in, int64_t ldi, int64_t rows, int cols, c64* out, int64_t ldo, hipStream_t st);
hipError_t launch_breduce(const c128* part, int nsplit, int K, int R, c128* out, int64_t ldo, bool accumulate,
                          c128* copy, int64_t ldc, hipStream_t st);
hipError_t launch_bgemm_nk(const void* A, bool a32, int64_t lda, int64_t M, int K, const c128* C, int64_t ldc, int R,
                           double alpha, double beta, const c128* in, int64_t ldi, c128* out, int64_t ldo,
                           hipStream_t st, bool fp32 = false);
hipError_t launch_chol(const c128* G, int R, bool scale, double shift, bool first, double dep_tol, c128* F, c128* Finv,
                       c128* Rtot, int32_t* dep, int32_t* flag, hipStream_t st);
hipError_t launch_fill_random(c128* x, int64_t N, uint64_t seed, hipStream_t st);
hipError_t launch_bhess_apply(const c128* refl, int R, int64_t rho0, int64_t rho1, c128* X, int64_t ldx, int ncols,
                              hipStream_t st);
hipError_t launch_bhess_apply_rev(const c128* refl, int R, int64_t rho0, int64_t rho1, c128* X, int64_t ldx,
                                  int ncols, hipStream_t st);
hipError_t launch_bhess_newqr(c128* refl, int R, int64_t jR, c128* X, int64_t ldx, hipStream_t st);
hipError_t launch_bres(const c128* g, int64_t ldg, int64_t row0, int R, const double* bnorm, double* res,
                       hipStream_t st);
hipError_t launch_btrsm_diag(const c128* U, int64_t ldu, const c128* g, int64_t ldg, c128* Y, int64_t ldy, int R,
                             hipStream_t st);
hipError_t launch_fill_zero_columns(c128* X, int64_t N, int R, const double* bnorm, hipStream_t st);
hipError_t launch_mask_zero_columns(c128* M, int64_t ldm, int rows, int R, const double* bnorm, hipStream_t st);
hipError_t launch_add_identity(c128* X, int64_t ldx, int64_t row0, int R, hipStream_t st);
hipError_t launch_copy2d(const c128* in, int64_t ldi, int64_t rows, int cols, c128* out, int64_t ldo, bool accumulate,
                         hipStream_t st);

// Kernel timing (mfs_api.hip): bracket a launch with events when recording is on.
struct TimedLaunch {
  TimedLaunch(int kind, double pairs, hipStream_t st);
  ~TimedLaunch();
  int kind;
  double pairs;
  hipStream_t st;
  void* ev0;
  void* ev1;
};

// Caching allocators (pool.hip).  pool_alloc returns a block of at least `bytes` (its size in *got);
// when the block is reused, work on `st` is ordered after its previous owner (the host waits when st
// is null).  pool_free hands a block back after the work enqueued on `last`.
void* pool_alloc(size_t bytes, hipStream_t st, size_t* got, hipError_t* err);
void pool_free(void* p, size_t bytes, hipStream_t last);
// The block size pool_alloc takes from HIP for a fresh request of `bytes`.
size_t pool_block_size(size_t bytes);
void* pinned_alloc(size_t bytes, size_t* got, hipError_t* err);
void pinned_free(void* p, size_t bytes);
void pool_query(int64_t* hits, int64_t* misses, int64_t* cached, int64_t* live, int64_t* limit);
void pool_trim();
void pool_set_limit(size_t bytes);
hipStream_t private_stream(hipError_t* err);

// Launch shapes of the pair sum (tune.hip).  nchunks: source slices per target block (distance
// chunks for the symmetric kernel); rt: right-hand sides per thread of the VALU kernel (0 = chosen
// by R); sym: the symmetric one-right-hand-side kernel where the scene allows it unless 0 (-1 = unset,
// as the heuristic: symmetric where possible).  The process-wide table is keyed by
// (dim, kernel variant, R, floor(log2 N)) and filled by the autotuner or a loaded file.
struct LaunchShape {
  int nchunks = 0;
  int rt = 0;
  int sym = -1;
};
enum TuneVariant { kTunePairF64 = 0, kTunePairF32 = 1, kTunePairMfma = 2 };
constexpr int kTuneMaxChunks = 1024;
bool tune_lookup(int dim, int variant, int R, int64_t N, LaunchShape* out);
void tune_store(int dim, int variant, int R, int64_t N, LaunchShape v);
void tune_clear();
int64_t tune_size();
bool tune_save(const char* path, std::string* err);
bool tune_load(const char* path, std::string* err);

// Reconstruction factors of one shape (lsq.hip): the pivoted QR of A (reflectors below the
// diagonal, R above it with its diagonal in alpha), Y = A^+ U, and the collocation points and MFS
// sources of the shape (body frame, [count][dim]); all in one device block from the pool.
struct ReconFactors {
  void* block;
  size_t block_bytes;
  c128* QA;      // m x n, ld m
  c128* alpha;   // [n]
  double* tau;   // [n]
  int* perm;     // [n]
  c128* Y;       // n x k, ld n
  double* colloc;
  double* src;
  int dim, m, n, k, rank;
  double kappa;
};
mfs_status build_recon_impl(const mfs_shape_desc* d, ReconFactors* out, hipStream_t st);
// Columns of a batched solve that live inside [R][total] arrays: column c is body bodies[c % nb]
// and right-hand side c / nb; its input starts at (c / nb) * ld_in + ptr_in[body] and its output
// at (c / nb) * ld_out + ptr_out[body].  bodies == null: plain column-major strides.
struct ColMap {
  const int32_t* bodies = nullptr;
  int nb = 0;
  const int64_t* ptr_in = nullptr;
  int64_t ld_in = 0;
  const int64_t* ptr_out = nullptr;
  int64_t ld_out = 0;
  __device__ int64_t in_offset(int c) const { return (int64_t)(c / nb) * ld_in + ptr_in[bodies[c % nb]]; }
  __device__ int64_t out_offset(int c) const { return (int64_t)(c / nb) * ld_out + ptr_out[bodies[c % nb]]; }
};
hipError_t launch_qr_reflect(const c128* QA, int rows, int ld, const double* tau, int rank, c128* rhs, int ldr,
                             int ncols, const ColMap& cm, hipStream_t st);
hipError_t launch_backsub(const c128* QA, int ld, const c128* alpha, int rank, c128* rhs, int ldr, const int* perm,
                          int cols_out, c128* X, int ldx, int ncols, const ColMap& cm, hipStream_t st);

// Near-field kernels (recon.hip).
struct NearTables {        // device tables, per shape s and per body b
  const double* const* colloc_of_shape;  // [n_shapes] -> [m_s][dim]
  const double* const* src_of_shape;     // [n_shapes] -> [n_s][dim]
  const c128* const* Y_of_shape;         // [n_shapes] -> n_s x k_s
  const int32_t* m_of_shape;
  const int32_t* n_of_shape;
  const double* psi2_of_shape;           // squared proxy radius
  const int64_t* cptr;                   // [T+1] collocation offsets
  const int64_t* sptr;                   // [T+1] MFS source offsets
  int64_t Mtot, Ntot;
  int mmax, nmax, kmax;
};
hipError_t launch_plane_wave_colloc(const SceneDev& s, const NearTables& t, const double* dirs, int R, c128* v,
                                    hipStream_t st);
hipError_t launch_recon_combine(const SceneDev& s, const NearTables& t, const c128* what, int R, c128* qmfs,
                                hipStream_t st);
hipError_t launch_eval_near(const SceneDev& s, const NearTables& t, const c128* qhat, const c128* qmfs, int R,
                            const double* targets, int64_t M, c128* partial, int nchunks, hipStream_t st);
int near_chunks_for(int64_t T, int64_t M);

// Least squares for S (lsq.hip).
mfs_status build_S_impl(const mfs_shape_desc* d, void* S64, void* S32, int64_t* k_out, int64_t* skel,
                        double* diag, hipStream_t st);

}  // namespace mfs
