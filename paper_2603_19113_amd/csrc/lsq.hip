// FP64 construction of the scattering matrix S of one shape (Sec. 4 of the paper) on the GPU.
//
// All matrices are complex128, column-major.  Least-squares problems M X = RHS are solved with
// Householder QR with column pivoting (Businger-Golub), applied to the right-hand sides as it
// goes, stopped when the largest remaining column norm falls to eps * |R_11| (the paper asks for
// a backward-stable truncated solve, Sec. 2.3 and Sec. 3.1), followed by back substitution on the
// leading r x r triangle (basic solution).  Each pivot step is two launches: one block picks the
// pivot, swaps it in and forms the reflector; then one block per remaining column (matrix and
// right-hand sides) applies the reflector and recomputes that column's trailing norm exactly
// (no norm downdating, so no cancellation safeguard is needed).
//
// Given equivalent points x_hat:  X = B_hat^+ [D | B],  Y = A^+ (X_B)^T,  S = X_D Y.
// Paper mode:  CPQR of B gives the skeleton I and R11^{-1} R12, hence Z* (eq. B_fac); U = Z*^T;
//              C = B^+ D; S = Z* C (A^+ U) (eq. scattering-matrix).
#include <cmath>
#include <string>
#include <vector>

#include "mfs_internal.h"
#include "phi.h"

namespace mfs {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ c128 cmul(c128 a, c128 b) { return c128{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 cconjmul(c128 a, c128 b) {  // conj(a) * b
  return c128{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// out(i, j) = phi(tg_i - src_j)
__global__ void assemble_kernel(int dim, double kappa, const double* __restrict__ tg, int rows,
                                const double* __restrict__ src, int cols, c128* __restrict__ out, int ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= rows) return;
  double r2 = 0.0;
  for (int d = 0; d < dim; ++d) {
    const double t = tg[(int64_t)i * dim + d] - src[(int64_t)j * dim + d];
    r2 += t * t;
  }
  const double r = sqrt(r2);
  double pr, pi;
  if (dim == 2) phi2d_f64(r, kappa, pr, pi);
  else phi3d_f64(r, kappa, pr, pi);
  out[(int64_t)j * ld + i] = c128{pr, pi};
}

struct QR {
  c128* M;
  int rows, cols, ld;
  c128* rhs;
  int nrhs, ldr;
  double* cnorm;  // [cols] squared norms of the rows >= step of each column
  int* perm;      // [cols]
  c128* alpha;    // [cols] diagonal of R
  double* tau;    // [cols] reflector scalars
  double* scal;   // [0] |R_11|, [1] rank so far, [2] stop flag
};

__global__ void qr_init_kernel(QR q) {
  __shared__ double red[kT / 64];
  const int j = blockIdx.x;
  const c128* col = q.M + (int64_t)j * q.ld;
  double s = 0.0;
  for (int i = threadIdx.x; i < q.rows; i += blockDim.x) s += col[i].re * col[i].re + col[i].im * col[i].im;
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    q.cnorm[j] = s;
    q.perm[j] = j;
    if (j == 0) {
      q.scal[0] = 0.0;
      q.scal[1] = 0.0;
      q.scal[2] = 0.0;
    }
  }
}

// Pivot choice, column swap and Householder reflector for step s (one block).
__global__ void qr_pivot_kernel(QR q, int s, double eps, int kcap) {
  __shared__ double bv[kT];
  __shared__ int bi[kT];
  __shared__ double red[kT / 64];
  __shared__ int p_sh;
  __shared__ int stop_sh;
  if (q.scal[2] != 0.0) return;
  // argmax of cnorm over j >= s, lowest index on ties
  double best = -1.0;
  int bidx = q.cols;
  for (int j = s + threadIdx.x; j < q.cols; j += blockDim.x) {
    const double v = q.cnorm[j];
    if (v > best) {
      best = v;
      bidx = j;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double v2 = bv[threadIdx.x + w];
      const int i2 = bi[threadIdx.x + w];
      if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int p = bi[0];
    const double nrm = sqrt(fmax(bv[0], 0.0));
    int stop = 0;
    if (s == 0) q.scal[0] = nrm;
    if (!(nrm > 0.0) || nrm <= eps * q.scal[0] || s >= kcap) stop = 1;
    if (stop) q.scal[2] = 1.0;
    p_sh = p;
    stop_sh = stop;
  }
  __syncthreads();
  if (stop_sh) return;
  const int p = p_sh;
  if (p != s) {
    c128* a = q.M + (int64_t)s * q.ld;
    c128* b = q.M + (int64_t)p * q.ld;
    for (int i = threadIdx.x; i < q.rows; i += blockDim.x) {
      const c128 t = a[i];
      a[i] = b[i];
      b[i] = t;
    }
    if (threadIdx.x == 0) {
      const double tn = q.cnorm[s];
      q.cnorm[s] = q.cnorm[p];
      q.cnorm[p] = tn;
      const int tp = q.perm[s];
      q.perm[s] = q.perm[p];
      q.perm[p] = tp;
    }
  }
  __syncthreads();
  // reflector for x = M[s:rows, s]: alpha = -e^{i arg x0} ||x||, v = x - alpha e1, tau = 2 / v^H v
  c128* x = q.M + (int64_t)s * q.ld;
  double ss = 0.0;
  for (int i = s + threadIdx.x; i < q.rows; i += blockDim.x) ss += x[i].re * x[i].re + x[i].im * x[i].im;
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    const double xn = sqrt(ss);
    const c128 x0 = x[s];
    const double a0 = hypot(x0.re, x0.im);
    const c128 ph = a0 > 0.0 ? c128{x0.re / a0, x0.im / a0} : c128{1.0, 0.0};
    const c128 alpha{-ph.re * xn, -ph.im * xn};
    x[s] = c128{x0.re - alpha.re, x0.im - alpha.im};
    const double vhv = 2.0 * xn * (xn + a0);
    q.alpha[s] = alpha;
    q.tau[s] = vhv > 0.0 ? 2.0 / vhv : 0.0;
    q.scal[1] = (double)(s + 1);
  }
}

// Apply the step-s reflector to one remaining matrix column or right-hand side per block.
__global__ void qr_apply_kernel(QR q, int s) {
  __shared__ double red[kT / 64];
  if (q.scal[2] != 0.0) return;
  const int nmat = q.cols - s - 1;
  const int b = blockIdx.x;
  c128* col;
  bool is_mat;
  if (b < nmat) {
    col = q.M + (int64_t)(s + 1 + b) * q.ld;
    is_mat = true;
  } else {
    col = q.rhs + (int64_t)(b - nmat) * q.ldr;
    is_mat = false;
  }
  const c128* v = q.M + (int64_t)s * q.ld;
  double dr = 0.0, di = 0.0;
  for (int i = s + threadIdx.x; i < q.rows; i += blockDim.x) {
    const c128 t = cconjmul(v[i], col[i]);
    dr += t.re;
    di += t.im;
  }
  dr = block_sum(dr, red);
  di = block_sum(di, red);
  const double tau = q.tau[s];
  const c128 f{tau * dr, tau * di};
  double nn = 0.0;
  for (int i = s + threadIdx.x; i < q.rows; i += blockDim.x) {
    const c128 t = cmul(v[i], f);
    c128 c = col[i];
    c.re -= t.re;
    c.im -= t.im;
    col[i] = c;
    if (i > s) nn += c.re * c.re + c.im * c.im;
  }
  if (is_mat) {
    nn = block_sum(nn, red);
    if (threadIdx.x == 0) q.cnorm[s + 1 + b] = nn;
  }
}

// Back substitution R11 x = rhs(0:r) per right-hand side column (one block each).
// If perm != null: X(perm[i], c) = x_i (i < r), X(perm[i], c) = 0 (r <= i < cols_out).
// Otherwise X(i, c) = x_i for i < r.  Column c sits at c * ldr in rhs and c * ldx in X, or where
// the column map puts it.
__global__ void backsub_kernel(const c128* __restrict__ M, int ldm, const c128* __restrict__ alpha, int r,
                               c128* rhs, int ldr, const int* __restrict__ perm, int cols_out, c128* X, int ldx,
                               ColMap cm) {
  __shared__ c128 xi_sh;
  const int c = blockIdx.x;
  c128* bcol = rhs + (cm.bodies ? cm.in_offset(c) : (int64_t)c * ldr);
  for (int i = r - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const c128 a = alpha[i];
      const double dd = a.re * a.re + a.im * a.im;
      const c128 bi = bcol[i];
      const c128 xv{(bi.re * a.re + bi.im * a.im) / dd, (bi.im * a.re - bi.re * a.im) / dd};
      bcol[i] = xv;
      xi_sh = xv;
    }
    __syncthreads();
    const c128 xv = xi_sh;
    const c128* mc = M + (int64_t)i * ldm;
    for (int t = threadIdx.x; t < i; t += blockDim.x) {
      const c128 u = cmul(mc[t], xv);
      bcol[t].re -= u.re;
      bcol[t].im -= u.im;
    }
    __syncthreads();
  }
  c128* xc = X + (cm.bodies ? cm.out_offset(c) : (int64_t)c * ldx);
  if (perm) {
    for (int i = threadIdx.x; i < cols_out; i += blockDim.x) xc[perm[i]] = i < r ? bcol[i] : c128{0.0, 0.0};
  } else {
    for (int i = threadIdx.x; i < r; i += blockDim.x) xc[i] = bcol[i];
  }
}

// Q^H applied to many right-hand sides with the stored reflectors of a factored matrix (one block
// per column): for s < rank, col[s:] -= v_s tau_s (v_s^H col[s:]), v_s = M[s:, s].
__global__ void qr_reflect_kernel(const c128* __restrict__ M, int rows, int ldm, const double* __restrict__ tau,
                                  int rank, c128* rhs, int ldr, ColMap cm) {
  __shared__ double red[kT / 64];
  c128* col = rhs + (cm.bodies ? cm.in_offset(blockIdx.x) : (int64_t)blockIdx.x * ldr);
  for (int s = 0; s < rank; ++s) {
    const c128* v = M + (int64_t)s * ldm;
    double dr = 0.0, di = 0.0;
    for (int i = s + threadIdx.x; i < rows; i += blockDim.x) {
      const c128 t = cconjmul(v[i], col[i]);
      dr += t.re;
      di += t.im;
    }
    dr = block_sum(dr, red);
    di = block_sum(di, red);
    const c128 f{tau[s] * dr, tau[s] * di};
    for (int i = s + threadIdx.x; i < rows; i += blockDim.x) {
      const c128 t = cmul(v[i], f);
      col[i].re -= t.re;
      col[i].im -= t.im;
    }
    __syncthreads();
  }
}

// C(MxN) = A(MxK) B(KxN), column-major, 16x16 tiles.
__global__ void zgemm_kernel(int Mr, int Nc, int K, const c128* __restrict__ A, int lda, const c128* __restrict__ B,
                             int ldb, c128* __restrict__ C, int ldc) {
  __shared__ c128 As[16][17];
  __shared__ c128 Bs[16][17];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = blockIdx.x * 16 + tx;
  const int j = blockIdx.y * 16 + ty;
  double ar = 0.0, ai = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int ka = k0 + ty;  // A tile: row i (tx), col ka
    As[tx][ty] = (i < Mr && ka < K) ? A[(int64_t)ka * lda + i] : c128{0.0, 0.0};
    const int kb = k0 + tx;  // B tile: row kb (tx), col j (ty)
    Bs[tx][ty] = (kb < K && j < Nc) ? B[(int64_t)j * ldb + kb] : c128{0.0, 0.0};
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const c128 a = As[tx][kk], b = Bs[kk][ty];
      ar = fma(a.re, b.re, fma(-a.im, b.im, ar));
      ai = fma(a.re, b.im, fma(a.im, b.re, ai));
    }
    __syncthreads();
  }
  if (i < Mr && j < Nc) C[(int64_t)j * ldc + i] = c128{ar, ai};
}

// out(j, i) = in(i, j) for an R x C block
__global__ void transpose_kernel(const c128* __restrict__ in, int ldi, int Rr, int Cc, c128* __restrict__ out,
                                 int ldo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < Rr) out[(int64_t)i * ldo + j] = in[(int64_t)j * ldi + i];
}

// Z*(k x m): Z*(:, perm[j]) = e_j for j < k, Z*(:, perm[k + l]) = T(:, l)
__global__ void build_zstar_kernel(const int* __restrict__ perm, int k, int m, const c128* __restrict__ T, int ldt,
                                   c128* __restrict__ Z) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;  // row of Z*
  const int j = blockIdx.y;                              // position in the pivot order
  if (i >= k) return;
  c128 v;
  if (j < k) v = c128{i == j ? 1.0 : 0.0, 0.0};
  else v = T[(int64_t)(j - k) * ldt + i];
  Z[(int64_t)perm[j] * k + i] = v;
}

__global__ void to_c64_kernel2(const c128* __restrict__ in, c64* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = c64{(float)in[i].re, (float)in[i].im};
}

// ------------------------------------------------------------------- host ---
struct DevMem {
  std::vector<void*> ptrs;
  ~DevMem() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
    if (e == hipSuccess) ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return e;
  }
};

#define LSQ_HIP(expr)                                                                       \
  do {                                                                                      \
    hipError_t e__ = (expr);                                                                \
    if (e__ != hipSuccess) {                                                                \
      (void)hipGetLastError();                                                              \
      return fail(e__ == hipErrorOutOfMemory ? MFS_ERR_NOMEM : MFS_ERR_HIP,                 \
                  std::string("build_S: ") + #expr + ": " + hipGetErrorString(e__));        \
    }                                                                                       \
  } while (0)

mfs_status assemble(int dim, double kappa, const double* tg, int rows, const double* src, int cols, c128* out, int ld,
                    hipStream_t st) {
  hipLaunchKernelGGL(assemble_kernel, dim3((rows + 127) / 128, cols), dim3(128), 0, st, dim, kappa, tg, rows, src,
                     cols, out, ld);
  LSQ_HIP(hipGetLastError());
  return MFS_OK;
}

// Factor M (rows x cols, destroyed) with column pivoting, apply Q^H to rhs (rows x nrhs, destroyed),
// and write the basic solution X (cols x nrhs, ld = cols).  Returns the numerical rank and
// |R_11| / |R_rr| through rank_out / ratio_out.  If X is null only the factorisation is done.
mfs_status qr_solve(DevMem& mem, c128* M, int rows, int cols, c128* rhs, int nrhs, double eps, int kcap, c128* X,
                    int* rank_out, double* ratio_out, int** perm_out, c128** alpha_out, hipStream_t st,
                    double** tau_out = nullptr) {
  QR q{};
  q.M = M;
  q.rows = rows;
  q.cols = cols;
  q.ld = rows;
  q.rhs = rhs;
  q.nrhs = nrhs;
  q.ldr = rows;
  LSQ_HIP(mem.alloc(&q.cnorm, cols));
  LSQ_HIP(mem.alloc(&q.perm, cols));
  LSQ_HIP(mem.alloc(&q.alpha, cols));
  LSQ_HIP(mem.alloc(&q.tau, cols));
  LSQ_HIP(mem.alloc(&q.scal, 4));
  hipLaunchKernelGGL(qr_init_kernel, dim3(cols), dim3(kT), 0, st, q);
  LSQ_HIP(hipGetLastError());
  const int steps = std::min(rows, cols);
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(qr_pivot_kernel, dim3(1), dim3(kT), 0, st, q, s, eps, kcap);
    const int nb = (cols - s - 1) + nrhs;
    if (nb > 0) hipLaunchKernelGGL(qr_apply_kernel, dim3(nb), dim3(kT), 0, st, q, s);
  }
  LSQ_HIP(hipGetLastError());
  double scal[3];
  LSQ_HIP(hipMemcpyAsync(scal, q.scal, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
  LSQ_HIP(hipStreamSynchronize(st));
  const int rank = (int)scal[1];
  if (rank == 0) return fail(MFS_ERR_RANK, "build_S: least-squares matrix has numerical rank 0");
  double ratio = 0.0;
  {
    c128 a0, ar;
    LSQ_HIP(hipMemcpy(&a0, q.alpha, sizeof(c128), hipMemcpyDeviceToHost));
    LSQ_HIP(hipMemcpy(&ar, q.alpha + (rank - 1), sizeof(c128), hipMemcpyDeviceToHost));
    ratio = std::hypot(a0.re, a0.im) / std::hypot(ar.re, ar.im);
  }
  if (X && nrhs > 0) {
    hipLaunchKernelGGL(backsub_kernel, dim3(nrhs), dim3(kT), 0, st, M, rows, q.alpha, rank, rhs, rows, q.perm, cols,
                       X, cols, ColMap{});
    LSQ_HIP(hipGetLastError());
  }
  *rank_out = rank;
  if (ratio_out) *ratio_out = ratio;
  if (perm_out) *perm_out = q.perm;
  if (alpha_out) *alpha_out = q.alpha;
  if (tau_out) *tau_out = q.tau;
  return MFS_OK;
}

mfs_status gemm(int Mr, int Nc, int K, const c128* A, int lda, const c128* B, int ldb, c128* C, int ldc,
                hipStream_t st) {
  hipLaunchKernelGGL(zgemm_kernel, dim3((Mr + 15) / 16, (Nc + 15) / 16), dim3(16, 16), 0, st, Mr, Nc, K, A, lda, B,
                     ldb, C, ldc);
  LSQ_HIP(hipGetLastError());
  return MFS_OK;
}

mfs_status transpose(const c128* in, int ldi, int Rr, int Cc, c128* out, int ldo, hipStream_t st) {
  hipLaunchKernelGGL(transpose_kernel, dim3((Rr + 127) / 128, Cc), dim3(128), 0, st, in, ldi, Rr, Cc, out, ldo);
  LSQ_HIP(hipGetLastError());
  return MFS_OK;
}

}  // namespace

mfs_status build_S_impl(const mfs_shape_desc* d, void* S64, void* S32, int64_t* k_out, int64_t* skel, double* diag,
                        hipStream_t st) {
  if (!d || !S64 || !k_out) return fail(MFS_ERR_ARG, "build_S: null descriptor, S64 or k_out");
  if (d->dim != 2 && d->dim != 3) return fail(MFS_ERR_ARG, "build_S: dim must be 2 or 3");
  if (!(d->kappa > 0.0)) return fail(MFS_ERR_ARG, "build_S: kappa must be > 0");
  if (!d->colloc || !d->src || !d->proxy) return fail(MFS_ERR_ARG, "build_S: null point set");
  if (d->m < 1 || d->n < 1 || d->p < 1 || d->n > d->m) return fail(MFS_ERR_ARG, "build_S: need 1 <= n <= m, p >= 1");
  if (d->m > 16384 || d->p > 16384) return fail(MFS_ERR_ARG, "build_S: m and p are limited to 16384");
  if (!(d->eps_ls > 0.0) || !(d->eps_ls < 1.0)) return fail(MFS_ERR_ARG, "build_S: need 0 < eps_ls < 1");
  const bool paper = d->eqpts == nullptr;
  if (!paper && (d->k < 1 || d->k > d->p || d->k > 4096))
    return fail(MFS_ERR_ARG, "build_S: given points need 1 <= k <= min(p, 4096)");
  if (paper && (d->k_cap < 1 || d->k_cap > std::min<int64_t>(std::min(d->p, d->m), 4096) ||
                !(d->eps_skel > 0.0) || !(d->eps_skel < 1.0)))
    return fail(MFS_ERR_ARG, "build_S: paper mode needs 1 <= k_cap <= min(p, m, 4096) and 0 < eps_skel < 1");
  const int dim = d->dim, m = (int)d->m, n = (int)d->n, p = (int)d->p;
  for (const double* arr : {d->colloc, d->src, d->proxy}) (void)arr;

  DevMem mem;
  double *xc, *ys, *zp, *xh = nullptr;
  LSQ_HIP(mem.alloc(&xc, (size_t)m * dim));
  LSQ_HIP(mem.alloc(&ys, (size_t)n * dim));
  LSQ_HIP(mem.alloc(&zp, (size_t)p * dim));
  LSQ_HIP(hipMemcpyAsync(xc, d->colloc, sizeof(double) * m * dim, hipMemcpyHostToDevice, st));
  LSQ_HIP(hipMemcpyAsync(ys, d->src, sizeof(double) * n * dim, hipMemcpyHostToDevice, st));
  LSQ_HIP(hipMemcpyAsync(zp, d->proxy, sizeof(double) * p * dim, hipMemcpyHostToDevice, st));

  int k = 0, rankA = 0, rankB = 0;
  double ratioB = 0.0;
  c128* Sdev = static_cast<c128*>(S64);
  mfs_status stt;

  c128* A;
  LSQ_HIP(mem.alloc(&A, (size_t)m * n));
  if ((stt = assemble(dim, d->kappa, xc, m, ys, n, A, m, st)) != MFS_OK) return stt;

  if (!paper) {
    k = (int)d->k;
    LSQ_HIP(mem.alloc(&xh, (size_t)k * dim));
    LSQ_HIP(hipMemcpyAsync(xh, d->eqpts, sizeof(double) * k * dim, hipMemcpyHostToDevice, st));
    c128 *Bh, *RHS1, *X1, *Ub, *Y;
    LSQ_HIP(mem.alloc(&Bh, (size_t)p * k));
    LSQ_HIP(mem.alloc(&RHS1, (size_t)p * (n + m)));
    LSQ_HIP(mem.alloc(&X1, (size_t)k * (n + m)));
    LSQ_HIP(mem.alloc(&Ub, (size_t)m * k));
    LSQ_HIP(mem.alloc(&Y, (size_t)n * k));
    if ((stt = assemble(dim, d->kappa, zp, p, xh, k, Bh, p, st)) != MFS_OK) return stt;
    if ((stt = assemble(dim, d->kappa, zp, p, ys, n, RHS1, p, st)) != MFS_OK) return stt;                    // D
    if ((stt = assemble(dim, d->kappa, zp, p, xc, m, RHS1 + (size_t)p * n, p, st)) != MFS_OK) return stt;   // B
    // X1 = B_hat^+ [D | B]   (k x (n + m))
    if ((stt = qr_solve(mem, Bh, p, k, RHS1, n + m, d->eps_ls, k, X1, &rankB, &ratioB, nullptr, nullptr, st)) !=
        MFS_OK)
      return stt;
    // Ub = (B_hat^+ B)^T  (m x k)
    if ((stt = transpose(X1 + (size_t)k * n, k, k, m, Ub, m, st)) != MFS_OK) return stt;
    // Y = A^+ Ub  (n x k)
    if ((stt = qr_solve(mem, A, m, n, Ub, k, d->eps_ls, n, Y, &rankA, nullptr, nullptr, nullptr, st)) != MFS_OK)
      return stt;
    // S = (B_hat^+ D) Y  (k x k)
    if ((stt = gemm(k, k, n, X1, k, Y, n, Sdev, k, st)) != MFS_OK) return stt;
  } else {
    const int kcap = (int)d->k_cap;
    c128 *B, *B2, *Dm, *C, *T, *Z, *U, *Y, *CY;
    LSQ_HIP(mem.alloc(&B, (size_t)p * m));
    if ((stt = assemble(dim, d->kappa, zp, p, xc, m, B, p, st)) != MFS_OK) return stt;
    int* perm = nullptr;
    c128* alphaB = nullptr;
    // CPQR of B stopped at eps_skel (Sec. 4.2): skeleton I = first k pivots
    if ((stt = qr_solve(mem, B, p, m, nullptr, 0, d->eps_skel, kcap, nullptr, &rankB, &ratioB, &perm, &alphaB, st)) !=
        MFS_OK)
      return stt;
    k = rankB;
    // T = R11^{-1} R12 with R12 = rows 0..k-1 of the remaining m - k columns
    LSQ_HIP(mem.alloc(&T, (size_t)k * std::max(1, m - k)));
    if (m > k) {
      c128* R12;
      LSQ_HIP(mem.alloc(&R12, (size_t)p * (m - k)));
      LSQ_HIP(hipMemcpy2DAsync(R12, sizeof(c128) * p, B + (size_t)k * p, sizeof(c128) * p, sizeof(c128) * k, m - k,
                               hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(backsub_kernel, dim3(m - k), dim3(kT), 0, st, B, p, alphaB, k, R12, p, (const int*)nullptr, k,
                         T, k, ColMap{});
      LSQ_HIP(hipGetLastError());
    }
    LSQ_HIP(mem.alloc(&Z, (size_t)k * m));
    hipLaunchKernelGGL(build_zstar_kernel, dim3((k + 127) / 128, m), dim3(128), 0, st, perm, k, m, T, k, Z);
    LSQ_HIP(hipGetLastError());
    // U = conj(Z) = (Z*)^T  (m x k)
    LSQ_HIP(mem.alloc(&U, (size_t)m * k));
    if ((stt = transpose(Z, k, k, m, U, m, st)) != MFS_OK) return stt;
    // C = B^+ D  (m x n), from a fresh B
    LSQ_HIP(mem.alloc(&B2, (size_t)p * m));
    LSQ_HIP(mem.alloc(&Dm, (size_t)p * n));
    LSQ_HIP(mem.alloc(&C, (size_t)m * n));
    if ((stt = assemble(dim, d->kappa, zp, p, xc, m, B2, p, st)) != MFS_OK) return stt;
    if ((stt = assemble(dim, d->kappa, zp, p, ys, n, Dm, p, st)) != MFS_OK) return stt;
    int rankB2 = 0;
    if ((stt = qr_solve(mem, B2, p, m, Dm, n, d->eps_ls, std::min(p, m), C, &rankB2, nullptr, nullptr, nullptr, st)) !=
        MFS_OK)
      return stt;
    // Y = A^+ U (n x k); CY = C Y (m x k); S = Z* CY (k x k)
    LSQ_HIP(mem.alloc(&Y, (size_t)n * k));
    LSQ_HIP(mem.alloc(&CY, (size_t)m * k));
    if ((stt = qr_solve(mem, A, m, n, U, k, d->eps_ls, n, Y, &rankA, nullptr, nullptr, nullptr, st)) != MFS_OK)
      return stt;
    if ((stt = gemm(m, k, n, C, m, Y, n, CY, m, st)) != MFS_OK) return stt;
    if ((stt = gemm(k, k, m, Z, k, CY, m, Sdev, k, st)) != MFS_OK) return stt;
    if (skel) {
      std::vector<int> ph(k);
      LSQ_HIP(hipMemcpyAsync(ph.data(), perm, sizeof(int) * k, hipMemcpyDeviceToHost, st));
      LSQ_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < k; ++i) skel[i] = ph[i];
    }
  }
  if (S32) {
    const int64_t kk = (int64_t)k * k;
    hipLaunchKernelGGL(to_c64_kernel2, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, st, Sdev,
                       static_cast<c64*>(S32), kk);
    LSQ_HIP(hipGetLastError());
  }
  LSQ_HIP(hipStreamSynchronize(st));
  *k_out = k;
  if (diag) {
    std::vector<c128> Sh((size_t)k * k);
    LSQ_HIP(hipMemcpy(Sh.data(), Sdev, sizeof(c128) * Sh.size(), hipMemcpyDeviceToHost));
    double num = 0.0, den = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const c128 a = Sh[(size_t)j * k + i], b = Sh[(size_t)i * k + j];
        num += (a.re - b.re) * (a.re - b.re) + (a.im - b.im) * (a.im - b.im);
        den += a.re * a.re + a.im * a.im;
      }
    diag[0] = rankA;
    diag[1] = rankB;
    diag[2] = ratioB;
    diag[3] = den > 0.0 ? std::sqrt(num / den) : 0.0;
  }
  return MFS_OK;
}

// Factors for the reconstruction of a body's MFS sources (Sec. 4.6): the pivoted QR of A, kept,
// and Y = A^+ U with U the map from values at the equivalent points to values at the collocation
// points ((B_hat^+ B)^T for given points, conj(Z) = (Z*)^T in paper mode; the same U as in S).
mfs_status build_recon_impl(const mfs_shape_desc* d, ReconFactors* out, hipStream_t st) {
  if (!d || !out) return fail(MFS_ERR_ARG, "recon: null descriptor or output");
  if (d->dim != 2 && d->dim != 3) return fail(MFS_ERR_ARG, "recon: dim must be 2 or 3");
  if (!(d->kappa > 0.0)) return fail(MFS_ERR_ARG, "recon: kappa must be > 0");
  if (!d->colloc || !d->src || !d->proxy) return fail(MFS_ERR_ARG, "recon: null point set");
  if (d->m < 1 || d->n < 1 || d->p < 1 || d->n > d->m) return fail(MFS_ERR_ARG, "recon: need 1 <= n <= m, p >= 1");
  if (d->m > 16384 || d->p > 16384) return fail(MFS_ERR_ARG, "recon: m and p are limited to 16384");
  if (!(d->eps_ls > 0.0) || !(d->eps_ls < 1.0)) return fail(MFS_ERR_ARG, "recon: need 0 < eps_ls < 1");
  const bool paper = d->eqpts == nullptr;
  if (!paper && (d->k < 1 || d->k > d->p || d->k > 4096))
    return fail(MFS_ERR_ARG, "recon: given points need 1 <= k <= min(p, 4096)");
  if (paper && (d->k_cap < 1 || d->k_cap > std::min<int64_t>(std::min(d->p, d->m), 4096) ||
                !(d->eps_skel > 0.0) || !(d->eps_skel < 1.0)))
    return fail(MFS_ERR_ARG, "recon: paper mode needs 1 <= k_cap <= min(p, m, 4096) and 0 < eps_skel < 1");
  const int dim = d->dim, m = (int)d->m, n = (int)d->n, p = (int)d->p;
  DevMem mem;
  double *xc, *ys, *zp;
  LSQ_HIP(mem.alloc(&xc, (size_t)m * dim));
  LSQ_HIP(mem.alloc(&ys, (size_t)n * dim));
  LSQ_HIP(mem.alloc(&zp, (size_t)p * dim));
  LSQ_HIP(hipMemcpyAsync(xc, d->colloc, sizeof(double) * m * dim, hipMemcpyHostToDevice, st));
  LSQ_HIP(hipMemcpyAsync(ys, d->src, sizeof(double) * n * dim, hipMemcpyHostToDevice, st));
  LSQ_HIP(hipMemcpyAsync(zp, d->proxy, sizeof(double) * p * dim, hipMemcpyHostToDevice, st));
  mfs_status stt;
  int k = 0;
  c128* U = nullptr;  // m x k
  if (!paper) {
    k = (int)d->k;
    double* xh;
    c128 *Bh, *B, *X;
    LSQ_HIP(mem.alloc(&xh, (size_t)k * dim));
    LSQ_HIP(hipMemcpyAsync(xh, d->eqpts, sizeof(double) * k * dim, hipMemcpyHostToDevice, st));
    LSQ_HIP(mem.alloc(&Bh, (size_t)p * k));
    LSQ_HIP(mem.alloc(&B, (size_t)p * m));
    LSQ_HIP(mem.alloc(&X, (size_t)k * m));
    LSQ_HIP(mem.alloc(&U, (size_t)m * k));
    if ((stt = assemble(dim, d->kappa, zp, p, xh, k, Bh, p, st)) != MFS_OK) return stt;
    if ((stt = assemble(dim, d->kappa, zp, p, xc, m, B, p, st)) != MFS_OK) return stt;
    int rankB = 0;
    if ((stt = qr_solve(mem, Bh, p, k, B, m, d->eps_ls, k, X, &rankB, nullptr, nullptr, nullptr, st)) != MFS_OK)
      return stt;
    if ((stt = transpose(X, k, k, m, U, m, st)) != MFS_OK) return stt;
  } else {
    const int kcap = (int)d->k_cap;
    c128 *B, *T, *Z;
    LSQ_HIP(mem.alloc(&B, (size_t)p * m));
    if ((stt = assemble(dim, d->kappa, zp, p, xc, m, B, p, st)) != MFS_OK) return stt;
    int* perm = nullptr;
    c128* alphaB = nullptr;
    int rankB = 0;
    if ((stt = qr_solve(mem, B, p, m, nullptr, 0, d->eps_skel, kcap, nullptr, &rankB, nullptr, &perm, &alphaB, st)) !=
        MFS_OK)
      return stt;
    k = rankB;
    LSQ_HIP(mem.alloc(&T, (size_t)k * std::max(1, m - k)));
    if (m > k) {
      c128* R12;
      LSQ_HIP(mem.alloc(&R12, (size_t)p * (m - k)));
      LSQ_HIP(hipMemcpy2DAsync(R12, sizeof(c128) * p, B + (size_t)k * p, sizeof(c128) * p, sizeof(c128) * k, m - k,
                               hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(backsub_kernel, dim3(m - k), dim3(kT), 0, st, B, p, alphaB, k, R12, p, (const int*)nullptr, k,
                         T, k, ColMap{});
      LSQ_HIP(hipGetLastError());
    }
    LSQ_HIP(mem.alloc(&Z, (size_t)k * m));
    hipLaunchKernelGGL(build_zstar_kernel, dim3((k + 127) / 128, m), dim3(128), 0, st, perm, k, m, T, k, Z);
    LSQ_HIP(hipGetLastError());
    LSQ_HIP(mem.alloc(&U, (size_t)m * k));
    if ((stt = transpose(Z, k, k, m, U, m, st)) != MFS_OK) return stt;
  }
  // A = phi(x - y), factored in place; Y = A^+ U
  c128 *A, *Y;
  LSQ_HIP(mem.alloc(&A, (size_t)m * n));
  LSQ_HIP(mem.alloc(&Y, (size_t)n * k));
  if ((stt = assemble(dim, d->kappa, xc, m, ys, n, A, m, st)) != MFS_OK) return stt;
  int rankA = 0;
  int* permA = nullptr;
  c128* alphaA = nullptr;
  double* tauA = nullptr;
  if ((stt = qr_solve(mem, A, m, n, U, k, d->eps_ls, n, Y, &rankA, nullptr, &permA, &alphaA, st, &tauA)) != MFS_OK)
    return stt;
  // keep what applying A^+ to new data needs, plus Y and the point sets, in one device block
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t oQA = 0, oAl = oQA + up(sizeof(c128) * m * n), oTau = oAl + up(sizeof(c128) * n),
               oPerm = oTau + up(sizeof(double) * n), oY = oPerm + up(sizeof(int) * n),
               oXc = oY + up(sizeof(c128) * n * k), oYs = oXc + up(sizeof(double) * m * dim),
               total = oYs + up(sizeof(double) * n * dim);
  size_t got = 0;
  hipError_t pe = hipSuccess;
  char* blk = static_cast<char*>(pool_alloc(total, st, &got, &pe));
  if (!blk) return fail(MFS_ERR_NOMEM, std::string("recon: device allocation failed: ") + hipGetErrorString(pe));
  auto d2d = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(blk + off, src, bytes, hipMemcpyDeviceToDevice, st);
  };
  hipError_t e = d2d(oQA, A, sizeof(c128) * m * n);
  if (e == hipSuccess) e = d2d(oAl, alphaA, sizeof(c128) * n);
  if (e == hipSuccess) e = d2d(oTau, tauA, sizeof(double) * n);
  if (e == hipSuccess) e = d2d(oPerm, permA, sizeof(int) * n);
  if (e == hipSuccess) e = d2d(oY, Y, sizeof(c128) * n * k);
  if (e == hipSuccess) e = d2d(oXc, xc, sizeof(double) * m * dim);
  if (e == hipSuccess) e = d2d(oYs, ys, sizeof(double) * n * dim);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the temporaries above are freed on return
  if (e != hipSuccess) {
    pool_free(blk, got, st);
    return fail(MFS_ERR_HIP, std::string("recon: ") + hipGetErrorString(e));
  }
  out->block = blk;
  out->block_bytes = got;
  out->QA = reinterpret_cast<c128*>(blk + oQA);
  out->alpha = reinterpret_cast<c128*>(blk + oAl);
  out->tau = reinterpret_cast<double*>(blk + oTau);
  out->perm = reinterpret_cast<int*>(blk + oPerm);
  out->Y = reinterpret_cast<c128*>(blk + oY);
  out->colloc = reinterpret_cast<double*>(blk + oXc);
  out->src = reinterpret_cast<double*>(blk + oYs);
  out->dim = dim;
  out->m = m;
  out->n = n;
  out->k = k;
  out->rank = rankA;
  out->kappa = d->kappa;
  return MFS_OK;
}

hipError_t launch_qr_reflect(const c128* QA, int rows, int ld, const double* tau, int rank, c128* rhs, int ldr,
                             int ncols, const ColMap& cm, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(qr_reflect_kernel, dim3(ncols), dim3(kT), 0, st, QA, rows, ld, tau, rank, rhs, ldr, cm);
  return hipGetLastError();
}

hipError_t launch_backsub(const c128* QA, int ld, const c128* alpha, int rank, c128* rhs, int ldr, const int* perm,
                          int cols_out, c128* X, int ldx, int ncols, const ColMap& cm, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(backsub_kernel, dim3(ncols), dim3(kT), 0, st, QA, ld, alpha, rank, rhs, ldr, perm, cols_out, X,
                     ldx, cm);
  return hipGetLastError();
}

}  // namespace mfs
