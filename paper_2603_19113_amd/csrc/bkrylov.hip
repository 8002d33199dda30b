// Block GMRES on gfx950: one Krylov space for all R right-hand sides of the global system
// (I + S G_hat) qhat = S vhat (eq. mbody2), solved by GMRES in the paper (Sec. 2.3).
//
// With R right-hand sides, step j applies the operator to the R basis vectors of block j at once
// (one many-right-hand-side pair-sum launch, Sec. 2.3's matvec on an N x R block) and extends the
// space by R vectors: K V_j = sum_{i<=j} V_i H_ij + V_{j+1} H_{j+1,j}.  Every right-hand side is
// then the best combination of the whole block space, which needs far fewer steps than R separate
// spaces when the right-hand sides excite related scattering (plane waves from many directions).
//
// Data layout (all column-major, a column being one length-N vector):
//   V       basis, slot j = N x R (the R vectors of block j, one after the other), so slots
//           0..j form one N x (j+1)R matrix with leading dimension N; complex64 in the mixed
//           solve (the FP32 operator reads it directly), complex128 otherwise.
//   Hp      block Hessenberg matrix, column block j ((j+2)R x R, leading dimension (j+2)R) at
//           offset R^2 j (j + 3) / 2; transformed in place into the triangular factor U.
//   refl    Householder vectors, one per column of the Hessenberg matrix: vector rho (for row
//           rho) has R + 1 entries acting on rows rho .. rho + R, normalised to |v|^2 = 2 so that
//           the reflector is I - v v^H.
//   g       the least-squares right side ((m+1)R x R), initially [B0; 0] with r0 = V_0 B0.
// Kernels:
//   bdots      part[s] = A^H B over a slice s of the rows (FP64 matrix cores, complex as four real
//              products), A the basis (complex64 or complex128) or a block, B a complex128 block;
//   breduce    sum of the slices in a fixed order (deterministic);
//   bgemm_nk   out = beta in + alpha A C, A N x K (complex64 or complex128), C K x R: the
//              Gram-Schmidt update, the triangular scaling of CholeskyQR, the back substitution's
//              updates and the solution update;
//   chol       Cholesky factor and its inverse of an R x R Gram matrix (one workgroup);
//   bhess_*    the Householder QR of the block Hessenberg matrix, updated one column block per
//              step, and the per-column residual norms.
#include <algorithm>

#include "mfs_internal.h"

namespace mfs {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ c128 load_c(const c64* p) {
  const c64 v = *p;
  return c128{(double)v.re, (double)v.im};
}
__device__ __forceinline__ c128 load_c(const c128* p) { return *p; }

constexpr int kTile = 64;   // output tile edge (rows of A^H B or of A C; right-hand sides)
constexpr int kSlab = 32;   // reduction slab staged in LDS per iteration
constexpr int kPadD = 66;   // LDS row length in doubles (64 + 2)

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- bdots ---
// part[s][c][k] = sum_{n in slice s} conj(A[k][n]) B[c][n] for k < K, c < R (A column k at
// A + k lda, B column c at B + c ldb).  Block (kt, s): rows 64 kt .. 64 kt + 63 of A^H B, slice s
// of n.  Wave w owns rows 16 w .. 16 w + 15 and all 64 columns (four 16 x 16 tiles, real and
// imaginary accumulators).  The 16x16x4 FP64 matrix-core product takes A (16 x 4) with lane l
// holding row l % 16, column l / 16, B (4 x 16) with lane l holding row l / 16, column l % 16, and
// leaves D row 4 v + l / 16, column l % 16 in register v of lane l (the FP32 16x16x4 product
// instead keeps four consecutive rows per lane group: row 4 (l / 16) + v).
template <typename TA>
__global__ __launch_bounds__(256) void bdots_kernel(const TA* __restrict__ A, int64_t lda, int K,
                                                    const c128* __restrict__ B, int64_t ldb, int R, int64_t N,
                                                    int64_t slice_len, c128* __restrict__ part) {
  __shared__ double Are[kSlab][kPadD], Aim[kSlab][kPadD], Bre[kSlab][kPadD], Bim[kSlab][kPadD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k0 = blockIdx.x * kTile;
  const int s = blockIdx.y;
  const int64_t n0 = (int64_t)s * slice_len;
  const int64_t n1 = min(N, n0 + slice_len);
  d4 accR[4], accI[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) accR[t] = accI[t] = d4{0.0, 0.0, 0.0, 0.0};
  // staging: thread tid loads column tid / 4 (of the 64), 8 consecutive n from (tid % 4) * 8
  const int col = tid >> 2, nq = (tid & 3) * 8;
  for (int64_t nb = n0; nb < n1; nb += kSlab) {
    {
      const int ka = k0 + col;
      const bool oka = ka < K, okb = col < R;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t n = nb + nq + i;
        const bool okn = n < n1;
        c128 a = {0.0, 0.0}, b = {0.0, 0.0};
        if (oka && okn) a = load_c(A + (int64_t)ka * lda + n);
        if (okb && okn) b = B[(int64_t)col * ldb + n];
        Are[nq + i][col] = a.re;
        Aim[nq + i][col] = a.im;
        Bre[nq + i][col] = b.re;
        Bim[nq + i][col] = b.im;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 4) {
      const int r = kk + (lane >> 4);
      const double ar = Are[r][16 * w + (lane & 15)], ai = Aim[r][16 * w + (lane & 15)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double br = Bre[r][16 * t + (lane & 15)], bi = Bim[r][16 * t + (lane & 15)];
        // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
        accR[t] = mfma(ar, br, accR[t]);
        accR[t] = mfma(ai, bi, accR[t]);
        accI[t] = mfma(ar, bi, accI[t]);
        accI[t] = mfma(-ai, br, accI[t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 16 * w + 4 * v + (lane >> 4);
      if (k < K && c < R) part[((int64_t)s * R + c) * K + k] = c128{accR[t][v], accI[t][v]};
    }
  }
}

// out[k + c ldo] (= or +=) sum_s part[s][c][k], slices in order; copy[k + c ldc] gets the sum too
// when copy is not null.
__global__ __launch_bounds__(256) void breduce_kernel(const c128* __restrict__ part, int nsplit, int K, int R,
                                                      c128* __restrict__ out, int64_t ldo, int accumulate,
                                                      c128* __restrict__ copy, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * R) return;
  const int c = (int)(i / K), k = (int)(i % K);
  double re = 0.0, im = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const c128 v = part[((int64_t)s * R + c) * K + k];
    re += v.re;
    im += v.im;
  }
  if (copy) copy[k + (int64_t)c * ldc] = c128{re, im};
  c128* o = out + k + (int64_t)c * ldo;
  if (accumulate) {
    o->re += re;
    o->im += im;
  } else {
    *o = c128{re, im};
  }
}

// ------------------------------------------------------------- bgemm_nk ---
// out[c ldo + n] = beta in[c ldi + n] + alpha sum_k A[k lda + n] C[k + c ldc] for n < M, c < R.
// Block: 64 rows n; wave w owns n 16 w .. 16 w + 15 and all 64 columns.  in may equal out.
template <typename TA>
__global__ __launch_bounds__(256) void bgemm_nk_kernel(const TA* __restrict__ A, int64_t lda, int64_t M, int K,
                                                       const c128* __restrict__ C, int64_t ldc, int R, double alpha,
                                                       double beta, const c128* in, int64_t ldi, c128* out,
                                                       int64_t ldo) {
  __shared__ double Are[kSlab][kPadD], Aim[kSlab][kPadD], Cre[kSlab][kPadD], Cim[kSlab][kPadD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n0 = (int64_t)blockIdx.x * kTile;
  d4 accR[4], accI[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) accR[t] = accI[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < K; kb += kSlab) {
    // A slab: 32 columns k x 64 rows n; thread tid: column tid / 8, 8 consecutive n from (tid % 8) * 8
    {
      const int kc = tid >> 3, nq = (tid & 7) * 8;
      const int k = kb + kc;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t n = n0 + nq + i;
        c128 a = {0.0, 0.0};
        if (k < K && n < M) a = load_c(A + (int64_t)k * lda + n);
        Are[kc][nq + i] = a.re;
        Aim[kc][nq + i] = a.im;
      }
      // C slab: 32 rows k x 64 columns c; thread tid: column tid / 4, 8 consecutive k from (tid % 4) * 8
      const int cc = tid >> 2, kq = (tid & 3) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = kb + kq + i;
        c128 v = {0.0, 0.0};
        if (kk < K && cc < R) v = C[kk + (int64_t)cc * ldc];
        Cre[kq + i][cc] = v.re;
        Cim[kq + i][cc] = v.im;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 4) {
      const int r = kk + (lane >> 4);
      const double ar = Are[r][16 * w + (lane & 15)], ai = Aim[r][16 * w + (lane & 15)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double cr = Cre[r][16 * t + (lane & 15)], ci = Cim[r][16 * t + (lane & 15)];
        // a c = (ar cr - ai ci) + i (ar ci + ai cr)
        accR[t] = mfma(ar, cr, accR[t]);
        accR[t] = mfma(-ai, ci, accR[t]);
        accI[t] = mfma(ar, ci, accI[t]);
        accI[t] = mfma(ai, cr, accI[t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + (lane & 15);
    if (c >= R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t n = n0 + 16 * w + 4 * v + (lane >> 4);
      if (n >= M) continue;
      c128 o = {alpha * accR[t][v], alpha * accI[t][v]};
      if (beta != 0.0) {
        const c128 x = in[(int64_t)c * ldi + n];
        o.re += beta * x.re;
        o.im += beta * x.im;
      }
      out[(int64_t)c * ldo + n] = o;
    }
  }
}

// ------------------------------------------------- FP32 matrix-core forms ---
// The same two products on the FP32 matrix cores (twice the FP64 rate), for the Gram-Schmidt passes
// of the mixed solve, whose basis is complex64 already: operands are rounded to FP32 when staged,
// each 32-long slab of the reduction is accumulated in FP32 (relative error ~ sqrt(32) 2^-24 of the
// slab's sum) and then added into FP64 accumulators, so the error does not grow with N or K.  The
// 16x16x4 FP32 product leaves D row 4 (l / 16) + v, column l % 16 in register v of lane l.
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kPadF = 68;  // LDS row length in floats (64 + 4)

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Staging of one slab: thread tid holds 8 consecutive entries of one column in registers (loaded
// for the next slab while the matrix cores work on the current one) and writes them to LDS.
struct SlabRegs {
  double re[8], im[8];
};

template <typename TA>
__device__ __forceinline__ void slab_load(SlabRegs& g, const TA* __restrict__ X, int64_t ldx, int col, bool okc,
                                          int64_t n, int64_t nend) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    c128 v = {0.0, 0.0};
    if (okc && n + i < nend) v = load_c(X + (int64_t)col * ldx + n + i);
    g.re[i] = v.re;
    g.im[i] = v.im;
  }
}

// The FP32 kernels stage in FP32: the rounding happens at the load instead of the LDS store (same
// values), and the staging takes half the registers.
struct SlabRegs32 {
  float re[8], im[8];
};

template <typename TA>
__device__ __forceinline__ void slab_load32(SlabRegs32& g, const TA* __restrict__ X, int64_t ldx, int col, bool okc,
                                            int64_t n, int64_t nend) {
  const TA* p = X + (int64_t)col * ldx + n;
  if (okc && n + 8 <= nend) {  // the common case: eight loads with no per-entry test
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const c128 v = load_c(p + i);
      g.re[i] = (float)v.re;
      g.im[i] = (float)v.im;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    c128 v = {0.0, 0.0};
    if (okc && n + i < nend) v = load_c(p + i);
    g.re[i] = (float)v.re;
    g.im[i] = (float)v.im;
  }
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void bdots32_kernel(const TA* __restrict__ A, int64_t lda, int K,
                                                      const TB* __restrict__ B, int64_t ldb, int R, int64_t N,
                                                      int64_t slice_len, c128* __restrict__ part) {
  __shared__ float Are[kSlab][kPadF], Aim[kSlab][kPadF], Bre[kSlab][kPadF], Bim[kSlab][kPadF];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k0 = blockIdx.x * kTile;
  const int s = blockIdx.y;
  const int64_t n0 = (int64_t)s * slice_len;
  const int64_t n1 = min(N, n0 + slice_len);
  d4 sumR[4], sumI[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) sumR[t] = sumI[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int col = tid >> 2, nq = (tid & 3) * 8;
  const bool oka = k0 + col < K, okb = col < R;
  SlabRegs32 ga, gb;
  if (n0 < n1) {
    slab_load32(ga, A, lda, k0 + col, oka, n0 + nq, n1);
    slab_load32(gb, B, ldb, col, okb, n0 + nq, n1);
  }
  for (int64_t nb = n0; nb < n1; nb += kSlab) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      Are[nq + i][col] = ga.re[i];
      Aim[nq + i][col] = ga.im[i];
      Bre[nq + i][col] = gb.re[i];
      Bim[nq + i][col] = gb.im[i];
    }
    __syncthreads();
    if (nb + kSlab < n1) {  // next slab in flight during the products
      slab_load32(ga, A, lda, k0 + col, oka, nb + kSlab + nq, n1);
      slab_load32(gb, B, ldb, col, okb, nb + kSlab + nq, n1);
    }
    f4 accR[4], accI[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) accR[t] = accI[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 4) {
      const int r = kk + (lane >> 4);
      const float ar = Are[r][16 * w + (lane & 15)], ai = Aim[r][16 * w + (lane & 15)];
      float br[4], bi[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        br[t] = Bre[r][16 * t + (lane & 15)];
        bi[t] = Bim[r][16 * t + (lane & 15)];
      }
      // eight accumulators between two products into the same one: no back-to-back dependence
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        accR[t] = mfma32(ar, br[t], accR[t]);
        accI[t] = mfma32(ar, bi[t], accI[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        accR[t] = mfma32(ai, bi[t], accR[t]);
        accI[t] = mfma32(-ai, br[t], accI[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sumR[t][v] += (double)accR[t][v];
        sumI[t][v] += (double)accI[t][v];
      }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 16 * w + 4 * (lane >> 4) + v;
      if (k < K && c < R) part[((int64_t)s * R + c) * K + k] = c128{sumR[t][v], sumI[t][v]};
    }
  }
}

template <typename TA, typename TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void bgemm32_nk_kernel(const TA* __restrict__ A, int64_t lda, int64_t M, int K,
                                                         const TC* __restrict__ C, int64_t ldc, int R, double alpha,
                                                         double beta, const c128* in, int64_t ldi, c128* out,
                                                         int64_t ldo) {
  __shared__ float Are[kSlab][kPadF], Aim[kSlab][kPadF], Cre[kSlab][kPadF], Cim[kSlab][kPadF];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n0 = (int64_t)blockIdx.x * kTile;
  d4 sumR[4], sumI[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) sumR[t] = sumI[t] = d4{0.0, 0.0, 0.0, 0.0};
  // A slab: 32 columns k x 64 rows n, thread tid: column tid / 8, n from (tid % 8) * 8;
  // C slab: 32 rows k x 64 columns c, thread tid: column tid / 4, k from (tid % 4) * 8
  const int kc = tid >> 3, nq = (tid & 7) * 8;
  const int cc = tid >> 2, kq = (tid & 3) * 8;
  SlabRegs32 ga, gc;
  auto load = [&](int kb) {
    const int k = kb + kc;
    const TA* pa = A + (int64_t)k * lda + n0 + nq;
    if (k < K && n0 + nq + 8 <= M) {  // the common case: no per-entry test
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const c128 a = load_c(pa + i);
        ga.re[i] = (float)a.re;
        ga.im[i] = (float)a.im;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        c128 a = {0.0, 0.0};
        if (k < K && n0 + nq + i < M) a = load_c(pa + i);
        ga.re[i] = (float)a.re;
        ga.im[i] = (float)a.im;
      }
    }
    const TC* pc = C + kb + kq + (int64_t)cc * ldc;
    if (cc < R && kb + kq + 8 <= K) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const c128 v = load_c(pc + i);
        gc.re[i] = (float)v.re;
        gc.im[i] = (float)v.im;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        c128 v = {0.0, 0.0};
        if (cc < R && kb + kq + i < K) v = load_c(pc + i);
        gc.re[i] = (float)v.re;
        gc.im[i] = (float)v.im;
      }
    }
  };
  if (K > 0) load(0);
  for (int kb = 0; kb < K; kb += kSlab) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      Are[kc][nq + i] = ga.re[i];
      Aim[kc][nq + i] = ga.im[i];
      Cre[kq + i][cc] = gc.re[i];
      Cim[kq + i][cc] = gc.im[i];
    }
    __syncthreads();
    if (kb + kSlab < K) load(kb + kSlab);  // next slab in flight during the products
    f4 accR[4], accI[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) accR[t] = accI[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 4) {
      const int r = kk + (lane >> 4);
      const float ar = Are[r][16 * w + (lane & 15)], ai = Aim[r][16 * w + (lane & 15)];
      float cr[4], ci[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        cr[t] = Cre[r][16 * t + (lane & 15)];
        ci[t] = Cim[r][16 * t + (lane & 15)];
      }
      // eight accumulators between two products into the same one: no back-to-back dependence
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        accR[t] = mfma32(ar, cr[t], accR[t]);
        accI[t] = mfma32(ar, ci[t], accI[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        accR[t] = mfma32(-ai, ci[t], accR[t]);
        accI[t] = mfma32(ai, cr[t], accI[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sumR[t][v] += (double)accR[t][v];
        sumI[t][v] += (double)accI[t][v];
      }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + (lane & 15);
    if (c >= R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t n = n0 + 16 * w + 4 * (lane >> 4) + v;
      if (n >= M) continue;
      c128 o = {alpha * sumR[t][v], alpha * sumI[t][v]};
      if (beta != 0.0) {
        const c128 x = in[(int64_t)c * ldi + n];
        o.re += beta * x.re;
        o.im += beta * x.im;
      }
      out[(int64_t)c * ldo + n] = o;
    }
  }
}

// ----------------------------------------------------------------- chol ---
// One step of shifted CholeskyQR on an R x R Gram matrix G = W^H W (column-major, Hermitian).
// scale != 0: the columns are first scaled to unit norm (d_c = sqrt(G_cc), 1 where G_cc = 0) and
// shift * I is added, the first step of shifted CholeskyQR3.  Writes the upper factor F = U D and
// Finv = D^{-1} U^{-1} (W Finv has orthonormal columns, W = (W Finv) F) and updates the
// accumulated factor: Rtot = F Rtot (Rtot = F when first != 0).
// A column whose pivot^2 falls to dep_tol (W's column k lies in the span of columns 0..k-1) is
// dependent: its row of F is zero and its column of Finv is zero, so W = (W Finv) F still holds
// whatever vector later takes that (zero) column of W Finv; dep[k] is set to 1 and *flag to 1.
__global__ __launch_bounds__(256) void chol_kernel(const c128* __restrict__ G, int R, int scale, double shift, int first,
                                                   double dep_tol, c128* __restrict__ F, c128* __restrict__ Finv,
                                                   c128* __restrict__ Rtot, int32_t* __restrict__ dep,
                                                   int32_t* __restrict__ flag) {
  __shared__ double Ur[64][65], Ui[64][65], Vr[64][65], Vi[64][65], d[64];
  __shared__ int dk[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    const c128 v = G[e];
    Ur[i][j] = v.re;
    Ui[i][j] = v.im;
  }
  if (tid < R) {
    if (first) dep[tid] = 0;
    dk[tid] = 0;
  }
  __syncthreads();
  if (tid < R) {
    const double gg = Ur[tid][tid];
    d[tid] = scale ? (gg > 0.0 ? sqrt(gg) : 1.0) : 1.0;
  }
  __syncthreads();
  if (scale) {
    for (int e = tid; e < R * R; e += blockDim.x) {
      const int i = e % R, j = e / R;
      const double f = 1.0 / (d[i] * d[j]);
      Ur[i][j] *= f;
      Ui[i][j] *= f;
      if (i == j) Ur[i][j] += shift;
    }
    __syncthreads();
  }
  // upper Cholesky G = U^H U, right-looking on the upper triangle
  for (int k = 0; k < R; ++k) {
    if (tid == 0) {
      const double p = Ur[k][k];
      if (!(p > dep_tol) || !(p > 1e-300)) {
        dk[k] = 1;  // dependent: unit pivot with a zero row, so the trailing update is unchanged
        Ur[k][k] = 1.0;
        dep[k] = 1;
        *flag = 1;
      } else {
        Ur[k][k] = sqrt(p);
      }
      Ui[k][k] = 0.0;
    }
    __syncthreads();
    const double inv = 1.0 / Ur[k][k];
    for (int j = k + 1 + tid; j < R; j += blockDim.x) {
      if (dk[k]) {
        Ur[k][j] = Ui[k][j] = 0.0;
      } else {
        Ur[k][j] *= inv;
        Ui[k][j] *= inv;
      }
    }
    __syncthreads();
    // U[i][j] -= conj(U[k][i]) U[k][j] for k < i <= j
    for (int e = tid; e < R * R; e += blockDim.x) {
      const int i = e % R, j = e / R;
      if (i > k && j >= i) {
        const double ar = Ur[k][i], ai = -Ui[k][i], br = Ur[k][j], bi = Ui[k][j];
        Ur[i][j] -= ar * br - ai * bi;
        Ui[i][j] -= ar * bi + ai * br;
      }
    }
    __syncthreads();
  }
  // zero the strict lower triangle; inverse of the upper factor, one column per thread:
  // U X = I, column j: X[i][j] for i = j down to 0
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    if (i > j) Ur[i][j] = Ui[i][j] = 0.0;
    Vr[i][j] = Vi[i][j] = 0.0;
  }
  __syncthreads();
  if (tid < R) {
    const int j = tid;
    for (int i = j; i >= 0; --i) {
      double sr = (i == j) ? 1.0 : 0.0, si = 0.0;
      for (int q = i + 1; q <= j; ++q) {
        sr -= Ur[i][q] * Vr[q][j] - Ui[i][q] * Vi[q][j];
        si -= Ur[i][q] * Vi[q][j] + Ui[i][q] * Vr[q][j];
      }
      Vr[i][j] = sr / Ur[i][i];  // the diagonal is real
      Vi[i][j] = si / Ur[i][i];
    }
  }
  __syncthreads();
  // dependent columns: zero row of F (including its unit pivot), zero column of Finv
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    if (dk[i]) Ur[i][j] = Ui[i][j] = 0.0;
    if (dk[j]) Vr[i][j] = Vi[i][j] = 0.0;
  }
  __syncthreads();
  // F = U D, Finv = D^{-1} U^{-1}
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    F[e] = c128{Ur[i][j] * d[j], Ui[i][j] * d[j]};
    Finv[e] = c128{Vr[i][j] / d[i], Vi[i][j] / d[i]};
  }
  __syncthreads();
  // Rtot = F Rtot (both upper triangular)
  if (first) {
    for (int e = tid; e < R * R; e += blockDim.x) {
      const int i = e % R, j = e / R;
      Rtot[e] = c128{Ur[i][j] * d[j], Ui[i][j] * d[j]};
    }
    return;
  }
  // stage Rtot in V (the inverse is no longer needed in LDS)
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    const c128 v = Rtot[e];
    Vr[i][j] = v.re;
    Vi[i][j] = v.im;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    double sr = 0.0, si = 0.0;
    for (int q = i; q <= j; ++q) {
      const double fr = Ur[i][q] * d[q], fi = Ui[i][q] * d[q];
      sr += fr * Vr[q][j] - fi * Vi[q][j];
      si += fr * Vi[q][j] + fi * Vr[q][j];
    }
    Rtot[e] = c128{sr, si};
  }
}

// --------------------------------------------------------- Householder ---
// The window of R + 1 rows a reflector acts on: lane p holds row base + p for p < 64; row base + 64
// (only when R = 64) sits in lane 63's second register.
struct Window {
  double ar, ai;  // row base + lane
  double br, bi;  // row base + 64 (lane 63, R = 64)
};

// A double moved across lanes by one DPP pattern (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Lane `src`'s value (src wave-uniform), in every lane.
__device__ __forceinline__ double read_lane_d(double x, int src) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave, the same bits in every lane: pairs within quads (quad_perm [1,0,3,2], then
// [2,3,0,1]), half rows (row_half_mirror) and rows of 16 (row_mirror) by DPP, every lane adding the
// same two values, then the four row sums (lanes 0, 16, 32, 48) in a fixed order.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x141>(x);
  x += dpp_d<0x140>(x);
  return (read_lane_d(x, 0) + read_lane_d(x, 16)) + (read_lane_d(x, 32) + read_lane_d(x, 48));
}

__device__ __forceinline__ void window_load(Window& wv, const c128* __restrict__ X, int64_t base, int R, int lane) {
  wv.ar = wv.ai = wv.br = wv.bi = 0.0;
  if (lane <= R && lane < 64) {
    const c128 v = X[base + lane];
    wv.ar = v.re;
    wv.ai = v.im;
  }
  if (R == 64 && lane == 63) {
    const c128 v = X[base + 64];
    wv.br = v.re;
    wv.bi = v.im;
  }
}

__device__ __forceinline__ void window_store(const Window& wv, c128* __restrict__ X, int64_t base, int R, int lane) {
  if (lane <= R && lane < 64) X[base + lane] = c128{wv.ar, wv.ai};
  if (R == 64 && lane == 63) X[base + 64] = c128{wv.br, wv.bi};
}

// One reflector's entries as the window holds them: lane p entry p, lane 63 also entry 64 (R = 64).
struct Refl {
  double vr, vi, ur, ui;
};

// Every lane loads (entries min(lane, R) and min(lane + 1, R): no branch around the loads, so that a
// load issued one reflector ahead stays in flight) and keeps what the window needs.
__device__ __forceinline__ Refl refl_load(const c128* __restrict__ v, int R, int lane) {
  const c128 t0 = v[min(lane, R)], t1 = v[min(lane + 1, R)];
  const bool in = lane <= R, last = R == 64 && lane == 63;
  return Refl{in ? t0.re : 0.0, in ? t0.im : 0.0, last ? t1.re : 0.0, last ? t1.im : 0.0};
}

// x <- (I - v v^H) x on the window
__device__ __forceinline__ void window_reflect(Window& wv, const Refl& f) {
  const double vr = f.vr, vi = f.vi, ur = f.ur, ui = f.ui;
  // s = v^H x
  double sr = vr * wv.ar + vi * wv.ai + ur * wv.br + ui * wv.bi;
  double si = vr * wv.ai - vi * wv.ar + ur * wv.bi - ui * wv.br;
  sr = wave_sum(sr);
  si = wave_sum(si);
  wv.ar -= vr * sr - vi * si;
  wv.ai -= vr * si + vi * sr;
  wv.br -= ur * sr - ui * si;
  wv.bi -= ur * si + ui * sr;
}

// Slide the window down one row: row base is final (stored), rows base+1 .. base+R stay (lane l
// receives lane l + 1's values: DPP wave_rol:1), and row base+R+1 = (nr_in, ni_in) comes in.
__device__ __forceinline__ void window_slide(Window& wv, c128* __restrict__ X, int64_t base, int R, int lane,
                                             double nr_in, double ni_in) {
  if (lane == 0) X[base] = c128{wv.ar, wv.ai};
  double nr = dpp_d<0x134>(wv.ar), ni = dpp_d<0x134>(wv.ai);
  if (R == 64) {
    if (lane == 63) {
      nr = wv.br;
      ni = wv.bi;
      wv.br = nr_in;
      wv.bi = ni_in;
    }
  } else if (lane == R) {
    nr = nr_in;
    ni = ni_in;
  } else if (lane > R) {
    nr = ni = 0.0;
  }
  wv.ar = nr;
  wv.ai = ni;
}

// Apply reflectors rho0 .. rho1 - 1 (reflector rho acts on rows rho .. rho + R) to column
// blockIdx.x of X (column c at X + c ldx).  One wave per column; columns are independent.  The
// chain from one reflector to the next is the wave's two sums and one row shift, all DPP: the next
// reflector's entries are loaded during the current one, and the rows the slides bring in are
// loaded 64 at a time (lane l: the row of slide 64 c + l), a chunk ahead of their use.
__global__ __launch_bounds__(64) void bhess_apply_kernel(const c128* __restrict__ refl, int R, int64_t rho0,
                                                         int64_t rho1, c128* __restrict__ X, int64_t ldx) {
  const int lane = threadIdx.x;
  c128* x = X + (int64_t)blockIdx.x * ldx;
  if (rho1 <= rho0) return;
  Window wv;
  window_load(wv, x, rho0, R, lane);
  // the slide after reflector rho brings in row rho + off (for rho < rho1 - 1); the next reflector
  // and the next incoming row are loaded one step ahead, without branches (clamped indices)
  const int64_t off = R == 64 ? 65 : R + 1;
  const int64_t rlast = rho1 - 2;  // the last reflector followed by a slide
  // the row slide rho brings in; past the last slide any row of the window (its value is unused),
  // so that no load leaves the rows the sweep touches
  auto row_in = [&](int64_t rho) { return rho <= rlast ? rho + off : rho0; };
  Refl f = refl_load(refl + rho0 * (R + 1), R, lane);
  c128 rin = x[row_in(rho0)];
  for (int64_t rho = rho0; rho < rho1; ++rho) {
    const int64_t rn = min(rho + 1, rho1 - 1);
    const Refl fn = refl_load(refl + rn * (R + 1), R, lane);
    const c128 rin_n = x[row_in(rho + 1)];
    window_reflect(wv, f);
    if (rho + 1 < rho1) window_slide(wv, x, rho, R, lane, rin.re, rin.im);
    f = fn;
    rin = rin_n;
  }
  window_store(wv, x, rho1 - 1, R, lane);
}

// Slide the window up one row: row base + R is final (stored), rows base-1 .. base+R-1 stay (lane l
// receives lane l - 1's values: DPP wave_ror:1) or load.
__device__ __forceinline__ void window_slide_up(Window& wv, c128* __restrict__ X, int64_t base, int R, int lane) {
  if (R == 64) {
    if (lane == 63) X[base + 64] = c128{wv.br, wv.bi};
  } else if (lane == R) {
    X[base + R] = c128{wv.ar, wv.ai};
  }
  double nr = dpp_d<0x13C>(wv.ar), ni = dpp_d<0x13C>(wv.ai);
  if (R == 64 && lane == 63) {
    wv.br = wv.ar;  // old row base + 63 becomes position 64
    wv.bi = wv.ai;
  }
  if (lane == 0) {
    const c128 t = X[base - 1];
    nr = t.re;
    ni = t.im;
  } else if (lane > R) {
    nr = ni = 0.0;
  }
  wv.ar = nr;
  wv.ai = ni;
}

// Apply reflectors rho1 - 1 down to rho0 (the product H_rho0 ... H_{rho1-1} = the unitary factor Q of
// the Hessenberg QR, where the forward order gives Q^H) to column blockIdx.x of X.
__global__ __launch_bounds__(64) void bhess_apply_rev_kernel(const c128* __restrict__ refl, int R, int64_t rho0,
                                                             int64_t rho1, c128* __restrict__ X, int64_t ldx) {
  const int lane = threadIdx.x;
  c128* x = X + (int64_t)blockIdx.x * ldx;
  if (rho1 <= rho0) return;
  Window wv;
  window_load(wv, x, rho1 - 1, R, lane);
  Refl f = refl_load(refl + (rho1 - 1) * (R + 1), R, lane);
  for (int64_t rho = rho1 - 1; rho >= rho0; --rho) {
    const Refl fn = rho > rho0 ? refl_load(refl + (rho - 1) * (R + 1), R, lane) : Refl{0.0, 0.0, 0.0, 0.0};
    window_reflect(wv, f);
    if (rho > rho0) window_slide_up(wv, x, rho, R, lane);
    f = fn;
  }
  window_store(wv, x, rho0, R, lane);
}

// QR of the new column block's bottom 2R x R part (rows jR .. (j+2)R - 1; the lower R x R block is
// upper triangular): for column c, the reflectors jR .. jR + c - 1 already built are applied, then
// reflector jR + c is formed from rows jR + c .. jR + c + R and stored, leaving alpha on the
// diagonal and zeros below.  One wave; the columns are done one after another.
__global__ __launch_bounds__(64) void bhess_newqr_kernel(c128* __restrict__ refl, int R, int64_t jR,
                                                         c128* __restrict__ X, int64_t ldx) {
  const int lane = threadIdx.x;
  for (int c = 0; c < R; ++c) {
    c128* x = X + (int64_t)c * ldx;
    Window wv;
    window_load(wv, x, jR, R, lane);
    for (int q = 0; q < c; ++q) {
      window_reflect(wv, refl_load(refl + (jR + q) * (R + 1), R, lane));
      const c128 tin = x[jR + q + (R == 64 ? 65 : R + 1)];  // the row the slide brings in
      window_slide(wv, x, jR + q, R, lane, tin.re, tin.im);
    }
    // reflector from the window at base jR + c: x -> alpha e_0, alpha = -e^{i arg x0} |x|
    const double nrm2 = wave_sum(wv.ar * wv.ar + wv.ai * wv.ai + wv.br * wv.br + wv.bi * wv.bi);
    const double x0r = __shfl(wv.ar, 0, 64), x0i = __shfl(wv.ai, 0, 64);
    const double nx = sqrt(nrm2), a0 = sqrt(x0r * x0r + x0i * x0i);
    const double er = a0 > 0.0 ? x0r / a0 : 1.0, ei = a0 > 0.0 ? x0i / a0 : 0.0;
    const double alr = -er * nx, ali = -ei * nx;
    // v = x - alpha e0, scaled to |v|^2 = 2
    double vr = wv.ar, vi = wv.ai, ur = wv.br, ui = wv.bi;
    if (lane == 0) {
      vr -= alr;
      vi -= ali;
    }
    const double nv2 = wave_sum(vr * vr + vi * vi + ur * ur + ui * ui);
    const double sc = nv2 > 0.0 ? sqrt(2.0 / nv2) : 0.0;
    c128* v = refl + (jR + c) * (R + 1);
    if (lane <= R && lane < 64) v[lane] = c128{vr * sc, vi * sc};
    if (R == 64 && lane == 63) v[64] = c128{ur * sc, ui * sc};
    // the column after its reflector: alpha on the diagonal, zeros below
    if (lane <= R && lane < 64) x[jR + c + lane] = lane == 0 ? c128{alr, ali} : c128{0.0, 0.0};
    if (R == 64 && lane == 63) x[jR + c + 64] = c128{0.0, 0.0};
    __syncthreads();  // the stored reflector is read by the next column
  }
}

// res[c] = |g[(j+1)R .. (j+2)R - 1, c]| / bnorm[c] (0 where bnorm is 0)
__global__ __launch_bounds__(64) void bres_kernel(const c128* __restrict__ g, int64_t ldg, int64_t row0, int R,
                                                  const double* __restrict__ bnorm, double* __restrict__ res) {
  const int c = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int i = lane; i < R; i += 64) {
    const c128 v = g[(int64_t)c * ldg + row0 + i];
    s += v.re * v.re + v.im * v.im;
  }
  s = wave_sum(s);
  if (lane == 0) res[c] = bnorm[c] > 0.0 ? sqrt(s) / bnorm[c] : 0.0;
}

// Y rows of block i = U_ii^{-1} g rows of block i (U_ii upper triangular R x R at U, leading
// dimension ldu), all R right-hand sides; one thread per right-hand side.
__global__ __launch_bounds__(64) void btrsm_diag_kernel(const c128* __restrict__ U, int64_t ldu, const c128* __restrict__ g,
                                                        int64_t ldg, c128* __restrict__ Y, int64_t ldy, int R) {
  __shared__ double Ur[64][65], Ui[64][65];
  const int tid = threadIdx.x;
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    const c128 v = U[i + (int64_t)j * ldu];
    Ur[i][j] = v.re;
    Ui[i][j] = v.im;
  }
  __syncthreads();
  if (tid >= R) return;
  const int c = tid;
  double yr[64], yi[64];
  for (int i = 0; i < R; ++i) {
    const c128 v = g[(int64_t)c * ldg + i];
    yr[i] = v.re;
    yi[i] = v.im;
  }
  for (int i = R - 1; i >= 0; --i) {
    double sr = yr[i], si = yi[i];
    for (int q = i + 1; q < R; ++q) {
      sr -= Ur[i][q] * yr[q] - Ui[i][q] * yi[q];
      si -= Ur[i][q] * yi[q] + Ui[i][q] * yr[q];
    }
    // (sr + i si) / (ur + i ui)
    const double ur = Ur[i][i], ui = Ui[i][i];
    const double den = ur * ur + ui * ui;
    yr[i] = den > 0.0 ? (sr * ur + si * ui) / den : 0.0;
    yi[i] = den > 0.0 ? (si * ur - sr * ui) / den : 0.0;
  }
  for (int i = 0; i < R; ++i) Y[(int64_t)c * ldy + i] = c128{yr[i], yi[i]};
}

// x[c][i] = i-th pseudo-random unit-modulus value (c seeds the sequence) where bnorm[c] == 0: a
// start vector for a right-hand side that is zero (its solution is zero whatever the vector).
__global__ void fill_zero_columns_kernel(c128* __restrict__ X, int64_t N, int R, const double* __restrict__ bnorm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N || bnorm[c] > 0.0) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + (uint64_t)(c + 1) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double a = (double)(z >> 11) * (2.0 * M_PI / 9007199254740992.0);
  X[(int64_t)c * N + i] = c128{cos(a), sin(a)};
}

// x[i] = a pseudo-random unit-modulus value, the sequence picked by seed (a start direction for a
// column that the block space has to complete).
__global__ void fill_random_kernel(c128* __restrict__ x, int64_t N, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + (seed + 1) * 0xD1B54A32D192ED03ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double a = (double)(z >> 11) * (2.0 * M_PI / 9007199254740992.0);
  x[i] = c128{cos(a), sin(a)};
}

// M[i + c ldm] = 0 for every row i < rows of the columns c with bnorm[c] == 0 (right-hand sides
// that are zero keep a zero least-squares right side, so their correction stays zero).
__global__ void mask_zero_columns_kernel(c128* __restrict__ M, int64_t ldm, int rows, int R,
                                         const double* __restrict__ bnorm) {
  const int c = blockIdx.x;
  if (bnorm[c] > 0.0) return;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) M[i + (int64_t)c * ldm] = c128{0.0, 0.0};
}

// X[row0 + c + c ldx] += 1 for c < R: the identity of I + S G_hat on the diagonal block of the
// Hessenberg column (the operator is applied as S G_hat alone).
__global__ void add_identity_kernel(c128* __restrict__ X, int64_t ldx, int64_t row0, int R) {
  const int c = threadIdx.x;
  if (c < R) X[row0 + c + (int64_t)c * ldx].re += 1.0;
}

// out[i + c ldo] (= or +=) in[i + c ldi] for i < rows, c < cols.
__global__ void copy2d_kernel(const c128* __restrict__ in, int64_t ldi, int64_t rows, int cols, c128* __restrict__ out,
                              int64_t ldo, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= rows || c >= cols) return;
  const c128 v = in[i + (int64_t)c * ldi];
  c128* o = out + i + (int64_t)c * ldo;
  if (accumulate) {
    o->re += v.re;
    o->im += v.im;
  } else {
    *o = v;
  }
}

}  // namespace

hipError_t launch_copy2d(const c128* in, int64_t ldi, int64_t rows, int cols, c128* out, int64_t ldo, bool accumulate,
                         hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_kernel, dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0, st, in, ldi, rows,
                     cols, out, ldo, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mask_zero_columns(c128* M, int64_t ldm, int rows, int R, const double* bnorm, hipStream_t st) {
  hipLaunchKernelGGL(mask_zero_columns_kernel, dim3((unsigned)R), dim3(64), 0, st, M, ldm, rows, R, bnorm);
  return hipGetLastError();
}

hipError_t launch_fill_random(c128* x, int64_t N, uint64_t seed, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_random_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, x, N, seed);
  return hipGetLastError();
}

hipError_t launch_add_identity(c128* X, int64_t ldx, int64_t row0, int R, hipStream_t st) {
  hipLaunchKernelGGL(add_identity_kernel, dim3(1), dim3(64), 0, st, X, ldx, row0, R);
  return hipGetLastError();
}

int bdots_splits(int64_t N, int K) {
  const int ktiles = (K + kTile - 1) / kTile;
  // about 2048 blocks in flight, at least 2048 rows per slice, the partial sums within kBdotsPartMax
  int64_t s = std::max<int64_t>(1, 2048 / ktiles);
  s = std::min<int64_t>(s, std::max<int64_t>(1, N / 2048));
  s = std::min<int64_t>(s, std::max<int64_t>(1, kBdotsPartMax / std::max(K, 1)));
  return (int)s;
}

hipError_t launch_bdots(const void* A, bool a32, int64_t lda, int K, const c128* B, int64_t ldb, int R, int64_t N,
                        c128* part, int nsplit, hipStream_t st, bool fp32) {
  if (K <= 0 || N <= 0) return hipSuccess;
  const int64_t slice = ((N + nsplit - 1) / nsplit + kSlab - 1) / kSlab * kSlab;
  const dim3 grid((unsigned)((K + kTile - 1) / kTile), (unsigned)nsplit);
  if (fp32) {
    if (a32)
      hipLaunchKernelGGL((bdots32_kernel<c64, c128>), grid, dim3(256), 0, st, static_cast<const c64*>(A), lda, K, B, ldb,
                         R, N, slice, part);
    else
      hipLaunchKernelGGL((bdots32_kernel<c128, c128>), grid, dim3(256), 0, st, static_cast<const c128*>(A), lda, K, B,
                         ldb, R, N, slice, part);
    return hipGetLastError();
  }
  if (a32)
    hipLaunchKernelGGL(bdots_kernel<c64>, grid, dim3(256), 0, st, static_cast<const c64*>(A), lda, K, B, ldb, R, N,
                       slice, part);
  else
    hipLaunchKernelGGL(bdots_kernel<c128>, grid, dim3(256), 0, st, static_cast<const c128*>(A), lda, K, B, ldb, R,
                       N, slice, part);
  return hipGetLastError();
}

hipError_t launch_bdots32_b64(const c64* A, int64_t lda, int K, const c64* B, int64_t ldb, int R, int64_t N, c128* part,
                              int nsplit, hipStream_t st) {
  if (K <= 0 || N <= 0) return hipSuccess;
  const int64_t slice = ((N + nsplit - 1) / nsplit + kSlab - 1) / kSlab * kSlab;
  const dim3 grid((unsigned)((K + kTile - 1) / kTile), (unsigned)nsplit);
  hipLaunchKernelGGL((bdots32_kernel<c64, c64>), grid, dim3(256), 0, st, A, lda, K, B, ldb, R, N, slice, part);
  return hipGetLastError();
}

hipError_t launch_bgemm32_c64(const c64* A, int64_t lda, int64_t M, int K, const c64* C, int64_t ldc, int R,
                              double alpha, double beta, const c128* in, int64_t ldi, c128* out, int64_t ldo,
                              hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const dim3 grid((unsigned)((M + kTile - 1) / kTile));
  hipLaunchKernelGGL((bgemm32_nk_kernel<c64, c64>), grid, dim3(256), 0, st, A, lda, M, K, C, ldc, R, alpha, beta, in, ldi,
                     out, ldo);
  return hipGetLastError();
}

// out[k + c ldo] = (complex64) in[k + c ldi] for k < rows, c < cols
__global__ void to_c64_2d_kernel(const c128* __restrict__ in, int64_t ldi, int64_t rows, int cols, c64* __restrict__ out,
                                 int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= rows || c >= cols) return;
  const c128 v = in[i + (int64_t)c * ldi];
  out[i + (int64_t)c * ldo] = c64{(float)v.re, (float)v.im};
}

hipError_t launch_to_c64_2d(const c128* in, int64_t ldi, int64_t rows, int cols, c64* out, int64_t ldo, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_c64_2d_kernel, dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0, st, in, ldi,
                     rows, cols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_breduce(const c128* part, int nsplit, int K, int R, c128* out, int64_t ldo, bool accumulate,
                          c128* copy, int64_t ldc, hipStream_t st) {
  const int64_t n = (int64_t)K * R;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(breduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nsplit, K, R, out,
                     ldo, accumulate ? 1 : 0, copy, ldc);
  return hipGetLastError();
}

hipError_t launch_bgemm_nk(const void* A, bool a32, int64_t lda, int64_t M, int K, const c128* C, int64_t ldc, int R,
                           double alpha, double beta, const c128* in, int64_t ldi, c128* out, int64_t ldo,
                           hipStream_t st, bool fp32) {
  if (M <= 0) return hipSuccess;
  const dim3 grid((unsigned)((M + kTile - 1) / kTile));
  if (fp32) {
    if (a32)
      hipLaunchKernelGGL((bgemm32_nk_kernel<c64, c128>), grid, dim3(256), 0, st, static_cast<const c64*>(A), lda, M, K,
                         C, ldc, R, alpha, beta, in, ldi, out, ldo);
    else
      hipLaunchKernelGGL((bgemm32_nk_kernel<c128, c128>), grid, dim3(256), 0, st, static_cast<const c128*>(A), lda, M,
                         K, C, ldc, R, alpha, beta, in, ldi, out, ldo);
    return hipGetLastError();
  }
  if (a32)
    hipLaunchKernelGGL(bgemm_nk_kernel<c64>, grid, dim3(256), 0, st, static_cast<const c64*>(A), lda, M, K, C, ldc, R,
                       alpha, beta, in, ldi, out, ldo);
  else
    hipLaunchKernelGGL(bgemm_nk_kernel<c128>, grid, dim3(256), 0, st, static_cast<const c128*>(A), lda, M, K, C, ldc,
                       R, alpha, beta, in, ldi, out, ldo);
  return hipGetLastError();
}

hipError_t launch_chol(const c128* G, int R, bool scale, double shift, bool first, double dep_tol, c128* F, c128* Finv,
                       c128* Rtot, int32_t* dep, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, st, G, R, scale ? 1 : 0, shift, first ? 1 : 0, dep_tol, F,
                     Finv, Rtot, dep, flag);
  return hipGetLastError();
}

hipError_t launch_bhess_apply(const c128* refl, int R, int64_t rho0, int64_t rho1, c128* X, int64_t ldx, int ncols,
                              hipStream_t st) {
  if (rho1 <= rho0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(bhess_apply_kernel, dim3((unsigned)ncols), dim3(64), 0, st, refl, R, rho0, rho1, X, ldx);
  return hipGetLastError();
}

hipError_t launch_bhess_apply_rev(const c128* refl, int R, int64_t rho0, int64_t rho1, c128* X, int64_t ldx,
                                  int ncols, hipStream_t st) {
  if (rho1 <= rho0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(bhess_apply_rev_kernel, dim3((unsigned)ncols), dim3(64), 0, st, refl, R, rho0, rho1, X, ldx);
  return hipGetLastError();
}

hipError_t launch_bhess_newqr(c128* refl, int R, int64_t jR, c128* X, int64_t ldx, hipStream_t st) {
  hipLaunchKernelGGL(bhess_newqr_kernel, dim3(1), dim3(64), 0, st, refl, R, jR, X, ldx);
  return hipGetLastError();
}

hipError_t launch_bres(const c128* g, int64_t ldg, int64_t row0, int R, const double* bnorm, double* res,
                       hipStream_t st) {
  hipLaunchKernelGGL(bres_kernel, dim3((unsigned)R), dim3(64), 0, st, g, ldg, row0, R, bnorm, res);
  return hipGetLastError();
}

hipError_t launch_btrsm_diag(const c128* U, int64_t ldu, const c128* g, int64_t ldg, c128* Y, int64_t ldy, int R,
                             hipStream_t st) {
  hipLaunchKernelGGL(btrsm_diag_kernel, dim3(1), dim3(64), 0, st, U, ldu, g, ldg, Y, ldy, R);
  return hipGetLastError();
}

hipError_t launch_fill_zero_columns(c128* X, int64_t N, int R, const double* bnorm, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_columns_kernel, dim3((unsigned)((N + 255) / 256), (unsigned)R), dim3(256), 0, st, X, N, R,
                     bnorm);
  return hipGetLastError();
}

}  // namespace mfs
