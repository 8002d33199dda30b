// Full MFS sources of each body and the field near the bodies (Sec. 4.6), FP64.
//
// After the global solve the equivalent sources of body tau represent its field only outside its
// proxy surface.  Its MFS sources are reconstructed as q_tau = A^+ v_tau - Y (G_hat q_hat)_tau with
// Y = A^+ U (the same factor as in S); A^+ is applied with the kept Householder factors of A
// (lsq.hip), the rest here:
//   * plane-wave Dirichlet data at every body's collocation points,
//   * q_mfs -= Y w_hat per (body, right-hand side),
//   * field evaluation where each (target, body) pair takes the MFS sources when the target lies
//     inside the body's proxy radius and the equivalent points otherwise.
#include <algorithm>

#include "mfs_internal.h"
#include "phi.h"

namespace mfs {
namespace {

// v[r][cptr[b] + i] = -exp(i kappa d_r . (c_b + x_i)), x_i the collocation points of b's shape.
// Body-frame point p of body b in world coordinates: c_b + R_b p (R null: identity).
__device__ __forceinline__ double placed(const double* __restrict__ centres, const double* __restrict__ rot,
                                         int dim, int64_t b, const double* p, int d) {
  double v = centres[b * dim + d];
  if (rot) {
    const double* Rr = rot + (b * dim + d) * dim;
    for (int e = 0; e < dim; ++e) v += Rr[e] * p[e];
  } else {
    v += p[d];
  }
  return v;
}

__global__ void plane_wave_colloc_kernel(int dim, double kappa, const double* __restrict__ centres,
                                         const double* __restrict__ rot, const int32_t* __restrict__ shape_of,
                                         NearTables t, const double* __restrict__ dirs, c128* __restrict__ v) {
  const int b = blockIdx.y, r = blockIdx.z;
  const int s = shape_of[b];
  const int m = t.m_of_shape[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double* x = t.colloc_of_shape[s] + (int64_t)i * dim;
  double ph = 0.0;
  for (int d = 0; d < dim; ++d) ph += dirs[r * dim + d] * placed(centres, rot, dim, b, x, d);
  double sn, cs;
  sincos(kappa * ph, &sn, &cs);
  v[(int64_t)r * t.Mtot + t.cptr[b] + i] = c128{-cs, -sn};
}

// qmfs[r][sptr[b] + i] -= sum_j Y_s(i, j) w_hat[r][body_ptr[b] + j]; one block per (body, rhs).
__global__ __launch_bounds__(256) void recon_combine_kernel(const int64_t* __restrict__ body_ptr,
                                                            const int32_t* __restrict__ shape_of, NearTables t,
                                                            const c128* __restrict__ what, int64_t N,
                                                            c128* __restrict__ qmfs) {
  extern __shared__ c128 wsh[];
  const int b = blockIdx.x, r = blockIdx.y;
  const int s = shape_of[b];
  const int64_t k0 = body_ptr[b];
  const int k = (int)(body_ptr[b + 1] - k0);
  const int n = t.n_of_shape[s];
  for (int j = threadIdx.x; j < k; j += blockDim.x) wsh[j] = what[(int64_t)r * N + k0 + j];
  __syncthreads();
  const c128* Y = t.Y_of_shape[s];
  c128* out = qmfs + (int64_t)r * t.Ntot + t.sptr[b];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < k; ++j) {
      const c128 y = Y[(int64_t)j * n + i], w = wsh[j];
      ar = fma(y.re, w.re, fma(-y.im, w.im, ar));
      ai = fma(y.re, w.im, fma(y.im, w.re, ai));
    }
    out[i].re -= ar;
    out[i].im -= ai;
  }
}

template <int DIM>
__device__ __forceinline__ void phi64(double r, double kappa, double& pr, double& pi) {
  if constexpr (DIM == 2) phi2d_f64(r, kappa, pr, pi);
  else phi3d_f64(r, kappa, pr, pi);
}

// One thread per target, a chunk of bodies per grid.y, one right-hand side per grid.z.
template <int DIM>
__global__ __launch_bounds__(256) void eval_near_kernel(double kappa, const double* __restrict__ x0,
                                                        const double* __restrict__ x1, const double* __restrict__ x2,
                                                        const double* __restrict__ centres,
                                                        const double* __restrict__ rot,
                                                        const int64_t* __restrict__ body_ptr,
                                                        const int32_t* __restrict__ shape_of, NearTables t,
                                                        const c128* __restrict__ qhat, const c128* __restrict__ qmfs,
                                                        int64_t N, const double* __restrict__ targets, int64_t M,
                                                        int64_t T, int bchunk, c128* __restrict__ partial) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.z;
  const int64_t b0 = (int64_t)blockIdx.y * bchunk;
  const int64_t b1 = b0 + bchunk < T ? b0 + bchunk : T;
  const int64_t itc = it < M ? it : M - 1;
  double x[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < DIM; ++d) x[d] = targets[itc * DIM + d];
  double ar = 0.0, ai = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    const int s = shape_of[b];
    double c[3] = {0.0, 0.0, 0.0}, dc2 = 0.0;
    for (int d = 0; d < DIM; ++d) {
      c[d] = centres[b * DIM + d];
      dc2 += (x[d] - c[d]) * (x[d] - c[d]);
    }
    if (dc2 < t.psi2_of_shape[s]) {  // inside the proxy surface: the body's own MFS sources
      const double* y = t.src_of_shape[s];
      const int n = t.n_of_shape[s];
      const c128* q = qmfs + (int64_t)r * t.Ntot + t.sptr[b];
      for (int j = 0; j < n; ++j) {
        double d2 = 0.0;
        for (int d = 0; d < DIM; ++d) {
          const double e = x[d] - placed(centres, rot, DIM, b, y + j * DIM, d);
          d2 += e * e;
        }
        double pr, pi;
        phi64<DIM>(sqrt(d2), kappa, pr, pi);
        const c128 qq = q[j];
        ar = fma(pr, qq.re, fma(-pi, qq.im, ar));
        ai = fma(pr, qq.im, fma(pi, qq.re, ai));
      }
    } else {  // outside: the equivalent points
      const int64_t j0 = body_ptr[b], j1 = body_ptr[b + 1];
      const c128* q = qhat + (int64_t)r * N;
      for (int64_t j = j0; j < j1; ++j) {
        const double e0 = x[0] - x0[j], e1 = x[1] - x1[j];
        double d2 = e0 * e0 + e1 * e1;
        if constexpr (DIM == 3) {
          const double e2 = x[2] - x2[j];
          d2 += e2 * e2;
        }
        double pr, pi;
        phi64<DIM>(sqrt(d2), kappa, pr, pi);
        const c128 qq = q[j];
        ar = fma(pr, qq.re, fma(-pi, qq.im, ar));
        ai = fma(pr, qq.im, fma(pi, qq.re, ai));
      }
    }
  }
  if (it < M) partial[((int64_t)blockIdx.y * gridDim.z + r) * M + it] = c128{ar, ai};
}

}  // namespace

hipError_t launch_plane_wave_colloc(const SceneDev& s, const NearTables& t, const double* dirs, int R, c128* v,
                                    hipStream_t st) {
  hipLaunchKernelGGL(plane_wave_colloc_kernel, dim3((unsigned)((t.mmax + 255) / 256), (unsigned)s.T, (unsigned)R),
                     dim3(256), 0, st, s.dim, s.kappa, s.centres, s.rot, s.shape_of, t, dirs, v);
  return hipGetLastError();
}

hipError_t launch_recon_combine(const SceneDev& s, const NearTables& t, const c128* what, int R, c128* qmfs,
                                hipStream_t st) {
  hipLaunchKernelGGL(recon_combine_kernel, dim3((unsigned)s.T, (unsigned)R), dim3(256),
                     sizeof(c128) * (size_t)t.kmax, st, s.body_ptr, s.shape_of, t, what, s.N, qmfs);
  return hipGetLastError();
}

int near_chunks_for(int64_t T, int64_t M) {
  const int64_t blocks = (M + 255) / 256;
  int64_t want = (2048 + blocks - 1) / std::max<int64_t>(blocks, 1);
  want = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, T), 256));
  return (int)want;
}

hipError_t launch_eval_near(const SceneDev& s, const NearTables& t, const c128* qhat, const c128* qmfs, int R,
                            const double* targets, int64_t M, c128* partial, int nchunks, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const int bchunk = (int)((s.T + nchunks - 1) / nchunks);
  dim3 grid((unsigned)((M + 255) / 256), (unsigned)nchunks, (unsigned)R);
  if (s.dim == 2)
    hipLaunchKernelGGL(eval_near_kernel<2>, grid, dim3(256), 0, st, s.kappa, s.x64[0], s.x64[1], s.x64[2], s.centres,
                       s.rot, s.body_ptr, s.shape_of, t, qhat, qmfs, s.N, targets, M, s.T, bchunk, partial);
  else
    hipLaunchKernelGGL(eval_near_kernel<3>, grid, dim3(256), 0, st, s.kappa, s.x64[0], s.x64[1], s.x64[2], s.centres,
                       s.rot, s.body_ptr, s.shape_of, t, qhat, qmfs, s.N, targets, M, s.T, bchunk, partial);
  return hipGetLastError();
}

}  // namespace mfs
