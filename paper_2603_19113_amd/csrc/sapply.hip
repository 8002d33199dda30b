// Block-diagonal scattering-matrix products and elementwise helpers.
//
// y_tau = beta q_tau + S_shape(tau) t_tau for every body tau (eq. mbody1): one block per
// (body, right-hand side).  The block first sums the pair kernel's per-chunk partials for the
// body's k entries into LDS (fixed chunk order), then each thread forms rows of S t with S read
// column by column (column-major, so a column is one coalesced read across the block) and t
// broadcast from LDS.  Bodies of one shape share S, which stays resident in L2.
#include "mfs_internal.h"

namespace mfs {
namespace {

template <typename TQ, typename TS>
__global__ __launch_bounds__(256) void sapply_kernel(const int64_t* __restrict__ body_ptr,
                                                     const int32_t* __restrict__ shape_of,
                                                     const void* const* __restrict__ S_of_shape,
                                                     const Cplx<TS>* __restrict__ partial, int nchunks,
                                                     const int64_t* __restrict__ pptr, int64_t NP,
                                                     const Cplx<TQ>* __restrict__ q, TQ beta,
                                                     Cplx<TQ>* __restrict__ y, int64_t N, int R) {
  extern __shared__ unsigned char smem_raw[];
  Cplx<TS>* t = reinterpret_cast<Cplx<TS>*>(smem_raw);
  const int64_t body = blockIdx.x;
  const int r = blockIdx.y;
  const int64_t start = body_ptr[body];
  const int k = (int)(body_ptr[body + 1] - start);
  const Cplx<TS>* __restrict__ S = static_cast<const Cplx<TS>*>(S_of_shape[shape_of[body]]);
  const int64_t NPR = NP * R;
  const int64_t pstart = pptr[body];
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const int64_t idx = (int64_t)r * NP + pstart + j;
    double re = 0, im = 0;  // the symmetric pair kernel leaves hundreds of slices: add in FP64
#pragma unroll 8
    for (int c = 0; c < nchunks; ++c) {  // eight slice loads in flight per thread
      const Cplx<TS> v = partial[(int64_t)c * NPR + idx];
      re += (double)v.re;
      im += (double)v.im;
    }
    t[j] = Cplx<TS>{(TS)re, (TS)im};
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    TS ar = 0, ai = 0;
    const Cplx<TS>* col = S + i;
    for (int j = 0; j < k; ++j) {
      const Cplx<TS> s = col[(int64_t)j * k];
      const Cplx<TS> tj = t[j];
      ar = fma(s.re, tj.re, fma(-s.im, tj.im, ar));
      ai = fma(s.re, tj.im, fma(s.im, tj.re, ai));
    }
    const int64_t idx = (int64_t)r * N + start + i;
    Cplx<TQ> out;
    if (beta != TQ(0)) {
      const Cplx<TQ> qq = q[idx];
      out.re = beta * qq.re + (TQ)ar;
      out.im = beta * qq.im + (TQ)ai;
    } else {
      out.re = (TQ)ar;
      out.im = (TQ)ai;
    }
    y[idx] = out;
  }
}

template <typename TQ, typename TS>
hipError_t launch_sapply(const SceneDev& s, const void* const* S_tab, const Cplx<TS>* partial, int nchunks,
                         const Cplx<TQ>* q, TQ beta, Cplx<TQ>* y, int R, int kmax, hipStream_t st,
                         const int64_t* pptr = nullptr, int64_t NP = 0) {
  if (s.T == 0 || R == 0) return hipSuccess;
  if (!pptr) {
    pptr = s.body_ptr;
    NP = s.N;
  }
  int threads = ((kmax + 63) / 64) * 64;
  threads = threads < 64 ? 64 : (threads > 256 ? 256 : threads);
  const size_t shmem = sizeof(Cplx<TS>) * (size_t)kmax;
  hipLaunchKernelGGL((sapply_kernel<TQ, TS>), dim3((unsigned)s.T, (unsigned)R), dim3(threads), shmem, st,
                     s.body_ptr, s.shape_of, S_tab, partial, nchunks, pptr, NP, q, beta, y, s.N, R);
  return hipGetLastError();
}

// With many right-hand sides the products S_tau T_tau (k x k times k x R per body) are GEMMs and run
// on the FP32 matrix cores: the pair kernel's slices are first added in place into slice 0 (FP64
// sums, fixed order), then block (body, 64-row tile, 64-column tile) stages 32 columns of S and 32
// rows of T per step in LDS and four waves each form 16 rows x 64 columns of S T, a complex product
// as four real 16x16x4 products (the FP32 product leaves D row 4 (l / 16) + v, column l % 16 in
// register v of lane l).
template <typename TS>
__global__ void reduce_slices_kernel(Cplx<TS>* __restrict__ partial, int nchunks, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
#pragma unroll 8
  for (int c = 0; c < nchunks; ++c) {
    const Cplx<TS> v = partial[(int64_t)c * n + i];
    re += (double)v.re;
    im += (double)v.im;
  }
  partial[i] = Cplx<TS>{(TS)re, (TS)im};
}

typedef float f4s __attribute__((ext_vector_type(4)));
constexpr int kSmTile = 64, kSmSlab = 32, kSmPad = 68;

template <typename TQ>
__global__ __launch_bounds__(256) void sapply_mfma_kernel(const int64_t* __restrict__ body_ptr,
                                                          const int32_t* __restrict__ shape_of,
                                                          const void* const* __restrict__ S_of_shape,
                                                          const c64* __restrict__ t, const int64_t* __restrict__ pptr,
                                                          int64_t NP, const Cplx<TQ>* __restrict__ q, TQ beta,
                                                          Cplx<TQ>* __restrict__ y, int64_t N, int R) {
  __shared__ float Sre[kSmSlab][kSmPad], Sim[kSmSlab][kSmPad], Tre[kSmSlab][kSmPad], Tim[kSmSlab][kSmPad];
  const int64_t body = blockIdx.x;
  const int64_t start = body_ptr[body];
  const int k = (int)(body_ptr[body + 1] - start);
  const int i0 = blockIdx.y * kSmTile;
  if (i0 >= k) return;  // the whole block (uniform)
  const int r0 = blockIdx.z * kSmTile;
  const c64* __restrict__ S = static_cast<const c64*>(S_of_shape[shape_of[body]]);
  const c64* __restrict__ tb = t + pptr[body];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  f4s accR[4], accI[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) accR[c] = accI[c] = f4s{0.0f, 0.0f, 0.0f, 0.0f};
  // S tile: column j (tid / 8), rows i0 + (tid % 8) * 8 .. + 7 (contiguous: S is column-major);
  // T tile: column r (tid / 4), rows j0 + (tid % 4) * 8 .. + 7 (contiguous in j)
  const int sj = tid >> 3, si = (tid & 7) * 8;
  const int tr = tid >> 2, tj = (tid & 3) * 8;
  for (int j0 = 0; j0 < k; j0 += kSmSlab) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = i0 + si + e, j = j0 + sj;
      const c64 v = (i < k && j < k) ? S[(int64_t)j * k + i] : c64{0.0f, 0.0f};
      Sre[sj][si + e] = v.re;
      Sim[sj][si + e] = v.im;
      const int jj = j0 + tj + e, r = r0 + tr;
      const c64 u = (jj < k && r < R) ? tb[(int64_t)r * NP + jj] : c64{0.0f, 0.0f};
      Tre[tj + e][tr] = u.re;
      Tim[tj + e][tr] = u.im;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSmSlab; kk += 4) {
      const int jr = kk + (lane >> 4);
      const float ar = Sre[jr][16 * w + (lane & 15)], ai = Sim[jr][16 * w + (lane & 15)];
      float br[4], bi[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        br[c] = Tre[jr][16 * c + (lane & 15)];
        bi[c] = Tim[jr][16 * c + (lane & 15)];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        accR[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br[c], accR[c], 0, 0, 0);
        accI[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi[c], accI[c], 0, 0, 0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        accR[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi[c], accR[c], 0, 0, 0);
        accI[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br[c], accI[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int r = r0 + 16 * c + (lane & 15);
    if (r >= R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * w + 4 * (lane >> 4) + v;
      if (i >= k) continue;
      const int64_t idx = (int64_t)r * N + start + i;
      Cplx<TQ> out{(TQ)accR[c][v], (TQ)accI[c][v]};
      if (beta != TQ(0)) {
        const Cplx<TQ> qq = q[idx];
        out.re += beta * qq.re;
        out.im += beta * qq.im;
      }
      y[idx] = out;
    }
  }
}

// The matrix-core form from this many right-hand sides (FP32 S).
constexpr int kSapplyMfmaMinRhs = 16;

template <typename TQ>
hipError_t launch_sapply_mc(const SceneDev& s, c64* partial, int nchunks, const Cplx<TQ>* q, TQ beta,
                            Cplx<TQ>* y, int R, int kmax, hipStream_t st, const int64_t* pptr, int64_t NP) {
  if (s.T == 0 || R == 0) return hipSuccess;
  if (!pptr) {
    pptr = s.body_ptr;
    NP = s.N;
  }
  if (nchunks > 1) {  // the slices are scratch: add them into slice 0
    const int64_t n = NP * R;
    hipLaunchKernelGGL(reduce_slices_kernel<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partial,
                       nchunks, n);
  }
  const dim3 grid((unsigned)s.T, (unsigned)((kmax + kSmTile - 1) / kSmTile), (unsigned)((R + kSmTile - 1) / kSmTile));
  hipLaunchKernelGGL((sapply_mfma_kernel<TQ>), grid, dim3(256), 0, st, s.body_ptr, s.shape_of, s.S32,
                     static_cast<const c64*>(partial), pptr, NP, q, beta, y, s.N, R);
  return hipGetLastError();
}

// Padded layout: point ip belongs to body b = body_of_pad[ip] at offset o = ip - pad_ptr[b]; it is
// the body's point o if o < k_b, else a filler at the body centre (offset 0, charge 0).
__global__ void pad_scene_kernel(int dim, const int64_t* __restrict__ body_ptr, const int64_t* __restrict__ pad_ptr,
                                 const int32_t* __restrict__ body_of_pad, const float* __restrict__ l32, int64_t N,
                                 const float* __restrict__ lsq, int64_t NP, float* __restrict__ l32p,
                                 float* __restrict__ lsqp) {
  const int64_t ip = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ip >= NP) return;
  const int b = body_of_pad[ip];
  const int64_t o = ip - pad_ptr[b];
  const bool real = o < body_ptr[b + 1] - body_ptr[b];
  const int64_t i = body_ptr[b] + o;
  for (int d = 0; d < dim; ++d) l32p[d * NP + ip] = real ? l32[d * N + i] : 0.0f;
  lsqp[ip] = real ? lsq[i] : 0.0f;
}

__global__ void gather_pad_kernel(const int64_t* __restrict__ body_ptr, const int64_t* __restrict__ pad_ptr,
                                  const int32_t* __restrict__ body_of_pad, const c64* __restrict__ q, int64_t N,
                                  int64_t NP, c64* __restrict__ qp) {
  const int64_t ip = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (ip >= NP) return;
  const int b = body_of_pad[ip];
  const int64_t o = ip - pad_ptr[b];
  const bool real = o < body_ptr[b + 1] - body_ptr[b];
  qp[(int64_t)r * NP + ip] = real ? q[(int64_t)r * N + body_ptr[b] + o] : c64{0.0f, 0.0f};
}

__global__ void to_c64_kernel(const c128* __restrict__ in, c64* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = c64{(float)in[i].re, (float)in[i].im};
}

__global__ void plane_wave_kernel(int dim, double kappa, const double* __restrict__ x0, const double* __restrict__ x1,
                                  const double* __restrict__ x2, const double* __restrict__ dirs, int64_t N, int R,
                                  c128* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  double ph = dirs[r * dim + 0] * x0[i] + dirs[r * dim + 1] * x1[i];
  if (dim == 3) ph += dirs[r * dim + 2] * x2[i];
  double s, c;
  sincos(kappa * ph, &s, &c);
  v[(int64_t)r * N + i] = c128{-c, -s};  // v = -u_inc = -exp(i kappa d.x)
}

__global__ void pack_scene_kernel(int dim, int64_t T, const int32_t* __restrict__ shape_of,
                                  const double* __restrict__ centres, const double* __restrict__ rot,
                                  const int64_t* __restrict__ tmpl_ptr,
                                  const double* __restrict__ tmpl_pts, const int64_t* __restrict__ body_ptr,
                                  double ox, double oy, double oz, double* __restrict__ x64,
                                  float* __restrict__ x32, float* __restrict__ l32, float* __restrict__ lsq,
                                  int32_t* __restrict__ body_of, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  // body containing point i: largest tau with body_ptr[tau] <= i
  int64_t lo = 0, hi = T - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (body_ptr[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int64_t tau = lo;
  const int64_t l = i - body_ptr[tau];
  const int s = shape_of[tau];
  const double* p0 = tmpl_pts + (tmpl_ptr[s] + l) * dim;
  // body-frame offset turned with the body: p = R_tau p0 (R row-major [dim][dim]; null: identity)
  double p[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; ++d) {
    if (rot) {
      const double* Rr = rot + (tau * dim + d) * dim;
      for (int e = 0; e < dim; ++e) p[d] += Rr[e] * p0[e];
    } else {
      p[d] = p0[d];
    }
  }
  const double o[3] = {ox, oy, oz};
  float l2 = 0.0f;
  for (int d = 0; d < dim; ++d) {
    const double v = p[d] + centres[tau * dim + d];
    x64[d * N + i] = v;
    x32[d * N + i] = (float)(v - o[d]);
    const float lf = (float)p[d];
    l32[d * N + i] = lf;
    l2 = fmaf(lf, lf, l2);
  }
  lsq[i] = l2;
  body_of[i] = (int32_t)tau;
}

}  // namespace

hipError_t launch_sapply_f64(const SceneDev& s, const c128* partial, int nchunks, const c128* q, double beta,
                             c128* y, int R, int kmax, hipStream_t st) {
  return launch_sapply<double, double>(s, s.S64, partial, nchunks, q, beta, y, R, kmax, st);
}

hipError_t launch_sapply_f32(const SceneDev& s, const c64* partial, int nchunks, const c64* q, float beta, c64* y,
                             int R, int kmax, hipStream_t st, const int64_t* pptr, int64_t NP) {
  // from kSapplyMfmaMinRhs right-hand sides on the matrix cores; one slice (a caller's own t,
  // read-only) or several (scratch, reduced in place)
  if (R >= kSapplyMfmaMinRhs)
    return launch_sapply_mc<float>(s, const_cast<c64*>(partial), nchunks, q, beta, y, R, kmax, st, pptr, NP);
  return launch_sapply<float, float>(s, s.S32, partial, nchunks, q, beta, y, R, kmax, st, pptr, NP);
}

hipError_t launch_sapply_mixed(const SceneDev& s, const c64* partial, int nchunks, const c128* q, double beta,
                               c128* y, int R, int kmax, hipStream_t st, const int64_t* pptr, int64_t NP) {
  if (R >= kSapplyMfmaMinRhs)
    return launch_sapply_mc<double>(s, const_cast<c64*>(partial), nchunks, q, beta, y, R, kmax, st, pptr, NP);
  return launch_sapply<double, float>(s, s.S32, partial, nchunks, q, beta, y, R, kmax, st, pptr, NP);
}

hipError_t launch_pad_scene(const SceneDev& s, float* l32p, float* lsqp, hipStream_t st) {
  if (s.Npad == 0) return hipSuccess;
  hipLaunchKernelGGL(pad_scene_kernel, dim3((unsigned)((s.Npad + 255) / 256)), dim3(256), 0, st, s.dim, s.body_ptr,
                     s.pad_ptr, s.body_of_pad, s.l32[0], s.N, s.lsq32, s.Npad, l32p, lsqp);
  return hipGetLastError();
}

hipError_t launch_gather_pad(const SceneDev& s, const c64* q, int R, c64* qp, hipStream_t st) {
  if (s.Npad == 0 || R == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_pad_kernel, dim3((unsigned)((s.Npad + 255) / 256), (unsigned)R), dim3(256), 0, st,
                     s.body_ptr, s.pad_ptr, s.body_of_pad, q, s.N, s.Npad, qp);
  return hipGetLastError();
}

hipError_t launch_to_c64(const c128* in, c64* out, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_c64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_plane_wave(const SceneDev& s, const double* dirs_dev, int R, c128* vhat, hipStream_t st) {
  if (s.N == 0 || R == 0) return hipSuccess;
  hipLaunchKernelGGL(plane_wave_kernel, dim3((unsigned)((s.N + 255) / 256), (unsigned)R), dim3(256), 0, st, s.dim,
                     s.kappa, s.x64[0], s.x64[1], s.x64[2], dirs_dev, s.N, R, vhat);
  return hipGetLastError();
}

hipError_t launch_pack_scene(int dim, int64_t T, const int32_t* shape_of, const double* centres,
                             const double* rot, const int64_t* tmpl_ptr, const double* tmpl_pts, const int64_t* body_ptr,
                             const double* origin, double* x64_soa, float* x32_soa, float* l32_soa,
                             float* lsq, int32_t* body_of, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(pack_scene_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, dim, T, shape_of,
                     centres, rot, tmpl_ptr, tmpl_pts, body_ptr, origin[0], origin[1], origin[2], x64_soa, x32_soa,
                     l32_soa, lsq, body_of, N);
  return hipGetLastError();
}

}  // namespace mfs
