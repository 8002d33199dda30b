// FP64 GMRES building blocks (Saad & Schultz; the paper solves eq. mbody2 with GMRES, Sec. 2.3).
//
// Every right-hand side r has its own Arnoldi process; vectors are [R][N] complex128 and the
// basis is V[(m+1)][R][N].  Orthogonalisation is classical Gram-Schmidt applied twice (CGS2):
// one pass computes all j+1 inner products at once, which reads each basis vector once.
// Reductions are two-stage with a fixed order (per-block partial sums, then one wave per value),
// so results are reproducible run to run.  The Hessenberg column update, Givens rotations and
// the residual estimate run on the device; the host only reads how many columns are still active.
#include <algorithm>

#include "mfs_internal.h"

namespace mfs {
namespace {

constexpr int kThreads = 256;
constexpr int kElems = 4;   // vector elements per thread in the dot kernels
constexpr int kElems32 = 2; // the inner products with a complex64 basis
constexpr int kGroup = 16;  // basis vectors per dot-product block

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// part[r][i][blk] = sum over the block's elements of conj(V_i[r][n]) w[r][n].
// grid = (vector chunks, groups of kGroup basis vectors, right-hand sides): each block keeps its
// chunk of w in registers and reads kGroup basis-vector chunks once.
template <typename VT, int ELEMS = kElems>
__global__ __launch_bounds__(kThreads) void dots_kernel(const VT* __restrict__ V, const c128* __restrict__ w,
                                                        int64_t N, int R, int jcount_h, int nblk,
                                                        double* __restrict__ part, const int32_t* __restrict__ flag,
                                                        const int32_t* __restrict__ jdev) {
  __shared__ double red[kThreads / 64][2 * kGroup];
  const int r = blockIdx.z;
  if (flag && !flag[r]) return;
  const int jcount = jdev ? *jdev + 1 : jcount_h;
  const int i0 = blockIdx.y * kGroup;
  if (i0 >= jcount) return;  // graph replays size the grid for the largest step of their bucket
  const int64_t base = (int64_t)blockIdx.x * (kThreads * ELEMS);
  c128 wl[ELEMS];
#pragma unroll
  for (int e = 0; e < ELEMS; ++e) {
    const int64_t n = base + e * kThreads + threadIdx.x;
    wl[e] = n < N ? w[(int64_t)r * N + n] : c128{0.0, 0.0};
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // v[g] = real part and v[kGroup + g] = imaginary part of conj(V_{i0+g}) . w over this lane's elements
  double v[2 * kGroup];
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    double ar = 0.0, ai = 0.0;
    const int i = i0 + g;
    if (i < jcount) {
      const VT* Vi = V + ((int64_t)i * R + r) * N;
#pragma unroll
      for (int e = 0; e < ELEMS; ++e) {
        const int64_t n = base + e * kThreads + threadIdx.x;
        if (n < N) {
          const VT xv = Vi[n];
          const double xr = xv.re, xi = xv.im;
          ar = fma(xr, wl[e].re, fma(xi, wl[e].im, ar));   // conj(v) * w
          ai = fma(xr, wl[e].im, fma(-xi, wl[e].re, ai));
        }
      }
    }
    v[g] = ar;
    v[kGroup + g] = ai;
  }
  // Sum the 32 values over the wave by recursive halving: at distance d a lane keeps one half of
  // its values and adds its partner's copy of that half, so 16 + 8 + 4 + 2 + 1 + 1 = 32 shuffles
  // replace 6 per value.  Lanes 2t and 2t + 1 end with the total of value t.
#pragma unroll
  for (int half = kGroup, d = 32; half >= 1; half >>= 1, d >>= 1) {
    const bool up = (lane & d) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const double a = v[k], b = v[k + half];
      const double send = up ? a : b;
      const double keep = up ? b : a;
      v[k] = keep + __shfl_xor(send, d, 64);
    }
  }
  v[0] += __shfl_xor(v[0], 1, 64);
  if ((lane & 1) == 0) red[wave][lane >> 1] = v[0];
  __syncthreads();
  if (threadIdx.x < 2 * kGroup) {
    const int t = threadIdx.x;
    const int g = t % kGroup, c = t / kGroup;
    const int i = i0 + g;
    if (i < jcount) {
      double sum = 0.0;
      for (int wv = 0; wv < kThreads / 64; ++wv) sum += red[wv][t];
      part[(((int64_t)r * jcount + i) * nblk + blockIdx.x) * 2 + c] = sum;
    }
  }
}

// out[r][i] = sum_blk part[r][i][blk] (+ add[r][i] if add != null); one wave per (i, r).
__global__ void dots_reduce_kernel(const double* __restrict__ part, int jcount_h, int nblk, int R, int ld,
                                   c128* __restrict__ out, const c128* __restrict__ add,
                                   const int32_t* __restrict__ flag, const int32_t* __restrict__ jdev) {
  const int i = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int jcount = jdev ? *jdev + 1 : jcount_h;
  if (i >= jcount) return;
  if (flag && !flag[r]) {
    if (lane == 0) out[(int64_t)r * ld + i] = c128{0.0, 0.0};
    return;
  }
  double sr = 0.0, si = 0.0;
  for (int b = lane; b < nblk; b += 64) {
    const int64_t o = (((int64_t)r * jcount + i) * nblk + b) * 2;
    sr += part[o];
    si += part[o + 1];
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    c128 v{sr, si};
    if (add) {
      v.re += add[(int64_t)r * ld + i].re;
      v.im += add[(int64_t)r * ld + i].im;
    }
    out[(int64_t)r * ld + i] = v;
  }
}

// w[r][n] -= sum_{i<jcount} h[r][i] V_i[r][n]
template <typename VT>
__global__ __launch_bounds__(kThreads) void basis_axpy_kernel(const VT* __restrict__ V, const c128* __restrict__ h,
                                                              int ld, int64_t N, int R, int jcount_h,
                                                              c128* __restrict__ w, const int32_t* __restrict__ flag,
                                                              const int32_t* __restrict__ jdev) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= N || (flag && !flag[r])) return;
  const int jcount = jdev ? *jdev + 1 : jcount_h;
  // h is read with wave-uniform addresses (scalar loads); eight basis loads are kept in flight
  double ar = 0.0, ai = 0.0;
  const c128* hr = h + (int64_t)r * ld;
  const VT* Vn = V + (int64_t)r * N + n;
  const int64_t stride = (int64_t)R * N;
#pragma unroll 8
  for (int i = 0; i < jcount; ++i) {
    const c128 hi = hr[i];
    const VT vv = Vn[i * stride];
    const double vr = vv.re, vi = vv.im;
    ar = fma(hi.re, vr, fma(-hi.im, vi, ar));
    ai = fma(hi.re, vi, fma(hi.im, vr, ai));
  }
  c128 x = w[(int64_t)r * N + n];
  x.re -= ar;
  x.im -= ai;
  w[(int64_t)r * N + n] = x;
}

// part[r][blk] = sum |v|^2 over the block's elements
__global__ __launch_bounds__(kThreads) void norm_partial_kernel(const c128* __restrict__ v, int64_t N, int nblk,
                                                                double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int r = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * (kThreads * kElems);
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < kElems; ++e) {
    const int64_t n = base + e * kThreads + threadIdx.x;
    if (n < N) {
      const c128 x = v[(int64_t)r * N + n];
      s = fma(x.re, x.re, fma(x.im, x.im, s));
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int wv = 0; wv < kThreads / 64; ++wv) t += red[wv];
    part[(int64_t)r * nblk + blockIdx.x] = t;
  }
}

__global__ void norm_reduce_kernel(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  const int r = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += part[(int64_t)r * nblk + b];
  s = wave_sum(s);
  if (lane == 0) out[r] = sqrt(s);
}

// Second Gram-Schmidt pass only where the first one cancelled: reorthogonalise when
// ||w'||^2 = ||w||^2 - sum |h_i|^2 falls below eta^2 ||w||^2 (the test of Daniel, Gragg, Kaufman
// and Stewart; eta2 = eta^2 is an argument).  One block per right-hand side; the sum is reduced in
// a fixed order.
__global__ __launch_bounds__(256) void reorth_decide_kernel(int jcount_h, int R, int ld, const c128* __restrict__ h,
                                                            const double* __restrict__ wn2,
                                                            int32_t* __restrict__ flag, int32_t* __restrict__ count,
                                                            double eta2, double* __restrict__ ratio_log, int m,
                                                            const int32_t* __restrict__ jdev) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (r >= R) return;
  const int jcount = jdev ? *jdev + 1 : jcount_h;
  double sum = 0.0;
  for (int i = threadIdx.x; i < jcount; i += blockDim.x) {
    const c128 v = h[(int64_t)r * ld + i];
    sum += v.re * v.re + v.im * v.im;
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double ssum = red[0] + red[1] + red[2] + red[3];
  const double w2 = wn2[r] * wn2[r];
  const int f = (w2 - ssum) < eta2 * w2 ? 1 : 0;
  flag[r] = f;
  count[r] += f;
  if (ratio_log) ratio_log[(int64_t)r * 2 * m + jcount - 1] = w2 > 0.0 ? sqrt(fmax(w2 - ssum, 0.0) / w2) : 0.0;
}

// Start of a cycle: V_0 = r0 / beta, g = (beta, 0, ...).  Columns with beta == 0 stay inactive.
template <typename VT>
__global__ void start_scale_kernel(const c128* __restrict__ r0, const double* __restrict__ beta, int64_t N, int R,
                                   VT* __restrict__ V0) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= N) return;
  const double b = beta[r];
  const double s = b > 0.0 ? 1.0 / b : 0.0;
  const c128 x = r0[(int64_t)r * N + n];
  V0[(int64_t)r * N + n] = VT{(decltype(VT::re))(x.re * s), (decltype(VT::re))(x.im * s)};
}

__global__ void start_state_kernel(const double* __restrict__ beta, const double* __restrict__ bnorm,
                                   int32_t* __restrict__ active, int32_t* __restrict__ jlen, c128* __restrict__ g,
                                   double* __restrict__ res, int m, int R, int32_t* __restrict__ jdev,
                                   double* __restrict__ tol_dev, double tol) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0 && jdev) {
    *jdev = 0;
    *tol_dev = tol;
  }
  if (r >= R) return;
  jlen[r] = 0;
  g[(int64_t)r * (m + 1)] = c128{beta[r], 0.0};
  const double bn = bnorm[r];
  res[r] = bn > 0.0 ? beta[r] / bn : 0.0;
  active[r] = (beta[r] > 0.0 && active[r] != 0) ? 1 : 0;
}

// Column j of H from the Gram-Schmidt coefficients and ||w||, previous rotations, new rotation,
// residual estimate.  The Arnoldi vectors come from w = K v_j for the operator shift I + K, so the
// shift is added to the diagonal entry.  One block per right-hand side.
//
// Applying rotations 0..j-1 to the new column b is a chain: with carry_0 = b_0,
//   H(i, j) = conj(c_i) carry_i + conj(s_i) b_{i+1},   carry_{i+1} = -s_i carry_i + c_i b_{i+1},
// a first-order linear recurrence in the carry.  Each thread composes the affine maps of one
// contiguous segment of rotations, a scan over the segments gives every segment its incoming carry,
// and the segments are then replayed in parallel.  |s_i| <= 1, so the composed maps stay bounded.
constexpr int kGivensThreads = 256;

__device__ __forceinline__ c128 cmul(c128 a, c128 b) { return c128{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 cadd(c128 a, c128 b) { return c128{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c128 cconj(c128 a) { return c128{a.re, -a.im}; }

__global__ __launch_bounds__(kGivensThreads) void givens_kernel(int j_h, int m, int R, double shift,
                                                               const c128* __restrict__ hcol,
                                                               const c128* __restrict__ h2,
                                                               const double* __restrict__ hnorm, c128* __restrict__ H,
                                                               c128* __restrict__ cs, c128* __restrict__ sn,
                                                               c128* __restrict__ g, double* __restrict__ res,
                                                               const double* __restrict__ bnorm, double tol_h,
                                                               int32_t* __restrict__ active, int32_t* __restrict__ jlen,
                                                               const int32_t* __restrict__ jdev,
                                                               const double* __restrict__ tol_dev) {
  __shared__ c128 segA[kGivensThreads], segB[kGivensThreads];
  __shared__ c128 carry_in[kGivensThreads + 1];
  const int r = blockIdx.x;
  if (r >= R || !active[r]) return;  // uniform over the block
  const int j = jdev ? *jdev : j_h;
  const double tol = jdev ? *tol_dev : tol_h;
  const int tid = threadIdx.x;
  c128* Hc = H + ((int64_t)r * m + j) * (m + 1);
  const c128* hc1 = hcol + (int64_t)r * (m + 1);
  const c128* hc2 = h2 + (int64_t)r * (m + 1);
  const c128* c = cs + (int64_t)r * m;
  const c128* s = sn + (int64_t)r * m;
  // b_i = hcol_i + h2_i (+ shift on the diagonal)
  auto bval = [&](int i) {
    c128 v = cadd(hc1[i], hc2[i]);
    if (i == j) v.re += shift;  // H(shift I + K) = H(K) + shift I
    return v;
  };
  // segment of rotations [i0, i1) for this thread
  const int per = (j + kGivensThreads - 1) / kGivensThreads;
  const int i0 = min(j, tid * per), i1 = min(j, i0 + per);
  // compose carry -> A carry + B over the segment
  c128 A{1.0, 0.0}, B{0.0, 0.0};
  for (int i = i0; i < i1; ++i) {
    const c128 ms{-s[i].re, -s[i].im};
    const c128 cb = cmul(c[i], bval(i + 1));
    A = cmul(ms, A);
    B = cadd(cmul(ms, B), cb);
  }
  segA[tid] = A;
  segB[tid] = B;
  __syncthreads();
  if (tid == 0) {  // incoming carry of every segment (256 compositions, in order)
    c128 cr = bval(0);
    for (int t = 0; t < kGivensThreads; ++t) {
      carry_in[t] = cr;
      cr = cadd(cmul(segA[t], cr), segB[t]);
    }
    carry_in[kGivensThreads] = cr;  // carry_j
  }
  __syncthreads();
  c128 cr = carry_in[tid];
  for (int i = i0; i < i1; ++i) {
    const c128 b = bval(i + 1);
    Hc[i] = cadd(cmul(cconj(c[i]), cr), cmul(cconj(s[i]), b));
    cr = cadd(cmul(c128{-s[i].re, -s[i].im}, cr), cmul(c[i], b));
  }
  if (tid != 0) return;
  // new rotation on (carry_j, ||w||)
  const c128 a = carry_in[kGivensThreads];
  const c128 bb{hnorm[r], 0.0};
  const double den = hypot(hypot(a.re, a.im), bb.re);
  c128 cj{1.0, 0.0}, sj{0.0, 0.0};
  if (den > 0.0) {
    cj = c128{a.re / den, a.im / den};
    sj = c128{bb.re / den, bb.im / den};
  }
  cs[(int64_t)r * m + j] = cj;
  sn[(int64_t)r * m + j] = sj;
  Hc[j] = c128{den, 0.0};
  Hc[j + 1] = c128{0.0, 0.0};
  c128* gr = g + (int64_t)r * (m + 1);
  const c128 gj = gr[j];
  gr[j + 1] = c128{-(sj.re * gj.re - sj.im * gj.im), -(sj.re * gj.im + sj.im * gj.re)};
  gr[j] = c128{cj.re * gj.re + cj.im * gj.im, cj.re * gj.im - cj.im * gj.re};
  const double bn = bnorm[r];
  const double e = hypot(gr[j + 1].re, gr[j + 1].im);
  res[r] = bn > 0.0 ? e / bn : 0.0;
  jlen[r] = j + 1;
  // converged, or breakdown (the Krylov space is invariant: the solution is exact in it)
  if (res[r] <= tol || !(hnorm[r] > 1e-300)) active[r] = 0;
}

// V_{j+1} = w / ||w||.
template <typename VT>
__global__ void scale_next_kernel(const c128* __restrict__ w, const double* __restrict__ hnorm, int64_t N, int R,
                                  VT* __restrict__ V, int j_h, const int32_t* __restrict__ jdev) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= N) return;
  const int j = jdev ? *jdev : j_h;
  VT* Vn = V + (int64_t)(j + 1) * R * N;
  const double h = hnorm[r];
  const double s = h > 1e-300 ? 1.0 / h : 0.0;
  const c128 x = w[(int64_t)r * N + n];
  Vn[(int64_t)r * N + n] = VT{(decltype(VT::re))(x.re * s), (decltype(VT::re))(x.im * s)};
}

// End of a replayed step: the next replay works on step j + 1.
__global__ void step_advance_kernel(int32_t* __restrict__ jdev) {
  if (threadIdx.x == 0) *jdev += 1;
}

// y = H(0:len,0:len)^{-1} g(0:len), column-oriented back substitution; one block per right-hand
// side: y_i = g_i / H_ii, then g_t -= H_ti y_i for t < i in parallel.  g is consumed.
__global__ __launch_bounds__(1024) void hess_solve_kernel(int m, int R, const c128* __restrict__ H, c128* __restrict__ g,
                                                          const int32_t* __restrict__ jlen, c128* __restrict__ y,
                                                          int ylen) {
  __shared__ c128 yi_sh;
  const int r = blockIdx.x;
  const int len = jlen[r];
  c128* gr = g + (int64_t)r * (m + 1);
  c128* yr = y + (int64_t)r * m;
  for (int i = len - 1; i >= 0; --i) {
    const c128* Hc = H + ((int64_t)r * m + i) * (m + 1);
    if (threadIdx.x == 0) {
      const c128 d = Hc[i];
      const double dd = d.re * d.re + d.im * d.im;
      const c128 acc = gr[i];
      const c128 v = dd > 0.0 ? c128{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd}
                              : c128{0.0, 0.0};
      yr[i] = v;
      yi_sh = v;
    }
    __syncthreads();
    const c128 v = yi_sh;
    for (int t = threadIdx.x; t < i; t += blockDim.x) {
      const c128 hh = Hc[t];
      gr[t].re -= hh.re * v.re - hh.im * v.im;
      gr[t].im -= hh.re * v.im + hh.im * v.re;
    }
    __syncthreads();
  }
  for (int i = len + threadIdx.x; i < ylen; i += blockDim.x) yr[i] = c128{0.0, 0.0};
}

// Deflation in coefficient space for column r, which kept kold[r] + 1 <= o vectors:
// h[r][0..or) -= q[r] (q[r]^H h[r][0..or)) with or = kold[r] + 1 and q of unit norm, and the
// coefficients on the slots or..o-1 (vectors of steps after the column had converged) are zeroed.
// A column with keep[r] == 0 gets all o coefficients zeroed.  One block per right-hand side; the
// inner product is reduced in a fixed order.
__global__ __launch_bounds__(256) void deflate_coeffs_kernel(const c128* __restrict__ q, int o,
                                                             const int32_t* __restrict__ kold, c128* __restrict__ h,
                                                             int ld, const int32_t* __restrict__ flag,
                                                             const int32_t* __restrict__ keep) {
  __shared__ double red[2][4];
  const int r = blockIdx.x;
  if (flag && !flag[r]) return;
  const c128* qr = q + (int64_t)r * ld;
  c128* hr = h + (int64_t)r * ld;
  if (keep && !keep[r]) {
    for (int i = threadIdx.x; i < o; i += blockDim.x) hr[i] = c128{0.0, 0.0};
    return;
  }
  const int orr = min(o, kold[r] + 1);
  for (int i = orr + threadIdx.x; i < o; i += blockDim.x) hr[i] = c128{0.0, 0.0};
  double sr = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < orr; i += blockDim.x) {  // conj(q_i) h_i
    const c128 a = qr[i], b = hr[i];
    sr += a.re * b.re + a.im * b.im;
    si += a.re * b.im - a.im * b.re;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  const double tr = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const double ti = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  for (int i = threadIdx.x; i < orr; i += blockDim.x) {
    const c128 a = qr[i];
    hr[i].re -= a.re * tr - a.im * ti;
    hr[i].im -= a.re * ti + a.im * tr;
  }
}

// Rotation i of a process acts on entries (i, i+1) as G_i = [[conj(c), conj(s)], [-s, c]] (the
// Givens kernel's convention); G = G_{k-1} ... G_0 takes the Hessenberg matrix to triangular form.
// q = G^H e_k, the unit vector orthogonal to the Hessenberg matrix's range, and e <- G e.  One
// thread per right-hand side: a chain of k dependent rotations, run once per correction solve.
__global__ void givens_last_column_kernel(const c128* __restrict__ cs, const c128* __restrict__ sn, int m, int R,
                                          const int32_t* __restrict__ koldv, c128* __restrict__ q) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int kold = koldv[r];
  const c128* c = cs + (int64_t)r * m;
  const c128* s = sn + (int64_t)r * m;
  c128* qr = q + (int64_t)r * (m + 1);
  for (int i = 0; i < kold; ++i) qr[i] = c128{0.0, 0.0};
  qr[kold] = c128{1.0, 0.0};
  for (int i = kold - 1; i >= 0; --i) {  // (x_i, x_{i+1}) <- (c x_i - conj(s) x_{i+1}, s x_i + conj(c) x_{i+1})
    const c128 a = qr[i], b = qr[i + 1];
    const c128 ci = c[i], si = s[i];
    qr[i] = c128{ci.re * a.re - ci.im * a.im - (si.re * b.re + si.im * b.im),
                 ci.re * a.im + ci.im * a.re - (si.re * b.im - si.im * b.re)};
    qr[i + 1] = c128{si.re * a.re - si.im * a.im + (ci.re * b.re + ci.im * b.im),
                     si.re * a.im + si.im * a.re + (ci.re * b.im - ci.im * b.re)};
  }
}

__global__ void givens_apply_kernel(const c128* __restrict__ cs, const c128* __restrict__ sn, int m, int R,
                                    const int32_t* __restrict__ koldv, c128* __restrict__ e) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int kold = koldv[r];
  const c128* c = cs + (int64_t)r * m;
  const c128* s = sn + (int64_t)r * m;
  c128* er = e + (int64_t)r * (m + 1);
  c128 carry = er[0];
  for (int i = 0; i < kold; ++i) {  // (x_i, x_{i+1}) <- (conj(c) x_i + conj(s) x_{i+1}, -s x_i + c x_{i+1})
    const c128 b = er[i + 1];
    const c128 ci = c[i], si = s[i];
    er[i] = c128{ci.re * carry.re + ci.im * carry.im + si.re * b.re + si.im * b.im,
                 ci.re * carry.im - ci.im * carry.re + si.re * b.im - si.im * b.re};
    carry = c128{-(si.re * carry.re - si.im * carry.im) + ci.re * b.re - ci.im * b.im,
                 -(si.re * carry.im + si.im * carry.re) + ci.re * b.im + ci.im * b.re};
  }
  er[kold] = carry;
}

// x[r][n] += sum_{i<len_r} y[r][i] V_i[r][n]
template <typename VT>
__global__ __launch_bounds__(kThreads) void update_x_kernel(const VT* __restrict__ V, const c128* __restrict__ y,
                                                            const int32_t* __restrict__ jlen, int m, int64_t N, int R,
                                                            c128* __restrict__ x) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= N) return;
  const int len = jlen[r];
  double ar = 0.0, ai = 0.0;
#pragma unroll 8
  for (int i = 0; i < len; ++i) {
    const c128 yi = y[(int64_t)r * m + i];
    const VT vv = V[((int64_t)i * R + r) * N + n];
    const double vr = vv.re, vi = vv.im;
    ar = fma(yi.re, vr, fma(-yi.im, vi, ar));
    ai = fma(yi.re, vi, fma(yi.im, vr, ai));
  }
  c128 xx = x[(int64_t)r * N + n];
  xx.re += ar;
  xx.im += ai;
  x[(int64_t)r * N + n] = xx;
}

__global__ void axpby_kernel(const c128* __restrict__ a, const c128* __restrict__ b, c128* __restrict__ out,
                             double alpha, double beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const c128 u = a[i], v = b[i];
  out[i] = c128{alpha * u.re + beta * v.re, alpha * u.im + beta * v.im};
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_norms(const c128* v, int64_t N, int R, double* part, int nblk, double* out_norm, hipStream_t st) {
  hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk, R), dim3(kThreads), 0, st, v, N, nblk, part);
  hipLaunchKernelGGL(norm_reduce_kernel, dim3(R), dim3(64), 0, st, part, nblk, out_norm);
  return hipGetLastError();
}

// Basis vector `slot` of process k, and the per-column arrays shifted to the process's first index.
template <typename VT>
inline VT* slot_ptr(const KrylovDev& k, int slot) {
  return static_cast<VT*>(k.V) + (int64_t)slot * k.R * k.N;
}

hipError_t launch_start_cycle(KrylovDev k, const c128* r0, hipStream_t st) {
  hipError_t e = launch_norms(r0, k.N, k.R, k.part, k.nblk, k.beta, st);
  if (e != hipSuccess) return e;
  if (k.v32)
    hipLaunchKernelGGL(start_scale_kernel<c64>, dim3(blocks_for(k.N, 256), k.R), dim3(256), 0, st, r0, k.beta, k.N,
                       k.R, slot_ptr<c64>(k, k.joff));
  else
    hipLaunchKernelGGL(start_scale_kernel<c128>, dim3(blocks_for(k.N, 256), k.R), dim3(256), 0, st, r0, k.beta, k.N,
                       k.R, slot_ptr<c128>(k, k.joff));
  hipLaunchKernelGGL(start_state_kernel, dim3(blocks_for(k.R, 64)), dim3(64), 0, st, k.beta, k.bnorm, k.active,
                     k.jlen, k.g + k.joff, k.res, k.m, k.R, k.jdev, k.tol_dev, k.tol);
  return hipGetLastError();
}

// Gram-Schmidt: hcol = V^H w; w -= V hcol; then, where the first pass cancelled, h2 = V^H w;
// w -= V h2 (the H column is hcol + h2, summed in the Givens kernel).
hipError_t launch_arnoldi_orth(KrylovDev k, int j, c128* w, hipStream_t st) {
  if (k.joff != 0 && k.jdev) return hipErrorInvalidValue;  // offset processes launch eagerly
  // With a device step counter (graph replay) the grids cover the largest step of j's bucket and
  // the kernels read the actual step from k.jdev.
  const int jc = k.jdev ? std::min(k.m, (j / kStepBucket + 1) * kStepBucket) : k.joff + j + 1;
  const int ld = k.m + 1;
  hipError_t e = launch_norms(w, k.N, k.R, k.part, k.nblk, k.wn, st);
  if (e != hipSuccess) return e;
  for (int pass = 0; pass < 2; ++pass) {
    c128* h = pass == 0 ? k.hcol : k.h2;
    const int32_t* flag = pass == 0 ? nullptr : k.reorth;
    if (pass == 1)
      hipLaunchKernelGGL(reorth_decide_kernel, dim3(k.R), dim3(256), 0, st, jc, k.R, ld, k.hcol, k.wn,
                         k.reorth, k.n_reorth, k.reorth_eta * k.reorth_eta, k.ratio_log, k.m,
                         (const int32_t*)k.jdev);
    // a complex64 basis: half the elements per thread and twice the blocks
    const int nb = k.v32 ? (int)((k.N + kThreads * kElems32 - 1) / (kThreads * kElems32)) : k.nblk;
    const dim3 dgrid(nb, (jc + kGroup - 1) / kGroup, k.R);
    if (k.v32)
      hipLaunchKernelGGL((dots_kernel<c64, kElems32>), dgrid, dim3(kThreads), 0, st, static_cast<const c64*>(k.V), w,
                         k.N, k.R, jc, nb, k.part, flag, (const int32_t*)k.jdev);
    else
      hipLaunchKernelGGL(dots_kernel<c128>, dgrid, dim3(kThreads), 0, st, static_cast<const c128*>(k.V), w, k.N,
                         k.R, jc, nb, k.part, flag, (const int32_t*)k.jdev);
    hipLaunchKernelGGL(dots_reduce_kernel, dim3(jc, k.R), dim3(64), 0, st, k.part, jc, nb, k.R, ld, h,
                       (const c128*)nullptr, flag, (const int32_t*)k.jdev);
    if (k.qdef)
      hipLaunchKernelGGL(deflate_coeffs_kernel, dim3(k.R), dim3(256), 0, st, k.qdef, k.joff,
                         (const int32_t*)k.kold, h, ld, flag, (const int32_t*)nullptr);
    const dim3 agrid(blocks_for(k.N, kThreads), k.R);
    if (k.v32)
      hipLaunchKernelGGL(basis_axpy_kernel<c64>, agrid, dim3(kThreads), 0, st, static_cast<const c64*>(k.V), h, ld,
                         k.N, k.R, jc, w, flag, (const int32_t*)k.jdev);
    else
      hipLaunchKernelGGL(basis_axpy_kernel<c128>, agrid, dim3(kThreads), 0, st, static_cast<const c128*>(k.V), h, ld,
                         k.N, k.R, jc, w, flag, (const int32_t*)k.jdev);
  }
  return hipGetLastError();
}

// ||w|| -> H(j+1, j); rotations; residual estimate; V_{j+1} = w / ||w||.
hipError_t launch_arnoldi_finish(KrylovDev k, int j, c128* w, double tol, hipStream_t st) {
  hipError_t e = launch_norms(w, k.N, k.R, k.part, k.nblk, k.hnorm, st);
  if (e != hipSuccess) return e;
  const int o = k.joff;
  hipLaunchKernelGGL(givens_kernel, dim3(k.R), dim3(kGivensThreads), 0, st, j, k.m, k.R, 1.0, k.hcol + o, k.h2 + o,
                     k.hnorm, k.H + (int64_t)o * (k.m + 1), k.cs + o, k.sn + o, k.g + o, k.res, k.bnorm, tol, k.active,
                     k.jlen, (const int32_t*)k.jdev, (const double*)k.tol_dev);
  if (k.v32)
    hipLaunchKernelGGL(scale_next_kernel<c64>, dim3(blocks_for(k.N, 256), k.R), dim3(256), 0, st, w, k.hnorm, k.N,
                       k.R, slot_ptr<c64>(k, o), j, (const int32_t*)k.jdev);
  else
    hipLaunchKernelGGL(scale_next_kernel<c128>, dim3(blocks_for(k.N, 256), k.R), dim3(256), 0, st, w, k.hnorm, k.N,
                       k.R, slot_ptr<c128>(k, o), j, (const int32_t*)k.jdev);
  if (k.jdev) hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, st, k.jdev);
  return hipGetLastError();
}

// y = H^{-1} g per column, then x += V y.
hipError_t launch_gmres_update_x(KrylovDev k, c128* x, hipStream_t st) {
  const int o = k.joff;
  hipLaunchKernelGGL(hess_solve_kernel, dim3(k.R), dim3(1024), 0, st, k.m, k.R, k.H + (int64_t)o * (k.m + 1),
                     k.g + o, k.jlen, k.y + o, k.m - o);
  return launch_update_from_y(k, x, st);
}

hipError_t launch_update_from_y(KrylovDev k, c128* x, hipStream_t st) {
  const int o = k.joff;
  if (k.v32)
    hipLaunchKernelGGL(update_x_kernel<c64>, dim3(blocks_for(k.N, kThreads), k.R), dim3(kThreads), 0, st,
                       slot_ptr<c64>(k, o), k.y + o, k.jlen, k.m, k.N, k.R, x);
  else
    hipLaunchKernelGGL(update_x_kernel<c128>, dim3(blocks_for(k.N, kThreads), k.R), dim3(kThreads), 0, st,
                       slot_ptr<c128>(k, o), k.y + o, k.jlen, k.m, k.N, k.R, x);
  return hipGetLastError();
}

hipError_t launch_basis_dots(KrylovDev k, const c128* w, int count, c128* out, hipStream_t st) {
  if (count < 1 || count > k.m + 1) return hipErrorInvalidValue;
  const int ld = k.m + 1;
  const int nb = k.v32 ? (int)((k.N + kThreads * kElems32 - 1) / (kThreads * kElems32)) : k.nblk;
  const dim3 dgrid(nb, (count + kGroup - 1) / kGroup, k.R);
  if (k.v32)
    hipLaunchKernelGGL((dots_kernel<c64, kElems32>), dgrid, dim3(kThreads), 0, st, static_cast<const c64*>(k.V), w,
                       k.N, k.R, count, nb, k.part, (const int32_t*)nullptr, (const int32_t*)nullptr);
  else
    hipLaunchKernelGGL(dots_kernel<c128>, dgrid, dim3(kThreads), 0, st, static_cast<const c128*>(k.V), w, k.N, k.R,
                       count, nb, k.part, (const int32_t*)nullptr, (const int32_t*)nullptr);
  hipLaunchKernelGGL(dots_reduce_kernel, dim3(count, k.R), dim3(64), 0, st, k.part, count, nb, k.R, ld, out,
                     (const c128*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr);
  return hipGetLastError();
}

hipError_t launch_basis_axpy(KrylovDev k, const c128* h, int count, c128* w, hipStream_t st) {
  if (count < 1 || count > k.m + 1) return hipErrorInvalidValue;
  const dim3 agrid(blocks_for(k.N, kThreads), k.R);
  if (k.v32)
    hipLaunchKernelGGL(basis_axpy_kernel<c64>, agrid, dim3(kThreads), 0, st, static_cast<const c64*>(k.V), h, k.m + 1,
                       k.N, k.R, count, w, (const int32_t*)nullptr, (const int32_t*)nullptr);
  else
    hipLaunchKernelGGL(basis_axpy_kernel<c128>, agrid, dim3(kThreads), 0, st, static_cast<const c128*>(k.V), h,
                       k.m + 1, k.N, k.R, count, w, (const int32_t*)nullptr, (const int32_t*)nullptr);
  return hipGetLastError();
}

hipError_t launch_givens_last_column(KrylovDev k, const int32_t* kold, c128* q, hipStream_t st) {
  hipLaunchKernelGGL(givens_last_column_kernel, dim3(blocks_for(k.R, 64)), dim3(64), 0, st, k.cs, k.sn, k.m, k.R,
                     kold, q);
  return hipGetLastError();
}

hipError_t launch_givens_apply(KrylovDev k, const int32_t* kold, c128* e, hipStream_t st) {
  hipLaunchKernelGGL(givens_apply_kernel, dim3(blocks_for(k.R, 64)), dim3(64), 0, st, k.cs, k.sn, k.m, k.R, kold, e);
  return hipGetLastError();
}

hipError_t launch_deflate_coeffs(const c128* q, int o, const int32_t* kold, c128* h, int R, int ld,
                                 const int32_t* keep, hipStream_t st) {
  if (o < 1 || o > ld) return hipErrorInvalidValue;
  hipLaunchKernelGGL(deflate_coeffs_kernel, dim3(R), dim3(256), 0, st, q, o, kold, h, ld, (const int32_t*)nullptr,
                     keep);
  return hipGetLastError();
}

hipError_t launch_axpby(const c128* a, const c128* b, c128* out, double alpha, double beta, int64_t n,
                        hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, out, alpha, beta, n);
  return hipGetLastError();
}

int krylov_nblk(int64_t N) { return (int)((N + kThreads * kElems - 1) / (kThreads * kElems)); }
int krylov_part_blocks(int64_t N) {
  return std::max(krylov_nblk(N), (int)((N + kThreads * kElems32 - 1) / (kThreads * kElems32)));
}

}  // namespace mfs
