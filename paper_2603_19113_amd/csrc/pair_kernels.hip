// Pair sums t_i = sum_j phi_kappa(x_i - xhat_j) q_j on gfx950 (eq. Gmtx-entries, eq. out_skel).
//
// Layout and mapping
//   * One wave (64 lanes) owns 64*TPT consecutive targets; lane l holds targets base + 64*i + l.
//     Consecutive targets belong to one body (bodies are packed contiguously), so a wave's
//     targets span only one or two bodies.
//   * Sources are streamed in index order.  Every lane needs the same source at the same time,
//     so source coordinates, charges and body ids are read with wave-uniform addresses: the
//     compiler turns them into scalar (SGPR) loads and no LDS staging is needed.
//   * The source range is split into nchunks chunks (grid.y) to give the chip enough waves;
//     each chunk writes its own partial sum partial[c][r][M], and the consumer adds the chunks
//     in a fixed order, so the result is deterministic (no atomics).
//   * Same-body exclusion (G_hat has zero diagonal blocks, eq. mbody2): a wave computes the range
//     [body_ptr[bmin], body_ptr[bmax+1]) of sources that share a body with any of its targets;
//     only that range is evaluated with a per-pair body-id test, the rest runs unmasked.
//   * grid.z tiles the right-hand sides, RT per block; phi is computed once per pair and applied
//     to the RT charges.
#include <atomic>

#include "mfs_internal.h"
#include "phi.h"
#include "bodyphase.h"

namespace mfs {
namespace {

constexpr int kWaves = 4;  // waves per block
constexpr int kBlock = 64 * kWaves;
constexpr int kUnroll = 8;

template <typename T, int DIM>
struct PhiEval;

template <>
struct PhiEval<float, 2> {
  Phi2DConstsF32 c;
  __device__ __forceinline__ void operator()(float r2, float& pr, float& pi) const { phi2d_f32(r2, c, pr, pi); }
};
template <>
struct PhiEval<float, 3> {
  Phi3DConstsF32 c;
  __device__ __forceinline__ void operator()(float r2, float& pr, float& pi) const { phi3d_f32(r2, c, pr, pi); }
};
template <>
struct PhiEval<double, 2> {
  double kappa;
  __device__ __forceinline__ void operator()(double r2, double& pr, double& pi) const {
    phi2d_f64(sqrt(r2), kappa, pr, pi);
  }
};
template <>
struct PhiEval<double, 3> {
  double kappa;
  __device__ __forceinline__ void operator()(double r2, double& pr, double& pi) const {
    phi3d_f64(sqrt(r2), kappa, pr, pi);
  }
};

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

template <typename T, int DIM, int TPT, int RT>
struct Acc {
  T tx[TPT][DIM];
  int tb[TPT];
  T ar[TPT][RT];
  T ai[TPT][RT];
};

// One source j against all targets of the lane.
template <typename T, int DIM, int TPT, int RT, bool MASK>
__device__ __forceinline__ void accumulate_source(Acc<T, DIM, TPT, RT>& a, const PhiEval<T, DIM>& phi,
                                                  const T* __restrict__ s0, const T* __restrict__ s1,
                                                  const T* __restrict__ s2, const int32_t* __restrict__ sbody,
                                                  const Cplx<T>* __restrict__ q, int64_t N, int R, int r0,
                                                  int64_t j) {
  const T sx = s0[j];
  const T sy = s1[j];
  T sz = T(0);
  if constexpr (DIM == 3) sz = s2[j];
  T qr[RT], qi[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) {
    const int r = (r0 + rr < R) ? r0 + rr : R - 1;  // clamp keeps the load in bounds
    const Cplx<T> qq = q[(int64_t)r * N + j];
    qr[rr] = qq.re;
    qi[rr] = qq.im;
  }
  int sb = 0;
  if constexpr (MASK) sb = sbody[j];
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const T dx = a.tx[i][0] - sx;
    const T dy = a.tx[i][1] - sy;
    T r2 = dx * dx + dy * dy;
    if constexpr (DIM == 3) {
      const T dz = a.tx[i][2] - sz;
      r2 = r2 + dz * dz;
    }
    T pr, pi;
    phi(r2, pr, pi);
    if constexpr (MASK) {
      const bool same = (a.tb[i] == sb);
      pr = same ? T(0) : pr;
      pi = same ? T(0) : pi;
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      a.ar[i][rr] = fma(pr, qr[rr], fma(-pi, qi[rr], a.ar[i][rr]));
      a.ai[i][rr] = fma(pr, qi[rr], fma(pi, qr[rr], a.ai[i][rr]));
    }
  }
}

template <typename T, int DIM, int TPT, int RT, bool MASK>
__device__ __forceinline__ void run_range(Acc<T, DIM, TPT, RT>& a, const PhiEval<T, DIM>& phi,
                                          const T* __restrict__ s0, const T* __restrict__ s1,
                                          const T* __restrict__ s2, const int32_t* __restrict__ sbody,
                                          const Cplx<T>* __restrict__ q, int64_t N, int R, int r0, int64_t lo,
                                          int64_t hi) {
  int64_t j = lo;
  for (; j + kUnroll <= hi; j += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      accumulate_source<T, DIM, TPT, RT, MASK>(a, phi, s0, s1, s2, sbody, q, N, R, r0, j + u);
  }
  for (; j < hi; ++j) accumulate_source<T, DIM, TPT, RT, MASK>(a, phi, s0, s1, s2, sbody, q, N, R, r0, j);
}

// EXT: targets are external FP64 points (field evaluation, no exclusion); otherwise the targets
// are the scene's own points and same-body pairs are excluded.
template <typename T, int DIM, int TPT, int RT, bool EXT>
__global__ __launch_bounds__(kBlock) void pair_sum_kernel(
    PhiEval<T, DIM> phi, const T* __restrict__ s0, const T* __restrict__ s1, const T* __restrict__ s2,
    const int32_t* __restrict__ sbody, const int64_t* __restrict__ body_ptr, const Cplx<T>* __restrict__ q,
    int64_t N, int R, const double* __restrict__ targets, double ox, double oy, double oz, int64_t M,
    int64_t chunk_len, Cplx<T>* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * kWaves + wave) * (64 * TPT);
  if (base >= M) return;  // whole wave idle (uniform)
  const int r0 = blockIdx.z * RT;
  const int64_t c0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t c1 = min(N, c0 + chunk_len);

  Acc<T, DIM, TPT, RT> a;
  int bmin = 0x7fffffff, bmax = -1;
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int64_t t = base + 64 * i + lane;
    const bool ok = t < M;
    const int64_t tc = ok ? t : M - 1;
    if constexpr (EXT) {
      // FP32 sources are relative to the scene origin; FP64 sources are absolute (ox = oy = oz = 0)
      a.tx[i][0] = (T)(targets[tc * DIM + 0] - ox);
      a.tx[i][1] = (T)(targets[tc * DIM + 1] - oy);
      if constexpr (DIM == 3) a.tx[i][2] = (T)(targets[tc * DIM + 2] - oz);
      a.tb[i] = -1;
    } else {
      a.tx[i][0] = s0[tc];
      a.tx[i][1] = s1[tc];
      if constexpr (DIM == 3) a.tx[i][2] = s2[tc];
      a.tb[i] = ok ? sbody[tc] : -1;
      if (ok) {
        bmin = min(bmin, a.tb[i]);
        bmax = max(bmax, a.tb[i]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) a.ar[i][rr] = a.ai[i][rr] = T(0);
  }

  if constexpr (EXT) {
    run_range<T, DIM, TPT, RT, false>(a, phi, s0, s1, s2, sbody, q, N, R, r0, c0, c1);
  } else {
    bmin = wave_min_i32(bmin);
    bmax = wave_max_i32(bmax);
    const int64_t s_lo = body_ptr[bmin];
    const int64_t s_hi = body_ptr[bmax + 1];
    run_range<T, DIM, TPT, RT, false>(a, phi, s0, s1, s2, sbody, q, N, R, r0, c0, min(c1, s_lo));
    run_range<T, DIM, TPT, RT, true>(a, phi, s0, s1, s2, sbody, q, N, R, r0, max(c0, s_lo), min(c1, s_hi));
    run_range<T, DIM, TPT, RT, false>(a, phi, s0, s1, s2, sbody, q, N, R, r0, max(c0, s_hi), c1);
  }

#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int64_t t = base + 64 * i + lane;
    if (t >= M) continue;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const int r = r0 + rr;
      if (r >= R) continue;
      Cplx<T> v;
      v.re = a.ar[i][rr];
      v.im = a.ai[i][rr];
      partial[((int64_t)blockIdx.y * R + r) * M + t] = v;
    }
  }
}

template <int DIM, int TPT, int RT>
struct BPAcc {
  float lx[TPT][DIM];  // target body-local offsets
  double c[TPT][DIM];  // target body centres
  int tb[TPT];
  double ar[TPT][RT], ai[TPT][RT];  // FP64 accumulators
  // per source body: u = A + |l_s|^2 + P . l_s with A = |l_t|^2 + 2 dc . l_t, P = -2 (l_t + dc)
  float A[TPT], P[TPT][DIM];
  float D[TPT], D2[TPT], ph0[TPT];
  float sr_[TPT][RT], si_[TPT][RT];  // FP32 partial sums over the current source body
};

template <int DIM, int TPT, int RT, bool MASK, int FAR = 0>
__device__ __forceinline__ void bp_source(BPAcc<DIM, TPT, RT>& a, const BodyPhaseConsts& k, int sb,
                                          const float* __restrict__ l0, const float* __restrict__ l1,
                                          const float* __restrict__ l2, const float* __restrict__ lsq,
                                          const c64* __restrict__ q, int64_t N, int R, int r0, int64_t j) {
  float ls[DIM];
  ls[0] = l0[j];
  ls[1] = l1[j];
  if constexpr (DIM == 3) ls[2] = l2[j];
  const float bs = lsq[j];
  float qr[RT], qi[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) {
    const int r = (r0 + rr < R) ? r0 + rr : R - 1;
    const c64 qq = q[(int64_t)r * N + j];
    qr[rr] = qq.re;
    qi[rr] = qq.im;
  }
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    // u = |dl|^2 + 2 dc.dl = A + |l_s|^2 + P . l_s
    float u = a.A[i] + bs;
#pragma unroll
    for (int d = 0; d < DIM; ++d) u = fmaf(a.P[i][d], ls[d], u);
    float pr, pi;
    bp_phi<DIM, FAR>(k, u, a.D[i], a.D2[i], a.ph0[i], pr, pi);
    if constexpr (MASK) {
      const bool same = a.tb[i] == sb;
      pr = same ? 0.0f : pr;
      pi = same ? 0.0f : pi;
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      a.sr_[i][rr] = fmaf(pr, qr[rr], fmaf(-pi, qi[rr], a.sr_[i][rr]));
      a.si_[i][rr] = fmaf(pr, qi[rr], fmaf(pi, qr[rr], a.si_[i][rr]));
    }
  }
}

template <int DIM, int TPT, int RT>
__global__ __launch_bounds__(kBlock) void ghat_bodyphase_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of, const int64_t* __restrict__ body_ptr,
    const c64* __restrict__ q, int64_t N, int R, int64_t chunk_len, c64* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * kWaves + wave) * (64 * TPT);
  if (base >= N) return;
  const int r0 = blockIdx.z * RT;
  const int64_t c0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t c1 = min(N, c0 + chunk_len);

  BPAcc<DIM, TPT, RT> a;
  int bmin = 0x7fffffff, bmax = -1;
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int64_t t = base + 64 * i + lane;
    const bool ok = t < N;
    const int64_t tc = ok ? t : N - 1;
    a.lx[i][0] = l0[tc];
    a.lx[i][1] = l1[tc];
    if constexpr (DIM == 3) a.lx[i][2] = l2[tc];
    const int tb = body_of[tc];
    a.tb[i] = ok ? tb : -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) a.c[i][d] = cen[(int64_t)tb * DIM + d];
    if (ok) {
      bmin = min(bmin, tb);
      bmax = max(bmax, tb);
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) a.ar[i][rr] = a.ai[i][rr] = 0.0;
  }
  bmin = wave_min_i32(bmin);
  bmax = wave_max_i32(bmax);

  if (c0 < c1) {
    const int sb0 = body_of[c0];
    const int sb1 = body_of[c1 - 1];
    for (int sb = sb0; sb <= sb1; ++sb) {
      const int64_t j0 = max(c0, body_ptr[sb]);
      const int64_t j1 = min(c1, body_ptr[sb + 1]);
      double cs[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) cs[d] = cen[(int64_t)sb * DIM + d];
#pragma unroll
      for (int i = 0; i < TPT; ++i) {
        double D2 = 0.0;
        float Ai = 0.0f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double dc = a.c[i][d] - cs[d];
          D2 = fma(dc, dc, D2);
          const float dcf = (float)dc;
          Ai = fmaf(a.lx[i][d], a.lx[i][d] + 2.0f * dcf, Ai);
          a.P[i][d] = -2.0f * (a.lx[i][d] + dcf);
        }
        a.A[i] = Ai;
        const double D = sqrt(D2);
        const double ph = D * k.kappa_rev64;
        a.D[i] = (float)D;
        a.D2[i] = (float)D2;
        // phase of kappa D in revolutions, minus pi/4 (2D) folded in
        a.ph0[i] = (float)(ph - floor(ph)) - (DIM == 2 ? 0.125f : 0.0f);
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) a.sr_[i][rr] = a.si_[i][rr] = 0.0f;
      }
      const bool masked = sb >= bmin && sb <= bmax;
      // every pair of this wave and source body in the far regime (z >= 12): branch-free loop
      bool far_lane = true;
#pragma unroll
      for (int i = 0; i < TPT; ++i) far_lane = far_lane && (a.tb[i] < 0 || a.D[i] >= k.far_D);
      const bool far_all = DIM == 2 && !masked && __all(far_lane);
      bool vfar_lane = true;
#pragma unroll
      for (int i = 0; i < TPT; ++i) vfar_lane = vfar_lane && (a.tb[i] < 0 || a.D[i] >= k.vfar_D);
      const bool vfar_all = far_all && __all(vfar_lane);
      int64_t j = j0;
      if (vfar_all) {  // every pair at z >= 100: shorter asymptotic expansions
        for (; j + kUnroll <= j1; j += kUnroll) {
#pragma unroll
          for (int uu = 0; uu < kUnroll; ++uu)
            bp_source<DIM, TPT, RT, false, 2>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j + uu);
        }
        for (; j < j1; ++j) bp_source<DIM, TPT, RT, false, 2>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j);
      } else if (far_all) {
        for (; j + kUnroll <= j1; j += kUnroll) {
#pragma unroll
          for (int uu = 0; uu < kUnroll; ++uu)
            bp_source<DIM, TPT, RT, false, 1>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j + uu);
        }
        for (; j < j1; ++j) bp_source<DIM, TPT, RT, false, 1>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j);
      } else if (!masked) {
        for (; j + kUnroll <= j1; j += kUnroll) {
#pragma unroll
          for (int uu = 0; uu < kUnroll; ++uu)
            bp_source<DIM, TPT, RT, false>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j + uu);
        }
        for (; j < j1; ++j) bp_source<DIM, TPT, RT, false>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j);
      } else {
        for (; j < j1; ++j) bp_source<DIM, TPT, RT, true>(a, k, sb, l0, l1, l2, lsq, q, N, R, r0, j);
      }
#pragma unroll
      for (int i = 0; i < TPT; ++i)
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          a.ar[i][rr] += (double)a.sr_[i][rr];
          a.ai[i][rr] += (double)a.si_[i][rr];
        }
    }
  }

#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int64_t t = base + 64 * i + lane;
    if (t >= N) continue;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const int r = r0 + rr;
      if (r >= R) continue;
      partial[((int64_t)blockIdx.y * R + r) * N + t] = c64{(float)a.ar[i][rr], (float)a.ai[i][rr]};
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric pair sum, one right-hand side: G_hat is symmetric (phi depends on |x_i - x_j| only),
// so each unordered pair of points on different bodies needs one evaluation of phi, applied to
// both t_i += phi q_j and t_j += phi q_i.
//
// Requires every body to hold a multiple of 64 points, so that every aligned tile of 64 points
// lies on one body.  Points are cut into groups of kSymGroup = 256 (four tiles); with G groups,
// group g meets group h = (g + d) mod G for d = 0 .. Dmax (Dmax = floor(G/2)):
//   * 1 <= d < G/2: symmetric, each unordered pair of groups is met once, by g;
//   * d = 0 (the group with itself) and d = G/2 for even G: one-sided, only t of group g.
// A wave owns a group of targets, four per lane (lane l: targets 64 m + l).  Against a source tile
// staged in LDS twice over (entries e and e + 64) it makes 64 steps: at step s lane l takes source
// (l + s) mod 64 from entry l + s, so the 64 lanes see 64 different sources and after 64 steps
// every (target, source) pair of the tile has been formed once.  The source-side sums travel with
// the sources: at step s lane l holds the running sum of source (l + s) mod 64, adds its products
// into it and hands it on with a wave rotation (DPP wave_rol:1, lane l receives lane l + 1's
// value), so after 64 steps lane j holds source j's sum.  Everything stays in registers and in
// program order: deterministic, no atomics.  Two block shapes:
//   * ghat_sym_kernel, one wave per block and a range of distances (grid.y); it stages its own
//     source tiles and stores its source-side sums of distance d into the slice of d:
//       partial[c][N]                    target-side sums of distance chunk c (c < nchunks_d)
//       partial[nchunks_d + d - 1][N]    source-side sums of distance d, written by group h - d;
//   * ghat_sym_shared_kernel, W waves per block (G padded with empty groups to a multiple of W),
//     wave w holding target group g = W b + w, and a chunk of block offsets hh (grid.y): at offset
//     hh every wave meets the same source group (W b + hh) mod G, wave w at distance d = hh - w
//     (idle where d lies outside 0 .. Dmax), so each source tile is staged once for the block, and
//     the waves' sums of it are added in wave order by one wave and stored once:
//       partial[c][N]                    target-side sums of offset chunk c (c < nchunks_d)
//       partial[nchunks_d + hh / W][N]   source-side sums of offset hh, written by block
//                                        ((h - hh) mod G) / W; for a given slice and source group
//                                        exactly one block and one offset qualify (G is a multiple
//                                        of W, so hh = h mod W + W * slice).
//     About W times fewer slices (HBM writes and footprint), for a barrier per tile.
// Both store plainly; the S product adds the slices in a fixed order.
// Body-centre phase split and the Hankel branches are those of the kernel above; the body pair of
// a (target tile, source tile) is wave-uniform, so are the far-field tests and the same-body skip.
// ---------------------------------------------------------------------------
constexpr int kSymTiles = 4;                 // target tiles per wave
constexpr int kSymGroup = 64 * kSymTiles;    // points per group
constexpr int kSubBlock = 16;                // points per sub-block (3D kernel on 16-point sub-blocks)
constexpr int kSubStride = 48;               // LDS floats per staged sub-block (that kernel)

template <int DIM, int RT>
struct SymLds {
  float l[DIM][128];
  float bs[128];
  float qr[RT][128], qi[RT][128];
};

// lane l receives lane (l + 1) mod 64's value
__device__ __forceinline__ float wave_rotate_next(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x134, 0xf, 0xf, false));
}

// All four target tiles against the staged source tile, every pair in the far regime (FAR = 2:
// z >= 100, the common case; FAR = 1: z >= 12): one pass over the 64 steps, phi of each (target,
// source) used for both sums of each of the RT right-hand sides.
template <int DIM, int RT, bool SYM, int FAR>
__device__ __forceinline__ void sym_steps4(const SymLds<DIM, RT>& sh, const BodyPhaseConsts& k, int lane,
                                           const float (&A)[kSymTiles], const float (&P)[kSymTiles][DIM],
                                           const float (&D)[kSymTiles], const float (&D2)[kSymTiles],
                                           const float (&ph0)[kSymTiles], const float (&qtr)[kSymTiles][RT],
                                           const float (&qti)[kSymTiles][RT], float (&tr)[kSymTiles][RT],
                                           float (&ti)[kSymTiles][RT], float (&ar)[RT], float (&ai)[RT]) {
  for (int s0 = 0; s0 < 64; s0 += 8) {
    const int e0 = lane + s0;
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int e = e0 + uu;
      float ls[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) ls[d] = sh.l[d][e];
      const float bs = sh.bs[e];
      float qr[RT], qi[RT], sr[RT], si[RT];
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) {
        qr[rr] = sh.qr[rr][e];
        qi[rr] = sh.qi[rr][e];
        sr[rr] = ar[rr];
        si[rr] = ai[rr];
      }
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m) {
        float u = A[m] + bs;
#pragma unroll
        for (int d = 0; d < DIM; ++d) u = fmaf(P[m][d], ls[d], u);
        float pr, pi;
        bp_phi<DIM, FAR>(k, u, D[m], D2[m], ph0[m], pr, pi);
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          tr[m][rr] = fmaf(pr, qr[rr], fmaf(-pi, qi[rr], tr[m][rr]));
          ti[m][rr] = fmaf(pr, qi[rr], fmaf(pi, qr[rr], ti[m][rr]));
          if constexpr (SYM) {
            sr[rr] = fmaf(pr, qtr[m][rr], fmaf(-pi, qti[m][rr], sr[rr]));
            si[rr] = fmaf(pr, qti[m][rr], fmaf(pi, qtr[m][rr], si[rr]));
          }
        }
      }
      if constexpr (SYM) {
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          ar[rr] = wave_rotate_next(sr[rr]);
          ai[rr] = wave_rotate_next(si[rr]);
        }
      }
    }
  }
}

// One target tile against the staged source tile, with the Hankel branch set FAR (any regime):
// the rare cases (near body pairs, partly filled or same-body tiles), kept lean in registers.
// 64 rotations bring the source-side sums back to their own lanes, so passes can follow each other.
template <int DIM, int RT, bool SYM, int FAR>
__device__ __forceinline__ void sym_steps1(const SymLds<DIM, RT>& sh, const BodyPhaseConsts& k, int lane, float A,
                                           const float (&P)[DIM], float D, float D2, float ph0,
                                           const float (&qtr)[RT], const float (&qti)[RT], float (&tr)[RT],
                                           float (&ti)[RT], float (&ar)[RT], float (&ai)[RT]) {
  for (int s0 = 0; s0 < 64; s0 += 8) {
    const int e0 = lane + s0;
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int e = e0 + uu;
      float u = A + sh.bs[e];
#pragma unroll
      for (int d = 0; d < DIM; ++d) u = fmaf(P[d], sh.l[d][e], u);
      float pr, pi;
      bp_phi<DIM, FAR>(k, u, D, D2, ph0, pr, pi);
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) {
        const float qr = sh.qr[rr][e], qi = sh.qi[rr][e];
        tr[rr] = fmaf(pr, qr, fmaf(-pi, qi, tr[rr]));
        ti[rr] = fmaf(pr, qi, fmaf(pi, qr, ti[rr]));
        if constexpr (SYM) {
          ar[rr] = wave_rotate_next(fmaf(pr, qtr[rr], fmaf(-pi, qti[rr], ar[rr])));
          ai[rr] = wave_rotate_next(fmaf(pr, qti[rr], fmaf(pi, qtr[rr], ai[rr])));
        }
      }
    }
  }
}

template <int DIM, int RT, bool SYM>
__device__ __forceinline__ void sym_tile(const SymLds<DIM, RT>& sh, const BodyPhaseConsts& k, int lane,
                                         const bool (&use)[kSymTiles], const float (&A)[kSymTiles],
                                         const float (&P)[kSymTiles][DIM], const float (&D)[kSymTiles],
                                         const float (&D2)[kSymTiles], const float (&ph0)[kSymTiles],
                                         const float (&qtr)[kSymTiles][RT], const float (&qti)[kSymTiles][RT],
                                         float (&tr)[kSymTiles][RT], float (&ti)[kSymTiles][RT], float (&ar)[RT],
                                         float (&ai)[RT]) {
  bool all = true;
  float dmin = 3.0e38f;
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    all = all && use[m];
    dmin = fminf(dmin, D[m]);
  }
  if (all && (DIM == 3 || dmin >= k.vfar_D)) {
    sym_steps4<DIM, RT, SYM, 2>(sh, k, lane, A, P, D, D2, ph0, qtr, qti, tr, ti, ar, ai);
    return;
  }
  if (DIM == 2 && all && dmin >= k.far_D) {  // closer scenes (serving at kappa 5 to 10)
    sym_steps4<DIM, RT, SYM, 1>(sh, k, lane, A, P, D, D2, ph0, qtr, qti, tr, ti, ar, ai);
    return;
  }
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    if (!use[m]) continue;
    if (DIM == 3 || D[m] >= k.vfar_D)
      sym_steps1<DIM, RT, SYM, 2>(sh, k, lane, A[m], P[m], D[m], D2[m], ph0[m], qtr[m], qti[m], tr[m], ti[m], ar, ai);
    else if (D[m] >= k.far_D)
      sym_steps1<DIM, RT, SYM, 1>(sh, k, lane, A[m], P[m], D[m], D2[m], ph0[m], qtr[m], qti[m], tr[m], ti[m], ar, ai);
    else
      sym_steps1<DIM, RT, SYM, 0>(sh, k, lane, A[m], P[m], D[m], D2[m], ph0[m], qtr[m], qti[m], tr[m], ti[m], ar, ai);
  }
}

// Occupancy target per right-hand-side grouping: the register file holds 4, 3 or 2 waves per SIMD.
template <int RT>
struct SymWaves {
  static constexpr int value = RT == 1 ? 4 : (RT == 2 ? 3 : 2);
};

// The block's walk over source tiles: the first tile at or after (hh, ts) of source group
// (gb + hh) mod G that holds points, skipping groups past N; false at the chunk's end hh1.  Every
// value here is uniform over the block, so are the barriers that follow the walk.
// First point of tile ts of source group (gb + hh) mod G: gb + hh < 2 G for every block offset of the
// plan (gb <= G - kSymW, hh < Dmax + 2 kSymW - 1; for G = kSymW, gb = 0 and hh < 2 G), so one
// conditional subtraction takes the place of a 64-bit remainder.
__device__ __forceinline__ int64_t sym_tile_start(int64_t gb, int64_t G, int hh, int ts) {
  int64_t h = gb + hh;
  if (h >= G) h -= G;
  return h * kSymGroup + 64 * ts;
}

__device__ __forceinline__ bool sym_seek(int64_t gb, int64_t G, int64_t N, int hh1, int& hh, int& ts) {
  while (hh < hh1) {
    if (ts < kSymTiles && sym_tile_start(gb, G, hh, ts) < N) return true;
    ++hh;
    ts = 0;
  }
  return false;
}

// Each wave's source-side sums of a staged tile (double-buffered with the tiles): lane l holds
// source l's sum, as the rotation leaves it.
template <int RT, int W>
struct SymComb {
  float re[2][W][RT][64], im[2][W][RT][64];
};

// One store per source of the tile: the block's waves' sums added in wave order (deterministic).
template <int RT, int W>
__device__ __forceinline__ void sym_combine(const SymComb<RT, W>& cb, int buf, int lane, int64_t j0, int64_t N, int R,
                                            int r0, int slice, float scale, c64* __restrict__ partial) {
  if (j0 + lane >= N) return;
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) {
    if (r0 + rr >= R) break;
    float xr = 0.0f, xi = 0.0f;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      xr += cb.re[buf][w][rr][lane];
      xi += cb.im[buf][w][rr][lane];
    }
    partial[((int64_t)slice * R + r0 + rr) * N + j0 + lane] = c64{xr * scale, xi * scale};
  }
}

// Staging of one source tile spread over the block: 64 / W sources per wave and one value per lane
// (value v: field v / (64 / W) of source (64 / W) * wave + v % (64 / W); the fields are the DIM
// coordinates, |l|^2, then the real and the imaginary parts of the RT charges, in the order of the
// staging arrays), so that the loads of the next tile stay in flight in one or two registers while
// the wave works on the current tile (with one wave per block, each lane holds its own source's
// fields).  Sources past N (only where tiles may be partly filled) take zero offset and charge and
// |l|^2 = 1, so that no distance is zero.
template <int DIM, int RT, int W>
struct SymStage {
  static constexpr int kSrc = 64 / W;
  static constexpr int kFields = DIM + 1 + 2 * RT;
  static constexpr int kVals = kSrc * kFields;
  static constexpr int kRegs = (kVals + 63) / 64;
  float v[kRegs];
};

template <int DIM, int RT, int W>
__device__ __forceinline__ void sym_stage_load(SymStage<DIM, RT, W>& st, const float* __restrict__ l0,
                                               const float* __restrict__ l1, const float* __restrict__ l2,
                                               const float* __restrict__ lsq, const c64* __restrict__ q,
                                               const int (&rof)[RT], int64_t N, int64_t j0, int wv, int lane) {
  constexpr int kSrc = SymStage<DIM, RT, W>::kSrc;
#pragma unroll
  for (int k = 0; k < SymStage<DIM, RT, W>::kRegs; ++k) {
    const int v = lane + 64 * k;
    float x = 0.0f;
    if (v < SymStage<DIM, RT, W>::kVals) {
      const int f = v / kSrc;
      const int64_t j = j0 + kSrc * wv + v % kSrc;
      if (j < N) {
        if (f < DIM) x = (f == 0 ? l0 : f == 1 ? l1 : l2)[j];
        else if (f == DIM) x = lsq[j];
        else {
          const int c = f - DIM - 1, rr = c < RT ? c : c - RT;
          int r = rof[0];
#pragma unroll
          for (int i = 1; i < RT; ++i) r = rr == i ? rof[i] : r;
          x = reinterpret_cast<const float*>(q)[2 * ((int64_t)r * N + j) + (c < RT ? 0 : 1)];
        }
      } else if (f == DIM) {
        x = 1.0f;
      }
    }
    st.v[k] = x;
  }
}

// Store the staged values into the staging arrays (flat view: field f at f * STRIDE), each source
// at entry E(p) and E(p) + DUP.
template <int STRIDE, int DUP, bool SUB16, int DIM, int RT, int W>
__device__ __forceinline__ void sym_stage_store(const SymStage<DIM, RT, W>& st, float* __restrict__ base, int wv,
                                                int lane) {
  constexpr int kSrc = SymStage<DIM, RT, W>::kSrc;
#pragma unroll
  for (int k = 0; k < SymStage<DIM, RT, W>::kRegs; ++k) {
    const int v = lane + 64 * k;
    if (v < SymStage<DIM, RT, W>::kVals) {
      const int f = v / kSrc, p = kSrc * wv + v % kSrc;
      const int e = f * STRIDE + (SUB16 ? (p >> 4) * kSubStride + (p & 15) : p);
      base[e] = st.v[k];
      base[e + DUP] = st.v[k];
    }
  }
}

template <int DIM, int RT>
__global__ __launch_bounds__(64, SymWaves<RT>::value) void ghat_sym_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of,
    const c64* __restrict__ q, int64_t N, int R, int64_t G, int Dmax, int even_G, int dpc, int nchunks_d,
    c64* __restrict__ partial) {
  __shared__ SymLds<DIM, RT> sh;
  const int lane = threadIdx.x;
  const int64_t g = blockIdx.x;
  const int c = blockIdx.y;
  const int r0 = blockIdx.z * RT;  // right-hand sides r0 .. r0 + RT - 1 (those >= R repeat R - 1, unstored)
  const int d0 = c * dpc;
  const int d1 = min(Dmax + 1, d0 + dpc);
  const float* lsrc[3] = {l0, l1, l2};
  int rof[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) rof[rr] = min(r0 + rr, R - 1);

  // targets of this wave: tile m covers points g*256 + 64 m + (0..63), all on one body
  bool act[kSymTiles];
  int tb[kSymTiles];
  float lt[kSymTiles][DIM], qtr[kSymTiles][RT], qti[kSymTiles][RT];
  double ar[kSymTiles][RT], ai[kSymTiles][RT];
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t0 = g * kSymGroup + 64 * m;
    act[m] = t0 < N;
    const int64_t t = act[m] ? t0 + lane : 0;
    tb[m] = act[m] ? __builtin_amdgcn_readfirstlane(body_of[t0]) : -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) lt[m][d] = lsrc[d][t];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const c64 qq = q[(int64_t)rof[rr] * N + t];
      qtr[m][rr] = act[m] ? qq.re : 0.0f;
      qti[m][rr] = act[m] ? qq.im : 0.0f;
      ar[m][rr] = ai[m][rr] = 0.0;
    }
  }

  for (int d = d0; d < d1; ++d) {
    int64_t h = g + d;
    if (h >= G) h -= G;
    const bool sym = d != 0 && !(even_G && d == Dmax);
    for (int ts = 0; ts < kSymTiles; ++ts) {
      const int64_t j0 = h * kSymGroup + 64 * ts;
      if (j0 >= N) break;
      const int sb = __builtin_amdgcn_readfirstlane(body_of[j0]);
      // stage the source tile (entries e and e + 64)
      {
        const int64_t j = j0 + lane;
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) sh.l[dd][lane] = sh.l[dd][lane + 64] = lsrc[dd][j];
        sh.bs[lane] = sh.bs[lane + 64] = lsq[j];
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          const c64 qq = q[(int64_t)rof[rr] * N + j];
          sh.qr[rr][lane] = sh.qr[rr][lane + 64] = qq.re;
          sh.qi[rr][lane] = sh.qi[rr][lane + 64] = qq.im;
        }
      }
      __syncthreads();
      // per target tile: body-centre split against the source body (uniform over the wave)
      double cs[DIM];
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd) cs[dd] = cen[(int64_t)sb * DIM + dd];
      bool use[kSymTiles];
      float A[kSymTiles], P[kSymTiles][DIM], D[kSymTiles], D2[kSymTiles], ph0[kSymTiles];
      float tr[kSymTiles][RT], ti[kSymTiles][RT];
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m) {
        use[m] = act[m] && tb[m] != sb;
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) tr[m][rr] = ti[m][rr] = 0.0f;
        const int bt = use[m] ? tb[m] : sb;
        double D2d = 0.0;
        float Am = 0.0f;
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) {
          const double dc = cen[(int64_t)bt * DIM + dd] - cs[dd];
          D2d = fma(dc, dc, D2d);
          const float dcf = (float)dc;
          Am = fmaf(lt[m][dd], lt[m][dd] + 2.0f * dcf, Am);
          P[m][dd] = -2.0f * (lt[m][dd] + dcf);
        }
        A[m] = Am;
        const double Dd = sqrt(D2d);
        const double ph = Dd * k.kappa_rev64;
        D[m] = (float)Dd;
        D2[m] = (float)D2d;
        ph0[m] = (float)(ph - floor(ph)) - (DIM == 2 ? 0.125f : 0.0f);
      }
      float sr[RT], si[RT];  // lane l: source-side sums of source j0 + l (after the tile)
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) sr[rr] = si[rr] = 0.0f;
      if (sym) sym_tile<DIM, RT, true>(sh, k, lane, use, A, P, D, D2, ph0, qtr, qti, tr, ti, sr, si);
      else sym_tile<DIM, RT, false>(sh, k, lane, use, A, P, D, D2, ph0, qtr, qti, tr, ti, sr, si);
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          ar[m][rr] += (double)tr[m][rr];
          ai[m][rr] += (double)ti[m][rr];
        }
      // source-side sums of this tile from the wave's targets -> slice of distance d
      if (sym) {
#pragma unroll
        for (int rr = 0; rr < RT; ++rr)
          if (r0 + rr < R)
            partial[((int64_t)(nchunks_d + d - 1) * R + r0 + rr) * N + j0 + lane] = c64{sr[rr], si[rr]};
      }
      __syncthreads();  // the tile's entries are read before the next tile is staged
    }
  }
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
      if (act[m] && r0 + rr < R)
        partial[((int64_t)c * R + r0 + rr) * N + g * kSymGroup + 64 * m + lane] =
            c64{(float)ar[m][rr], (float)ai[m][rr]};
}

// The symmetric pair sum with W waves per block sharing each staged source tile (see above).
template <int DIM, int RT, int W>
__global__ __launch_bounds__(64 * W, SymWaves<RT>::value) void ghat_sym_shared_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of,
    const c64* __restrict__ q, int64_t N, int R, int64_t G, int Dmax, int even_G, int HH, int dpc, int nchunks_d,
    c64* __restrict__ partial) {
  static_assert(W > 1, "one wave per block: ghat_sym_kernel");
  __shared__ SymLds<DIM, RT> sh[2];
  __shared__ SymComb<RT, W> cb;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t gb = (int64_t)blockIdx.x * W;  // the block's first target group
  const int64_t g = gb + wv;                        // this wave's
  const int c = blockIdx.y;
  const int r0 = blockIdx.z * RT;  // right-hand sides r0 .. r0 + RT - 1 (those >= R repeat R - 1, unstored)
  const int hh1 = min(HH, (c + 1) * dpc);
  const float* lsrc[3] = {l0, l1, l2};
  int rof[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) rof[rr] = min(r0 + rr, R - 1);

  // targets of this wave: tile m covers points g*256 + 64 m + (0..63), all on one body
  bool act[kSymTiles];
  int tb[kSymTiles];
  float lt[kSymTiles][DIM], qtr[kSymTiles][RT], qti[kSymTiles][RT];
  double ar[kSymTiles][RT], ai[kSymTiles][RT];
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t0 = g * kSymGroup + 64 * m;
    act[m] = t0 < N;
    const int64_t t = act[m] ? t0 + lane : 0;
    tb[m] = act[m] ? __builtin_amdgcn_readfirstlane(body_of[t0]) : -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) lt[m][d] = lsrc[d][t];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const c64 qq = q[(int64_t)rof[rr] * N + t];
      qtr[m][rr] = act[m] ? qq.re : 0.0f;
      qti[m][rr] = act[m] ? qq.im : 0.0f;
      ar[m][rr] = ai[m][rr] = 0.0;
    }
  }

  // Walk the source tiles of block offsets c*dpc .. hh1 - 1.  At offset hh all waves meet group
  // (gb + hh) mod G, wave w at distance hh - w.  One barrier per tile: the tile is staged into
  // buffer t & 1 before it, the previous tile's sums are added after it (by wave (t - 1) mod W)
  // while the waves work on this one, and the next tile's loads are in flight meanwhile.
  int hh = c * dpc, ts = 0, t = 0, buf = 0, psl = 0;
  int64_t pj0 = 0;
  bool have = sym_seek(gb, G, N, hh1, hh, ts);
  SymStage<DIM, RT, W> stg;
  if (have) {
    sym_stage_load(stg, l0, l1, l2, lsq, q, rof, N, sym_tile_start(gb, G, hh, ts), wv, lane);
    sym_stage_store<128, 64, false>(stg, &sh[0].l[0][0], wv, lane);
  }
  while (have) {
    const int64_t j0 = sym_tile_start(gb, G, hh, ts);
    __syncthreads();  // tile t staged in buffer t & 1; every wave's sums of tile t - 1 in cb
    int nhh = hh, nts = ts + 1;
    const bool nhave = sym_seek(gb, G, N, hh1, nhh, nts);
    if (nhave) sym_stage_load(stg, l0, l1, l2, lsq, q, rof, N, sym_tile_start(gb, G, nhh, nts), wv, lane);
    if (t > 0 && wv == (t - 1) % W) sym_combine(cb, buf ^ 1, lane, pj0, N, R, r0, nchunks_d + psl, 1.0f, partial);
    const int d = hh - wv;
    const bool active = act[0] && d >= 0 && d <= Dmax;
    const bool sym = active && d != 0 && !(even_G && d == Dmax);
    float sr[RT], si[RT];  // lane l: source-side sums of source j0 + l (after the tile)
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) sr[rr] = si[rr] = 0.0f;
    if (active) {
      const int sb = __builtin_amdgcn_readfirstlane(body_of[j0]);
      // per target tile: body-centre split against the source body (uniform over the wave)
      double cs[DIM];
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd) cs[dd] = cen[(int64_t)sb * DIM + dd];
      bool use[kSymTiles];
      float A[kSymTiles], P[kSymTiles][DIM], D[kSymTiles], D2[kSymTiles], ph0[kSymTiles];
      float tr[kSymTiles][RT], ti[kSymTiles][RT];
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m) {
        use[m] = act[m] && tb[m] != sb;
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) tr[m][rr] = ti[m][rr] = 0.0f;
        const int bt = use[m] ? tb[m] : sb;
        double D2d = 0.0;
        float Am = 0.0f;
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) {
          const double dc = cen[(int64_t)bt * DIM + dd] - cs[dd];
          D2d = fma(dc, dc, D2d);
          const float dcf = (float)dc;
          Am = fmaf(lt[m][dd], lt[m][dd] + 2.0f * dcf, Am);
          P[m][dd] = -2.0f * (lt[m][dd] + dcf);
        }
        A[m] = Am;
        const double Dd = sqrt(D2d);
        const double ph = Dd * k.kappa_rev64;
        D[m] = (float)Dd;
        D2[m] = (float)D2d;
        ph0[m] = (float)(ph - floor(ph)) - (DIM == 2 ? 0.125f : 0.0f);
      }
      if (sym) sym_tile<DIM, RT, true>(sh[buf], k, lane, use, A, P, D, D2, ph0, qtr, qti, tr, ti, sr, si);
      else sym_tile<DIM, RT, false>(sh[buf], k, lane, use, A, P, D, D2, ph0, qtr, qti, tr, ti, sr, si);
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          ar[m][rr] += (double)tr[m][rr];
          ai[m][rr] += (double)ti[m][rr];
        }
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {  // zero where this wave formed no symmetric pair with the tile
      cb.re[buf][wv][rr][lane] = sym ? sr[rr] : 0.0f;
      cb.im[buf][wv][rr][lane] = sym ? si[rr] : 0.0f;
    }
    // the next tile into the other buffer (every wave is past its last read there: the barrier)
    if (nhave) sym_stage_store<128, 64, false>(stg, &sh[buf ^ 1].l[0][0], wv, lane);
    pj0 = j0;
    psl = hh / W;
    buf ^= 1;
    ++t;
    hh = nhh;
    ts = nts;
    have = nhave;
  }
  __syncthreads();
  if (t > 0 && wv == (t - 1) % W) sym_combine(cb, buf ^ 1, lane, pj0, N, R, r0, nchunks_d + psl, 1.0f, partial);
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
      if (act[m] && r0 + rr < R)
        partial[((int64_t)c * R + r0 + rr) * N + g * kSymGroup + 64 * m + lane] =
            c64{(float)ar[m][rr], (float)ai[m][rr]};
}

// ---------------------------------------------------------------------------
// Symmetric pair sum in 3D on bodies of 16 n points, without padding to whole tiles.
//
// Same group schedules, outputs and body-centre split as ghat_sym_kernel (one wave per block:
// ghat_sym16_kernel) and ghat_sym_shared_kernel (W waves: ghat_sym16_shared_kernel), but a 64-point
// tile may straddle bodies: it is seen as four sub-blocks of 16 points, each on one body (every body holds a
// multiple of 16 points, so bodies start on sub-block boundaries).  The 64 steps against a staged
// source tile run in four phases of 16.  Lane l = 16 G + i (row G) takes, in phase p, sub-block
// b = (G + p) mod 4 of the source tile, and at step t of the phase source 16 b + ((i + t) mod 16):
// over the four phases every lane meets every source once.  Within a phase a lane's sources all
// lie on one body, so the per-lane body-centre constants (target body against that sub-block's
// body) are fixed for the phase and are recomputed only at phase starts, and only when the source
// tile straddles bodies.  The source-side running sums rotate by one lane inside each row of 16
// per step (DPP row rotation), and at the end of a phase move one row down (lane l receives lane
// l + 16), where the next phase's lanes for that sub-block are; after four phases every sum is back
// in its own lane.  Sub-block entries are staged twice (e and e + 16) at a stride of 48 floats, so
// that the two half-waves read different LDS banks.  3D only: the kernel has no Hankel branches.
// Idle target lanes and idle source slots (past N) carry zero charge and stay finite.  The pairs are
// summed as e^{i kappa r} / r and the sums scaled by 1/(4 pi) when stored.
// ---------------------------------------------------------------------------

template <int RT>
struct Sym16Lds {
  float l[3][4 * kSubStride];
  float bs[4 * kSubStride];
  float qr[RT][4 * kSubStride], qi[RT][4 * kSubStride];
  double cs[4][3];  // centres of the four sub-blocks' bodies (zero past N), staged with the tile
  int sbb[4];       // bodies of the four sub-blocks, -1 past N
};

// Body-centre difference of a (target lane, source sub-block) pair, target body centre minus source
// body centre in FP64.  Where the target lane or the source sub-block is idle the pair carries zero
// charge; its constants are those of a body with itself (difference zero), so that every distance
// stays finite.  Two sources of the centres: the scene's table in global memory (one wave per
// block), or LDS (the wave's own target bodies tbase .. tbase + 15 and the staged tile's sub-blocks).
struct CentresGlobal {
  const double* __restrict__ cen;
  __device__ __forceinline__ void diff(int tb, int sb, int, double (&dc)[3]) const {
    const int bt = tb >= 0 ? tb : (sb >= 0 ? sb : 0);
    const int bs = sb >= 0 ? sb : bt;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) dc[dd] = cen[(int64_t)bt * 3 + dd] - cen[(int64_t)bs * 3 + dd];
  }
};

template <int RT>
struct CentresLds {
  const double (*tcen)[3];
  int tbase;
  const Sym16Lds<RT>* sh;
  __device__ __forceinline__ void diff(int tb, int sb, int blk, double (&dc)[3]) const {
    const bool both = tb >= 0 && sb >= 0;
    const int ti = both ? tb - tbase : 0;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) dc[dd] = both ? tcen[ti][dd] - sh->cs[blk][dd] : 0.0;
  }
};

// lane l receives the value of lane (l & ~15) | ((l + 1) & 15): rotation by one lane inside each row
// of 16 (DPP row_ror:15)
__device__ __forceinline__ float row_rotate_next(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x12F, 0xf, 0xf, false));
}

// lane l receives the value of lane (l + 16) mod 64
__device__ __forceinline__ float rows_shift_next(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 16) & 63) << 2, __float_as_int(x)));
}

// one of four wave-uniform values picked by a per-lane index
__device__ __forceinline__ int pick4(const int (&v)[4], int b) {
  return b == 0 ? v[0] : b == 1 ? v[1] : b == 2 ? v[2] : v[3];
}

// Body-centre split of a target (local offset lt) against a source body, dc = target body centre
// minus source body centre (FP64): u = A + |l_s|^2 + P . l_s with A = |l_t|^2 + 2 dc . l_t,
// P = -2 (l_t + dc), D = |dc| and the phase of kappa D in revolutions.
__device__ __forceinline__ void split_consts3(const BodyPhaseConsts& k, const double (&dc)[3], const float (&lt)[3],
                                              float& A, float (&P)[3], float& D, float& D2, float& ph0) {
  double D2d = 0.0;
  float Am = 0.0f;
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    D2d = fma(dc[dd], dc[dd], D2d);
    const float dcf = (float)dc[dd];
    Am = fmaf(lt[dd], lt[dd] + 2.0f * dcf, Am);
    P[dd] = -2.0f * (lt[dd] + dcf);
  }
  A = Am;
  const double Dd = sqrt(D2d);
  const double ph = Dd * k.kappa_rev64;
  D = (float)Dd;
  D2 = (float)D2d;
  ph0 = (float)(ph - floor(ph));
}

// 4 pi phi in 3D with the body-centre split: e^{i kappa r} / r (the 1/(4 pi) is applied to the sums).
// The phase in revolutions, ph0 + kappa delta / 2 pi, stays within [-1.2, 2.2] here (ph0 in [0, 1),
// |delta| below two body radii), well inside the [-256, 256] revolutions that v_sin / v_cos take, so
// no v_fract is needed before them.
__device__ __forceinline__ void phi3_4pi(const BodyPhaseConsts& k, float u, float D, float D2, float ph0, float& pr,
                                         float& pi) {
  const float r2 = D2 + u;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  const float delta = u * __builtin_amdgcn_rcpf(D + r);
  const float rev = fmaf(delta, k.kappa_rev, ph0);
  pr = rinv * __builtin_amdgcn_cosf(rev);
  pi = rinv * __builtin_amdgcn_sinf(rev);
}
constexpr float kInv4Pi = 0.07957747154594767f;

// All four target tiles against the staged source tile; no pair of the meeting is on one body.
template <int RT, bool SYM, typename CC>
__device__ __forceinline__ void sym16_steps4(const Sym16Lds<RT>& sh, const BodyPhaseConsts& k, const CC& cc, int lane,
                                             const int (&tb)[kSymTiles], const int (&sbb)[4], bool pure,
                                             const float (&lt)[kSymTiles][3],
                                             const float (&qtr)[kSymTiles][RT], const float (&qti)[kSymTiles][RT],
                                             float (&tr)[kSymTiles][RT], float (&ti)[kSymTiles][RT], float (&sr)[RT],
                                             float (&si)[RT]) {
  const int row = lane >> 4, li = lane & 15;
  float A[kSymTiles], P[kSymTiles][3], D[kSymTiles], D2[kSymTiles], ph0[kSymTiles];
  for (int p = 0; p < 4; ++p) {
    const int blk = (row + p) & 3;
    if (p == 0 || !pure) {
      const int sb = pick4(sbb, blk);
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m) {
        double dc[3];
        cc.diff(tb[m], sb, blk, dc);
        split_consts3(k, dc, lt[m], A[m], P[m], D[m], D2[m], ph0[m]);
      }
    }
    const int e0 = blk * kSubStride + li;
    for (int t0 = 0; t0 < kSubBlock; t0 += 8) {
#pragma unroll
      for (int uu = 0; uu < 8; ++uu) {
        const int e = e0 + t0 + uu;
        const float ls0 = sh.l[0][e], ls1 = sh.l[1][e], ls2 = sh.l[2][e];
        const float bs = sh.bs[e];
        float qr[RT], qi[RT];
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          qr[rr] = sh.qr[rr][e];
          qi[rr] = sh.qi[rr][e];
        }
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) {
          float u = A[m] + bs;
          u = fmaf(P[m][0], ls0, u);
          u = fmaf(P[m][1], ls1, u);
          u = fmaf(P[m][2], ls2, u);
          float pr, pi;
          phi3_4pi(k, u, D[m], D2[m], ph0[m], pr, pi);
#pragma unroll
          for (int rr = 0; rr < RT; ++rr) {
            tr[m][rr] = fmaf(pr, qr[rr], fmaf(-pi, qi[rr], tr[m][rr]));
            ti[m][rr] = fmaf(pr, qi[rr], fmaf(pi, qr[rr], ti[m][rr]));
            if constexpr (SYM) {
              sr[rr] = fmaf(pr, qtr[m][rr], fmaf(-pi, qti[m][rr], sr[rr]));
              si[rr] = fmaf(pr, qti[m][rr], fmaf(pi, qtr[m][rr], si[rr]));
            }
          }
        }
        if constexpr (SYM) {
#pragma unroll
          for (int rr = 0; rr < RT; ++rr) {
            sr[rr] = row_rotate_next(sr[rr]);
            si[rr] = row_rotate_next(si[rr]);
          }
        }
      }
    }
    if constexpr (SYM) {
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) {
        sr[rr] = rows_shift_next(sr[rr], lane);
        si[rr] = rows_shift_next(si[rr], lane);
      }
    }
  }
}

// One target tile against the staged source tile, pairs on one body skipped (a lane's source body
// is fixed within a phase, so the test is per lane and phase): the rare meetings near the diagonal.
// Four phases bring the source-side sums back to their own lanes, so passes can follow each other.
template <int RT, bool SYM, typename CC>
__device__ __forceinline__ void sym16_steps1(const Sym16Lds<RT>& sh, const BodyPhaseConsts& k, const CC& cc, int lane,
                                             int tbm, const int (&sbb)[4], const float (&ltm)[3],
                                             const float (&qtr)[RT], const float (&qti)[RT],
                                             float (&tr)[RT], float (&ti)[RT], float (&sr)[RT], float (&si)[RT]) {
  const int row = lane >> 4, li = lane & 15;
  for (int p = 0; p < 4; ++p) {
    const int blk = (row + p) & 3;
    const int sb = pick4(sbb, blk);
    double dc[3];
    cc.diff(tbm, sb, blk, dc);
    float A, P[3], D, D2, ph0;
    split_consts3(k, dc, ltm, A, P, D, D2, ph0);
    const bool same = tbm >= 0 && tbm == sb;
    const int e0 = blk * kSubStride + li;
    for (int t0 = 0; t0 < kSubBlock; t0 += 8) {
#pragma unroll
      for (int uu = 0; uu < 8; ++uu) {
        const int e = e0 + t0 + uu;
        float u = A + sh.bs[e];
        u = fmaf(P[0], sh.l[0][e], u);
        u = fmaf(P[1], sh.l[1][e], u);
        u = fmaf(P[2], sh.l[2][e], u);
        float pr, pi;
        phi3_4pi(k, u, D, D2, ph0, pr, pi);
        pr = same ? 0.0f : pr;  // a select: also discards the non-finite value of a point with itself
        pi = same ? 0.0f : pi;
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          const float qr = sh.qr[rr][e], qi = sh.qi[rr][e];
          tr[rr] = fmaf(pr, qr, fmaf(-pi, qi, tr[rr]));
          ti[rr] = fmaf(pr, qi, fmaf(pi, qr, ti[rr]));
          if constexpr (SYM) {
            sr[rr] = row_rotate_next(fmaf(pr, qtr[rr], fmaf(-pi, qti[rr], sr[rr])));
            si[rr] = row_rotate_next(fmaf(pr, qti[rr], fmaf(pi, qtr[rr], si[rr])));
          }
        }
      }
    }
    if constexpr (SYM) {
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) {
        sr[rr] = rows_shift_next(sr[rr], lane);
        si[rr] = rows_shift_next(si[rr], lane);
      }
    }
  }
}

// Bodies and body centres of a tile's four sub-blocks into its staging buffer (lanes 0..3 of the
// calling wave): read once per tile and block, so that the waves find them in LDS.
template <int RT>
__device__ __forceinline__ void sym16_stage_meta(Sym16Lds<RT>& sh, const double* __restrict__ cen,
                                                 const int32_t* __restrict__ body_of, int64_t N, int64_t j0, int lane) {
  if (lane < 4) {
    const int64_t j = j0 + kSubBlock * lane;
    const int b = j < N ? body_of[j] : -1;
    sh.sbb[lane] = b;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) sh.cs[lane][dd] = b >= 0 ? cen[(int64_t)b * 3 + dd] : 0.0;
  }
}

template <int RT>
__global__ __launch_bounds__(64, SymWaves<RT>::value) void ghat_sym16_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of,
    const c64* __restrict__ q, int64_t N, int R, int64_t G, int Dmax, int even_G, int dpc, int nchunks_d,
    c64* __restrict__ partial) {
  __shared__ Sym16Lds<RT> sh;
  const int lane = threadIdx.x;
  const int64_t g = blockIdx.x;
  const int c = blockIdx.y;
  const int r0 = blockIdx.z * RT;  // right-hand sides r0 .. r0 + RT - 1 (those >= R repeat R - 1, unstored)
  const int d0 = c * dpc;
  const int d1 = min(Dmax + 1, d0 + dpc);
  const float* lsrc[3] = {l0, l1, l2};
  int rof[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) rof[rr] = min(r0 + rr, R - 1);

  // targets: lane l of tile m is point g*256 + 64 m + l; lanes past N are idle (tb = -1, zero charge)
  int tb[kSymTiles];
  float lt[kSymTiles][3], qtr[kSymTiles][RT], qti[kSymTiles][RT];
  double ar[kSymTiles][RT], ai[kSymTiles][RT];
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t = g * kSymGroup + 64 * m + lane;
    const bool ok = t < N;
    const int64_t tc = ok ? t : 0;
    tb[m] = ok ? body_of[tc] : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) lt[m][d] = ok ? lsrc[d][tc] : 0.0f;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const c64 qq = q[(int64_t)rof[rr] * N + tc];
      qtr[m][rr] = ok ? qq.re : 0.0f;
      qti[m][rr] = ok ? qq.im : 0.0f;
      ar[m][rr] = ai[m][rr] = 0.0;
    }
  }

  for (int d = d0; d < d1; ++d) {
    int64_t h = g + d;
    if (h >= G) h -= G;
    const bool sym = d != 0 && !(even_G && d == Dmax);
    for (int ts = 0; ts < kSymTiles; ++ts) {
      const int64_t j0 = h * kSymGroup + 64 * ts;
      if (j0 >= N) break;
      int sbb[4];  // body of each sub-block of the source tile, -1 past N (wave-uniform)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        sbb[u] = j0 + kSubBlock * u < N ? __builtin_amdgcn_readfirstlane(body_of[j0 + kSubBlock * u]) : -1;
      // stage the source tile: lane 16 u + i holds source j0 + 16 u + i at entries u*48 + i and + 16.
      // Idle slots: zero offset and charge, |l|^2 = 1 so that no distance is zero
      {
        const int64_t j = j0 + lane;
        const bool ok = j < N;
        const int64_t jc = ok ? j : 0;
        const int e = (lane >> 4) * kSubStride + (lane & 15);
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) sh.l[dd][e] = sh.l[dd][e + kSubBlock] = ok ? lsrc[dd][jc] : 0.0f;
        sh.bs[e] = sh.bs[e + kSubBlock] = ok ? lsq[jc] : 1.0f;
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          const c64 qq = q[(int64_t)rof[rr] * N + jc];
          sh.qr[rr][e] = sh.qr[rr][e + kSubBlock] = ok ? qq.re : 0.0f;
          sh.qi[rr][e] = sh.qi[rr][e + kSubBlock] = ok ? qq.im : 0.0f;
        }
      }
      __syncthreads();
      // is any pair of this meeting on one body?  (then the per-tile path with the same-body test)
      bool clash = false;
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int u = 0; u < 4; ++u) clash = clash || (tb[m] >= 0 && tb[m] == sbb[u]);
      const bool any_clash = __any(clash);
      const bool pure = sbb[0] >= 0 && sbb[1] == sbb[0] && sbb[2] == sbb[0] && sbb[3] == sbb[0];
      float tr[kSymTiles][RT], ti[kSymTiles][RT];
      float sr[RT], si[RT];  // lane l: source-side sums of source j0 + l (after the tile)
#pragma unroll
      for (int rr = 0; rr < RT; ++rr) {
        sr[rr] = si[rr] = 0.0f;
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) tr[m][rr] = ti[m][rr] = 0.0f;
      }
      if (!any_clash) {
        if (sym) sym16_steps4<RT, true>(sh, k, CentresGlobal{cen}, lane, tb, sbb, pure, lt, qtr, qti, tr, ti, sr, si);
        else sym16_steps4<RT, false>(sh, k, CentresGlobal{cen}, lane, tb, sbb, pure, lt, qtr, qti, tr, ti, sr, si);
      } else {
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) {
          if (g * kSymGroup + 64 * m >= N) continue;  // a tile with no targets
          if (sym) sym16_steps1<RT, true>(sh, k, CentresGlobal{cen}, lane, tb[m], sbb, lt[m], qtr[m], qti[m], tr[m], ti[m], sr, si);
          else sym16_steps1<RT, false>(sh, k, CentresGlobal{cen}, lane, tb[m], sbb, lt[m], qtr[m], qti[m], tr[m], ti[m], sr, si);
        }
      }
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          ar[m][rr] += (double)tr[m][rr];
          ai[m][rr] += (double)ti[m][rr];
        }
      // source-side sums of this tile from the wave's targets -> slice of distance d
      if (sym && j0 + lane < N) {
#pragma unroll
        for (int rr = 0; rr < RT; ++rr)
          if (r0 + rr < R)
            partial[((int64_t)(nchunks_d + d - 1) * R + r0 + rr) * N + j0 + lane] =
                c64{sr[rr] * kInv4Pi, si[rr] * kInv4Pi};
      }
      __syncthreads();  // the tile's entries are read before the next tile is staged
    }
  }
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t = g * kSymGroup + 64 * m + lane;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
      if (t < N && r0 + rr < R)
        partial[((int64_t)c * R + r0 + rr) * N + t] =
            c64{(float)(ar[m][rr] * (double)kInv4Pi), (float)(ai[m][rr] * (double)kInv4Pi)};
  }
}

// The sub-block pair sum with W waves per block sharing each staged source tile, its bodies and
// their centres, and each wave's target-body centres in LDS (the schedule of
// ghat_sym_shared_kernel).
template <int RT, int W>
__global__ __launch_bounds__(64 * W, SymWaves<RT>::value) void ghat_sym16_shared_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of,
    const c64* __restrict__ q, int64_t N, int R, int64_t G, int Dmax, int even_G, int HH, int dpc, int nchunks_d,
    c64* __restrict__ partial) {
  static_assert(W > 1, "one wave per block: ghat_sym16_kernel");
  __shared__ Sym16Lds<RT> sh[2];
  __shared__ SymComb<RT, W> cb;
  __shared__ double tcen[W][kSymGroup / kSubBlock][3];  // centres of each wave's target bodies
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t gb = (int64_t)blockIdx.x * W;  // the block's first target group
  const int64_t g = gb + wv;                        // this wave's
  const int c = blockIdx.y;
  const int r0 = blockIdx.z * RT;  // right-hand sides r0 .. r0 + RT - 1 (those >= R repeat R - 1, unstored)
  const int hh1 = min(HH, (c + 1) * dpc);
  const float* lsrc[3] = {l0, l1, l2};
  int rof[RT];
#pragma unroll
  for (int rr = 0; rr < RT; ++rr) rof[rr] = min(r0 + rr, R - 1);

  // targets: lane l of tile m is point g*256 + 64 m + l; lanes past N are idle (tb = -1, zero charge)
  int tb[kSymTiles];
  float lt[kSymTiles][3], qtr[kSymTiles][RT], qti[kSymTiles][RT];
  double ar[kSymTiles][RT], ai[kSymTiles][RT];
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t = g * kSymGroup + 64 * m + lane;
    const bool ok = t < N;
    const int64_t tc = ok ? t : 0;
    tb[m] = ok ? body_of[tc] : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) lt[m][d] = ok ? lsrc[d][tc] : 0.0f;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const c64 qq = q[(int64_t)rof[rr] * N + tc];
      qtr[m][rr] = ok ? qq.re : 0.0f;
      qti[m][rr] = ok ? qq.im : 0.0f;
      ar[m][rr] = ai[m][rr] = 0.0;
    }
  }
  const bool has_targets = g * kSymGroup < N;
  // the wave's targets lie on bodies tbase .. tlast, at most 16 of them (every body holds a
  // multiple of 16 points and starts on a 16-point boundary)
  const int tbase = has_targets ? body_of[g * kSymGroup] : 0;
  if (has_targets) {
    const int tlast = body_of[min(N, (g + 1) * kSymGroup) - 1];
    if (lane < 3 * (tlast - tbase + 1))
      tcen[wv][lane / 3][lane % 3] = cen[(int64_t)(tbase + lane / 3) * 3 + lane % 3];
  }

  // The tile walk and the per-tile barrier of ghat_sym_kernel.
  // source j0 + p sits at entries (p / 16) * 48 + p % 16 and + 16 of the staging arrays
  int hh = c * dpc, ts = 0, t = 0, buf = 0, psl = 0;
  int64_t pj0 = 0;
  bool have = sym_seek(gb, G, N, hh1, hh, ts);
  SymStage<3, RT, W> stg;
  if (have) {
    sym_stage_load(stg, l0, l1, l2, lsq, q, rof, N, sym_tile_start(gb, G, hh, ts), wv, lane);
    sym_stage_store<4 * kSubStride, kSubBlock, true>(stg, &sh[0].l[0][0], wv, lane);
    if (wv == 0) sym16_stage_meta(sh[0], cen, body_of, N, sym_tile_start(gb, G, hh, ts), lane);
  }
  while (have) {
    const int64_t j0 = sym_tile_start(gb, G, hh, ts);
    __syncthreads();  // tile t staged in buffer t & 1; every wave's sums of tile t - 1 in cb
    int nhh = hh, nts = ts + 1;
    const bool nhave = sym_seek(gb, G, N, hh1, nhh, nts);
    if (nhave) sym_stage_load(stg, l0, l1, l2, lsq, q, rof, N, sym_tile_start(gb, G, nhh, nts), wv, lane);
    // wave (t - 1) mod W adds the waves' sums of the previous tile and stages the next tile's
    // bodies and centres (every wave is past its last read of that buffer: the barrier)
    if (wv == (t + W - 1) % W) {
      if (t > 0) sym_combine(cb, buf ^ 1, lane, pj0, N, R, r0, nchunks_d + psl, kInv4Pi, partial);
      if (nhave) sym16_stage_meta(sh[buf ^ 1], cen, body_of, N, sym_tile_start(gb, G, nhh, nts), lane);
    }
    const int d = hh - wv;
    const bool active = has_targets && d >= 0 && d <= Dmax;
    const bool sym = active && d != 0 && !(even_G && d == Dmax);
    float sr[RT], si[RT];  // lane l: source-side sums of source j0 + l (after the tile)
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) sr[rr] = si[rr] = 0.0f;
    if (active) {
      int sbb[4];  // body of each sub-block of the source tile, -1 past N (wave-uniform)
#pragma unroll
      for (int u = 0; u < 4; ++u) sbb[u] = __builtin_amdgcn_readfirstlane(sh[buf].sbb[u]);
      // is any pair of this meeting on one body?  (then the per-tile path with the same-body test)
      bool clash = false;
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int u = 0; u < 4; ++u) clash = clash || (tb[m] >= 0 && tb[m] == sbb[u]);
      const bool any_clash = __any(clash);
      const bool pure = sbb[0] >= 0 && sbb[1] == sbb[0] && sbb[2] == sbb[0] && sbb[3] == sbb[0];
      float tr[kSymTiles][RT], ti[kSymTiles][RT];
#pragma unroll
      for (int rr = 0; rr < RT; ++rr)
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) tr[m][rr] = ti[m][rr] = 0.0f;
      if (!any_clash) {
        if (sym) sym16_steps4<RT, true>(sh[buf], k, CentresLds<RT>{tcen[wv], tbase, &sh[buf]}, lane, tb, sbb, pure, lt, qtr, qti, tr, ti, sr, si);
        else sym16_steps4<RT, false>(sh[buf], k, CentresLds<RT>{tcen[wv], tbase, &sh[buf]}, lane, tb, sbb, pure, lt, qtr, qti, tr, ti, sr, si);
      } else {
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) {
          if (g * kSymGroup + 64 * m >= N) continue;  // a tile with no targets
          if (sym)
            sym16_steps1<RT, true>(sh[buf], k, CentresLds<RT>{tcen[wv], tbase, &sh[buf]}, lane, tb[m], sbb, lt[m], qtr[m], qti[m], tr[m], ti[m], sr, si);
          else
            sym16_steps1<RT, false>(sh[buf], k, CentresLds<RT>{tcen[wv], tbase, &sh[buf]}, lane, tb[m], sbb, lt[m], qtr[m], qti[m], tr[m], ti[m], sr, si);
        }
      }
#pragma unroll
      for (int m = 0; m < kSymTiles; ++m)
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
          ar[m][rr] += (double)tr[m][rr];
          ai[m][rr] += (double)ti[m][rr];
        }
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {  // zero where this wave formed no symmetric pair with the tile
      cb.re[buf][wv][rr][lane] = sym ? sr[rr] : 0.0f;
      cb.im[buf][wv][rr][lane] = sym ? si[rr] : 0.0f;
    }
    if (nhave) sym_stage_store<4 * kSubStride, kSubBlock, true>(stg, &sh[buf ^ 1].l[0][0], wv, lane);
    pj0 = j0;
    psl = hh / W;
    buf ^= 1;
    ++t;
    hh = nhh;
    ts = nts;
    have = nhave;
  }
  __syncthreads();
  if (t > 0 && wv == (t - 1) % W) sym_combine(cb, buf ^ 1, lane, pj0, N, R, r0, nchunks_d + psl, kInv4Pi, partial);
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t = g * kSymGroup + 64 * m + lane;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
      if (t < N && r0 + rr < R)
        partial[((int64_t)c * R + r0 + rr) * N + t] =
            c64{(float)(ar[m][rr] * (double)kInv4Pi), (float)(ai[m][rr] * (double)kInv4Pi)};
  }
}


// ---------------------------------------------------------------------------
// FP64 symmetric pair sum in 3D, one right-hand side (the refinement residual of the mixed solve): the
// block schedule of ghat_sym_shared_kernel (W waves, each holding one target group of 256 points,
// sharing each staged source tile), with phi in FP64 from the absolute coordinates (no body-centre
// split) and same-body pairs removed pair by pair, so bodies of any size work and tiles may
// straddle them.  Idle target lanes and source slots (past N) carry body -1 and are masked too.
// Outputs as ghat_sym_shared_kernel's, complex128.
// ---------------------------------------------------------------------------
template <int DIM>
struct SymLds64 {
  double x[DIM][128];
  double qr[128], qi[128];
  int b[128];
};

// lane l receives lane (l + 1) mod 64's value (DPP wave_rol:1 on both halves)
__device__ __forceinline__ double wave_rotate_next_d(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, 0x134, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0x134, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <int DIM, int W>
__global__ __launch_bounds__(64 * W) void ghat_sym_f64_kernel(double kappa, const double* __restrict__ x0,
                                                              const double* __restrict__ x1,
                                                              const double* __restrict__ x2,
                                                              const int32_t* __restrict__ body_of,
                                                              const c128* __restrict__ q, int64_t N, int64_t G,
                                                              int Dmax, int even_G, int HH, int dpc, int nchunks_d,
                                                              c128* __restrict__ partial) {
  __shared__ SymLds64<DIM> sh[2];
  __shared__ double cbr[2][W][64], cbi[2][W][64];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t gb = (int64_t)blockIdx.x * W;
  const int64_t g = gb + wv;
  const int c = blockIdx.y;
  const int hh1 = min(HH, (c + 1) * dpc);
  const double* xs[3] = {x0, x1, x2};
  PhiEval<double, DIM> phi{kappa};

  int tb[kSymTiles];
  double tx[kSymTiles][DIM], tqr[kSymTiles], tqi[kSymTiles], ar[kSymTiles], ai[kSymTiles];
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t t = g * kSymGroup + 64 * m + lane;
    const bool ok = t < N;
    const int64_t tc = ok ? t : 0;
    tb[m] = ok ? body_of[tc] : -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) tx[m][d] = xs[d][tc];
    tqr[m] = ok ? q[tc].re : 0.0;
    tqi[m] = ok ? q[tc].im : 0.0;
    ar[m] = ai[m] = 0.0;
  }
  const bool has_targets = g * kSymGroup < N;

  // one barrier per tile: tile t staged in buffer t & 1 before it; the previous tile's sums added
  // after it by wave (t - 1) mod W
  int hh = c * dpc, ts = 0, t = 0, buf = 0, psl = 0;
  int64_t pj0 = 0;
  bool have = sym_seek(gb, G, N, hh1, hh, ts);
  while (have) {
    const int64_t j0 = sym_tile_start(gb, G, hh, ts);
    if (lane < 64 / W) {  // stage the tile, 64 / W sources per wave, entries e and e + 64
      const int e = (64 / W) * wv + lane;
      const int64_t j = j0 + e;
      const bool ok = j < N;
      const int64_t jc = ok ? j : 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) sh[buf].x[d][e] = sh[buf].x[d][e + 64] = xs[d][jc];
      const c128 qq = q[jc];
      sh[buf].qr[e] = sh[buf].qr[e + 64] = ok ? qq.re : 0.0;
      sh[buf].qi[e] = sh[buf].qi[e + 64] = ok ? qq.im : 0.0;
      sh[buf].b[e] = sh[buf].b[e + 64] = ok ? body_of[jc] : -1;
    }
    __syncthreads();
    if (t > 0 && wv == (t - 1) % W && pj0 + lane < N) {
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        xr += cbr[buf ^ 1][w][lane];
        xi += cbi[buf ^ 1][w][lane];
      }
      partial[(int64_t)(nchunks_d + psl) * N + pj0 + lane] = c128{xr, xi};
    }
    const int d = hh - wv;
    const bool active = has_targets && d >= 0 && d <= Dmax;
    const bool sym = active && d != 0 && !(even_G && d == Dmax);
    double sr = 0.0, si = 0.0;  // running source-side sum of the source this lane meets
    if (active) {
      const SymLds64<DIM>& S = sh[buf];
      for (int s0 = 0; s0 < 64; ++s0) {
        const int e = lane + s0;
        double sx[DIM];
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) sx[dd] = S.x[dd][e];
        const double sqr = S.qr[e], sqi = S.qi[e];
        const int sb = S.b[e];
#pragma unroll
        for (int m = 0; m < kSymTiles; ++m) {
          double r2 = 0.0;
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) {
            const double dx = tx[m][dd] - sx[dd];
            r2 = fma(dx, dx, r2);
          }
          double pr, pi;
          phi(r2, pr, pi);
          const bool ok = tb[m] >= 0 && sb >= 0 && tb[m] != sb;  // a select: drops the values of
          pr = ok ? pr : 0.0;                                    // a point with itself too
          pi = ok ? pi : 0.0;
          ar[m] = fma(pr, sqr, fma(-pi, sqi, ar[m]));
          ai[m] = fma(pr, sqi, fma(pi, sqr, ai[m]));
          if (sym) {
            sr = fma(pr, tqr[m], fma(-pi, tqi[m], sr));
            si = fma(pr, tqi[m], fma(pi, tqr[m], si));
          }
        }
        sr = wave_rotate_next_d(sr);
        si = wave_rotate_next_d(si);
      }
    }
    cbr[buf][wv][lane] = sym ? sr : 0.0;
    cbi[buf][wv][lane] = sym ? si : 0.0;
    pj0 = j0;
    psl = hh / W;
    buf ^= 1;
    ++t;
    ++ts;
    have = sym_seek(gb, G, N, hh1, hh, ts);
  }
  __syncthreads();
  if (t > 0 && wv == (t - 1) % W && pj0 + lane < N) {
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      xr += cbr[buf ^ 1][w][lane];
      xi += cbi[buf ^ 1][w][lane];
    }
    partial[(int64_t)(nchunks_d + psl) * N + pj0 + lane] = c128{xr, xi};
  }
#pragma unroll
  for (int m = 0; m < kSymTiles; ++m) {
    const int64_t tt = g * kSymGroup + 64 * m + lane;
    if (tt < N) partial[(int64_t)c * N + tt] = c128{ar[m], ai[m]};
  }
}

template <typename T, int DIM, int TPT, int RT, bool EXT>
hipError_t launch_pair(const PhiEval<T, DIM>& phi, const T* s0, const T* s1, const T* s2, const int32_t* sbody,
                       const int64_t* body_ptr, const Cplx<T>* q, int64_t N, int R, const double* targets,
                       const double* origin, int64_t M, Cplx<T>* partial, int nchunks, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int64_t chunk_len = (N + nchunks - 1) / nchunks;
  chunk_len = (chunk_len + kUnroll - 1) / kUnroll * kUnroll;
  const int64_t per_block = (int64_t)kBlock * TPT;
  dim3 grid((unsigned)((M + per_block - 1) / per_block), (unsigned)nchunks, (unsigned)((R + RT - 1) / RT));
  hipLaunchKernelGGL((pair_sum_kernel<T, DIM, TPT, RT, EXT>), grid, dim3(kBlock), 0, st, phi, s0, s1, s2,
                     sbody, body_ptr, q, N, R, targets, origin[0], origin[1], origin[2], M, chunk_len,
                     partial);
  return hipGetLastError();
}

template <typename T, int DIM, int TPT, bool EXT>
hipError_t dispatch_rt(const PhiEval<T, DIM>& phi, const T* s0, const T* s1, const T* s2, const int32_t* sbody,
                       const int64_t* body_ptr, const Cplx<T>* q, int64_t N, int R, const double* targets,
                       const double* origin, int64_t M, Cplx<T>* partial, int nchunks, hipStream_t st) {
  if (R == 1)
    return launch_pair<T, DIM, TPT, 1, EXT>(phi, s0, s1, s2, sbody, body_ptr, q, N, R, targets, origin, M,
                                            partial, nchunks, st);
  if (R == 2)
    return launch_pair<T, DIM, TPT, 2, EXT>(phi, s0, s1, s2, sbody, body_ptr, q, N, R, targets, origin, M,
                                            partial, nchunks, st);
  return launch_pair<T, DIM, TPT, 4, EXT>(phi, s0, s1, s2, sbody, body_ptr, q, N, R, targets, origin, M,
                                          partial, nchunks, st);
}

}  // namespace

int pair_chunks_for(int64_t n_sources, int64_t n_targets, int tpt) {
  // aim for ~16 waves per SIMD (256 CUs x 4 SIMDs) while keeping chunks >= 64 sources; small
  // systems thus still spread over the chip (N = 8192: 64 chunks, 4096 waves)
  const int64_t waves = (n_targets + 64 * tpt - 1) / (64 * tpt);
  int64_t want = (16384 + waves - 1) / std::max<int64_t>(waves, 1);
  want = std::min<int64_t>(want, std::max<int64_t>(1, n_sources / 64));
  want = std::max<int64_t>(1, std::min<int64_t>(want, 128));
  return (int)want;
}

static const double kZero3[3] = {0.0, 0.0, 0.0};


template <int DIM, int RT>
static hipError_t launch_bodyphase(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks,
                                   hipStream_t st) {
  constexpr int TPT = 2;
  int64_t chunk_len = (s.N + nchunks - 1) / nchunks;
  chunk_len = (chunk_len + kUnroll - 1) / kUnroll * kUnroll;
  const int64_t per_block = (int64_t)kBlock * TPT;
  dim3 grid((unsigned)((s.N + per_block - 1) / per_block), (unsigned)nchunks, (unsigned)((R + RT - 1) / RT));
  hipLaunchKernelGGL((ghat_bodyphase_kernel<DIM, TPT, RT>), grid, dim3(kBlock), 0, st, make_bodyphase(s.kappa, s.rho_max),
                     s.l32[0], s.l32[1], s.l32[2], s.lsq32, s.centres, s.body_of, s.body_ptr, q, s.N, R, chunk_len,
                     partial);
  return hipGetLastError();
}



int ghat_default_rt(int R) { return R == 1 ? 1 : R == 2 ? 2 : 4; }

SymPlan sym_plan(int64_t N, int nchunks_d, int W) {
  SymPlan p{};
  p.W = W;
  const int64_t G0 = (N + kSymGroup - 1) / kSymGroup;
  p.G = (G0 + W - 1) / W * W;
  p.Dmax = (int)(p.G / 2);
  p.even = p.G % 2 == 0;
  // one wave per block: distances 0 .. Dmax; W waves: offsets 0 .. HH - 1, wave w meeting distance
  // hh - w, so that every wave reaches Dmax
  p.HH = W == 1 ? p.Dmax + 1 : (p.Dmax + W + W - 1) / W * W;
  // heuristic: about 64k waves (63 chunks on the 2000-starfish scene, 42 on the 1000 spheres)
  int want = nchunks_d > 0 ? nchunks_d : (int)std::min<int64_t>(kTuneMaxChunks, (65536 + p.G - 1) / std::max<int64_t>(p.G, 1));
  want = std::max(1, std::min(want, p.HH));
  p.dpc = (p.HH + want - 1) / want;
  p.nchunks_d = (p.HH + p.dpc - 1) / p.dpc;  // no empty chunks
  // source-side slices: one per symmetric distance (1 .. Dmax, less Dmax itself for even G), or one
  // per W block offsets
  const int dsym = std::max(0, p.even ? p.Dmax - 1 : p.Dmax);
  p.slices = p.nchunks_d + (W == 1 ? dsym : p.HH / W);
  return p;
}

namespace {
std::atomic<int64_t> g_sym_slice_budget{0};  // <= 0: kSymSliceBudget
}

int64_t sym_slice_budget(int64_t bytes) {
  return g_sym_slice_budget.exchange(bytes);
}

int sym_block_waves(int64_t NP, int R) {
  int64_t budget = g_sym_slice_budget.load();
  if (budget <= 0) budget = kSymSliceBudget;
  const SymPlan p = sym_plan(NP, 0, 1);
  return (double)p.slices * (double)NP * (double)R * sizeof(c64) <= (double)budget ? 1 : kSymW;
}

bool ghat_sym_possible(const SceneDev& s, int R) {
  // up to 32 right-hand sides: the matrix-core kernel works on tiles of 64 of them, so below 32 most
  // of its products are on zero padding and the symmetric VALU kernel does less work
  if (R < 1 || R > kSymMaxRhs || s.N <= 0) return false;
  int64_t NP = s.N;
  if (sym_padded(s)) {
    // padded to whole tiles: worth it while the padded pair count stays below 1.4 times the real one
    // (the symmetric kernel does about 0.6 times the plain kernel's work per pair)
    if (!s.pad_ptr || (double)s.Npad * (double)s.Npad > 1.4 * (double)s.N * (double)s.N) return false;
    NP = s.Npad;
  }
  const SymPlan p = sym_plan(NP, 0, sym_block_waves(NP, R));
  // the source-side slices grow as N^2 / (512 W) per right-hand side: keep them within 8 GiB
  return (double)p.slices * (double)NP * (double)R * sizeof(c64) <= 8.0 * (1ull << 30);
}

bool sym_padded(const SceneDev& s) { return !s.all_k_mult64 && !s.sym16; }

SceneDev sym_view(const SceneDev& s) {
  if (!sym_padded(s)) return s;
  SceneDev v = s;
  v.N = s.Npad;
  for (int d = 0; d < 3; ++d) v.l32[d] = s.l32p[d];
  v.lsq32 = s.lsqp;
  v.body_of = s.body_of_pad;
  v.body_ptr = s.pad_ptr;
  v.all_k_mult64 = true;
  return v;
}

template <int DIM, int RT, int W>
static void launch_sym(const SceneDev& s, const SymPlan& p, const c64* q, int R, c64* partial, hipStream_t st) {
  const dim3 grid((unsigned)(p.G / W), (unsigned)p.nchunks_d, (unsigned)((R + RT - 1) / RT));
  const BodyPhaseConsts k = make_bodyphase(s.kappa, s.rho_max);
  if constexpr (W == 1)
    hipLaunchKernelGGL((ghat_sym_kernel<DIM, RT>), grid, dim3(64), 0, st, k, s.l32[0], s.l32[1], s.l32[2], s.lsq32,
                       s.centres, s.body_of, q, s.N, R, p.G, p.Dmax, p.even ? 1 : 0, p.dpc, p.nchunks_d, partial);
  else
    hipLaunchKernelGGL((ghat_sym_shared_kernel<DIM, RT, W>), grid, dim3(64 * W), 0, st, k, s.l32[0], s.l32[1],
                       s.l32[2], s.lsq32, s.centres, s.body_of, q, s.N, R, p.G, p.Dmax, p.even ? 1 : 0, p.HH, p.dpc,
                       p.nchunks_d, partial);
}

template <int RT, int W>
static void launch_sym16(const SceneDev& s, const SymPlan& p, const c64* q, int R, c64* partial, hipStream_t st) {
  const dim3 grid((unsigned)(p.G / W), (unsigned)p.nchunks_d, (unsigned)((R + RT - 1) / RT));
  const BodyPhaseConsts k = make_bodyphase(s.kappa, s.rho_max);
  if constexpr (W == 1)
    hipLaunchKernelGGL((ghat_sym16_kernel<RT>), grid, dim3(64), 0, st, k, s.l32[0], s.l32[1], s.l32[2], s.lsq32,
                       s.centres, s.body_of, q, s.N, R, p.G, p.Dmax, p.even ? 1 : 0, p.dpc, p.nchunks_d, partial);
  else
    hipLaunchKernelGGL((ghat_sym16_shared_kernel<RT, W>), grid, dim3(64 * W), 0, st, k, s.l32[0], s.l32[1],
                       s.l32[2], s.lsq32, s.centres, s.body_of, q, s.N, R, p.G, p.Dmax, p.even ? 1 : 0, p.HH, p.dpc,
                       p.nchunks_d, partial);
}

template <int W>
static void launch_sym_w(const SceneDev& s, const SymPlan& p, const c64* q, int R, c64* partial, int rt,
                         hipStream_t st) {
  if (s.sym16) {  // 3D, bodies of 16 n points: tiles may straddle bodies
    if (rt == 1) launch_sym16<1, W>(s, p, q, R, partial, st);
    else if (rt == 2) launch_sym16<2, W>(s, p, q, R, partial, st);
    else launch_sym16<4, W>(s, p, q, R, partial, st);
  } else if (s.dim == 2) {
    if (rt == 1) launch_sym<2, 1, W>(s, p, q, R, partial, st);
    else if (rt == 2) launch_sym<2, 2, W>(s, p, q, R, partial, st);
    else launch_sym<2, 4, W>(s, p, q, R, partial, st);
  } else {
    if (rt == 1) launch_sym<3, 1, W>(s, p, q, R, partial, st);
    else if (rt == 2) launch_sym<3, 2, W>(s, p, q, R, partial, st);
    else launch_sym<3, 4, W>(s, p, q, R, partial, st);
  }
}

hipError_t launch_ghat_f32_sym(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks_d, int rt,
                               hipStream_t st) {
  if (s.N <= 0) return hipSuccess;
  const int W = sym_block_waves(s.N, R);
  const SymPlan p = sym_plan(s.N, nchunks_d, W);
  if (rt != 1 && rt != 2 && rt != 4) rt = ghat_default_rt(R);
  if (W == 1) launch_sym_w<1>(s, p, q, R, partial, rt, st);
  else launch_sym_w<kSymW>(s, p, q, R, partial, rt, st);
  return hipGetLastError();
}

hipError_t launch_ghat_f32(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks, hipStream_t st,
                           int rt, void* split) {
  if (s.N <= 0) return hipSuccess;
  if (ghat_uses_mfma(s, R)) return launch_ghat_mc(s, q, R, partial, nchunks, split, st);
  if (rt != 1 && rt != 2 && rt != 4) rt = ghat_default_rt(R);
  if (s.dim == 2) {
    if (rt == 1) return launch_bodyphase<2, 1>(s, q, R, partial, nchunks, st);
    if (rt == 2) return launch_bodyphase<2, 2>(s, q, R, partial, nchunks, st);
    return launch_bodyphase<2, 4>(s, q, R, partial, nchunks, st);
  }
  if (rt == 1) return launch_bodyphase<3, 1>(s, q, R, partial, nchunks, st);
  if (rt == 2) return launch_bodyphase<3, 2>(s, q, R, partial, nchunks, st);
  return launch_bodyphase<3, 4>(s, q, R, partial, nchunks, st);
}

// waves per block of the FP64 symmetric kernel: one per SIMD (its registers allow 2 or 3 per SIMD,
// so blocks of 8 would leave one block per CU)
constexpr int kSymW64 = 4;

// 3D only: the 2D kernel's FP64 Hankel branches, four targets per lane, take every register of a
// SIMD (one wave), so the plain kernel stays the faster there
bool ghat_f64_sym(const SceneDev& s, int R) { return s.dim == 3 && R == 1 && s.N > 0; }

int ghat_f64_slices(const SceneDev& s, int R, int nchunks) {
  return ghat_f64_sym(s, R) ? sym_plan(s.N, 0, kSymW64).slices : nchunks;
}

hipError_t launch_ghat_f64(const SceneDev& s, const c128* q, int R, c128* partial, int nchunks, hipStream_t st,
                           bool allow_sym) {
  if (s.N <= 0) return hipSuccess;
  if (ghat_uses_mfma(s, R)) return launch_ghat_mc64(s, q, R, partial, nchunks, st);
  if (allow_sym && ghat_f64_sym(s, R)) {
    const SymPlan p = sym_plan(s.N, 0, kSymW64);
    const dim3 grid((unsigned)(p.G / kSymW64), (unsigned)p.nchunks_d, 1);
    hipLaunchKernelGGL((ghat_sym_f64_kernel<3, kSymW64>), grid, dim3(64 * kSymW64), 0, st, s.kappa, s.x64[0],
                       s.x64[1], s.x64[2], s.body_of, q, s.N, p.G, p.Dmax, p.even ? 1 : 0, p.HH, p.dpc, p.nchunks_d,
                       partial);
    return hipGetLastError();
  }
  if (s.dim == 2) {
    PhiEval<double, 2> phi{s.kappa};
    return dispatch_rt<double, 2, 1, false>(phi, s.x64[0], s.x64[1], nullptr, s.body_of, s.body_ptr, q, s.N, R,
                                            nullptr, kZero3, s.N, partial, nchunks, st);
  }
  PhiEval<double, 3> phi{s.kappa};
  return dispatch_rt<double, 3, 1, false>(phi, s.x64[0], s.x64[1], s.x64[2], s.body_of, s.body_ptr, q, s.N, R,
                                          nullptr, kZero3, s.N, partial, nchunks, st);
}

hipError_t launch_eval_f32(const SceneDev& s, const c64* q, int R, const double* targets, int64_t M, c64* partial,
                           int nchunks, hipStream_t st) {
  if (s.dim == 2) {
    PhiEval<float, 2> phi{make_phi2d_f32(s.kappa)};
    return dispatch_rt<float, 2, 2, true>(phi, s.x32[0], s.x32[1], nullptr, s.body_of, s.body_ptr, q, s.N, R,
                                          targets, s.origin, M, partial, nchunks, st);
  }
  PhiEval<float, 3> phi{Phi3DConstsF32{(float)(s.kappa / (2.0 * M_PI))}};
  return dispatch_rt<float, 3, 2, true>(phi, s.x32[0], s.x32[1], s.x32[2], s.body_of, s.body_ptr, q, s.N, R,
                                        targets, s.origin, M, partial, nchunks, st);
}

hipError_t launch_eval_f64(const SceneDev& s, const c128* q, int R, const double* targets, int64_t M,
                           c128* partial, int nchunks, hipStream_t st) {
  if (s.dim == 2) {
    PhiEval<double, 2> phi{s.kappa};
    return dispatch_rt<double, 2, 1, true>(phi, s.x64[0], s.x64[1], nullptr, s.body_of, s.body_ptr, q, s.N, R,
                                           targets, kZero3, M, partial, nchunks, st);
  }
  PhiEval<double, 3> phi{s.kappa};
  return dispatch_rt<double, 3, 1, true>(phi, s.x64[0], s.x64[1], s.x64[2], s.body_of, s.body_ptr, q, s.N, R,
                                         targets, kZero3, M, partial, nchunks, st);
}

// ----------------------------------------------------------- chunk reduce ---
template <typename T>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const Cplx<T>* __restrict__ partial, int nchunks,
                                                              int64_t MR, Cplx<T>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MR) return;
  double re = 0, im = 0;  // many slices (symmetric kernel): add them in FP64
  for (int c = 0; c < nchunks; ++c) {
    const Cplx<T> v = partial[(int64_t)c * MR + i];
    re += (double)v.re;
    im += (double)v.im;
  }
  out[i] = Cplx<T>{(T)re, (T)im};
}

__global__ __launch_bounds__(256) void reduce_partials_padded_kernel(const c64* __restrict__ partial, int nchunks,
                                                                      const int32_t* __restrict__ body_of,
                                                                      const int64_t* __restrict__ body_ptr,
                                                                      const int64_t* __restrict__ pad_ptr, int64_t N,
                                                                      int64_t NP, int R, c64* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const int b = body_of[i];
  const int64_t ip = pad_ptr[b] + (i - body_ptr[b]);
  double re = 0, im = 0;
  for (int c = 0; c < nchunks; ++c) {
    const c64 v = partial[((int64_t)c * R + r) * NP + ip];
    re += (double)v.re;
    im += (double)v.im;
  }
  out[(int64_t)r * N + i] = c64{(float)re, (float)im};
}

hipError_t launch_reduce_partials_padded(const SceneDev& s, const c64* partial, int nchunks, int R, c64* out,
                                         hipStream_t st) {
  if (s.N == 0 || R == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_padded_kernel, dim3((unsigned)((s.N + 255) / 256), (unsigned)R), dim3(256), 0, st,
                     partial, nchunks, s.body_of, s.body_ptr, s.pad_ptr, s.N, s.Npad, R, out);
  return hipGetLastError();
}

hipError_t launch_reduce_partials_f32(const c64* partial, int nchunks, int64_t M, int R, c64* out, hipStream_t st) {
  const int64_t MR = M * R;
  if (MR == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel<float>, dim3((unsigned)((MR + 255) / 256)), dim3(256), 0, st, partial,
                     nchunks, MR, out);
  return hipGetLastError();
}

hipError_t launch_reduce_partials_f64(const c128* partial, int nchunks, int64_t M, int R, c128* out,
                                      hipStream_t st) {
  const int64_t MR = M * R;
  if (MR == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3((unsigned)((MR + 255) / 256)), dim3(256), 0, st, partial,
                     nchunks, MR, out);
  return hipGetLastError();
}

}  // namespace mfs
