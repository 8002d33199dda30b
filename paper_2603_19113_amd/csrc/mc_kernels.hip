// Pair sums with many right-hand sides on the matrix cores: T = G_hat Q for Q [R][N], R >= 8, every
// body a multiple of 16 points.  Two forms: FP32 products (v_mfma_f32_16x16x4f32) and FP16 products
// of split operands (v_mfma_f32_16x16x32_f16), both with the body-centre split of the distance.
#include <cmath>
#include <type_traits>

#include "mfs_internal.h"
#include "bodyphase.h"

namespace mfs {

// ---------------------------------------------------------------------------
// Many right-hand sides: T = G_hat Q, Q [R][N], on the matrix cores.
//
// A block of 4 waves owns 64 targets and 64 right-hand sides.  Sources are taken 16 at a time:
//   * the block stages the charge tile Q(16 sources x 64 RHS) in LDS, transposed so that the
//     B operand of the MFMA is read without bank conflicts;
//   * each wave evaluates phi for its 16 targets x 16 sources with the same body-centre phase
//     split as the single-RHS kernel, directly in the A-operand layout of
//     v_mfma_f32_16x16x4f32 (lane l holds row l%16, k = l/16), so phi never goes through LDS;
//   * the complex product is four real MFMAs per (k-step, 16-RHS block):
//     Tr += Gr Qr - Gi Qi, Ti += Gr Qi + Gi Qr.
// FP32 MFMA accumulators are added into FP64 every 16 tiles (256 sources).  Requires every body
// to hold a multiple of 16 points, so that a 16-source tile lies in one body.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kMfmaTargets = 64;   // per block (16 per wave)
constexpr int kMfmaRhs = 64;       // per block (4 blocks of 16)
constexpr int kMfmaSrc = 16;       // sources per tile
constexpr int kMfmaFlush = 16;     // tiles between FP64 flushes
constexpr int kMfmaMinRhs = 8;     // fewer right-hand sides use the VALU kernel

template <int DIM>
__global__ __launch_bounds__(256) void ghat_mfma_kernel(
    BodyPhaseConsts k, const float* __restrict__ l0, const float* __restrict__ l1, const float* __restrict__ l2,
    const float* __restrict__ lsq, const double* __restrict__ cen, const int32_t* __restrict__ body_of,
    const c64* __restrict__ q, int64_t N, int R, int64_t chunk_len, c64* __restrict__ partial) {
  __shared__ c64 qt[2][kMfmaSrc][kMfmaRhs];  // transposed charge tiles, double-buffered
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tbase = (int64_t)blockIdx.x * kMfmaTargets + 16 * wave;
  const int r0 = blockIdx.z * kMfmaRhs;
  const int64_t c0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t c1 = min(N, c0 + chunk_len);

  // target of this lane in the A layout
  const int64_t tg = tbase + (lane & 15);
  const int64_t tgc = tg < N ? tg : N - 1;
  float lt[DIM];
  lt[0] = l0[tgc];
  lt[1] = l1[tgc];
  if constexpr (DIM == 3) lt[2] = l2[tgc];
  const int tb = tg < N ? body_of[tgc] : -1;
  double ct[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) ct[d] = cen[(int64_t)body_of[tgc] * DIM + d];

  v4f accR[4], accI[4];
  double sumR[4][4], sumI[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    accR[b] = v4f{0.f, 0.f, 0.f, 0.f};
    accI[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) sumR[b][i] = sumI[b][i] = 0.0;
  }
  int cur_sb = -1;
  float A = 0.f, D = 0.f, D2 = 0.f, ph0 = 0.f, P[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) P[d] = 0.f;

  // Software pipeline over tiles of 16 sources: while the matrix cores work on tile t (charges
  // from one LDS buffer, phi from registers), the wave loads the charges of tile t + 1, generates
  // its phi on the VALU and stores the charges into the other buffer; one barrier per tile.
  // Tiles are taken kMfmaFlush at a time with FP32 accumulators, then added into FP64 sums; the
  // flush sits outside the inner loop so the accumulators stay in the matrix-core registers.
  const int rr = threadIdx.x >> 2;        // right-hand side staged by this thread (0..63)
  const int sg = (threadIdx.x & 3) * 4;   // its four sources in the tile: 0, 4, 8, 12
  const int rq = r0 + rr;
  auto load_q = [&](int64_t j0, c64* qr) {
#pragma unroll
    for (int u = 0; u < 4; ++u) qr[u] = rq < R ? q[(int64_t)rq * N + j0 + sg + u] : c64{0.f, 0.f};
  };
  auto store_q = [&](int buf, const c64* qr) {
#pragma unroll
    for (int u = 0; u < 4; ++u) qt[buf][sg + u][rr] = qr[u];
  };
  // per (target, source body) quantities for the tile starting at j0; returns whether every target
  // of the wave is on another body and far from this one (then all pairs take the asymptotic branch)
  auto body_setup = [&](int64_t j0) {
    const int sb = body_of[j0];
    if (sb != cur_sb) {
      cur_sb = sb;
      double dd2 = 0.0;
      float Ai = 0.f;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dc = ct[d] - cen[(int64_t)sb * DIM + d];
        dd2 = fma(dc, dc, dd2);
        const float dcf = (float)dc;
        Ai = fmaf(lt[d], lt[d] + 2.0f * dcf, Ai);
        P[d] = -2.0f * (lt[d] + dcf);
      }
      const double dd = sqrt(dd2);
      const double ph = dd * k.kappa_rev64;
      A = Ai;
      D = (float)dd;
      D2 = (float)dd2;
      ph0 = (float)(ph - floor(ph)) - (DIM == 2 ? 0.125f : 0.0f);
    }
    return (bool)__all(tb < 0 || (tb != sb && D >= k.far_D));
  };
  // phi in the A layout: k-step s, source j0 + 4 s + lane / 16
  auto gen_phi = [&](int64_t j0, bool far_all, float* gr, float* gi) {
    const int sb = cur_sb;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t j = j0 + 4 * st + (lane >> 4);
      float u = A + lsq[j];
      u = fmaf(P[0], l0[j], u);
      u = fmaf(P[1], l1[j], u);
      if constexpr (DIM == 3) u = fmaf(P[2], l2[j], u);
      float pr, pi;
      if (far_all) {
        bp_phi<DIM, 1>(k, u, D, D2, ph0, pr, pi);
      } else {
        bp_phi<DIM>(k, u, D, D2, ph0, pr, pi);
        const bool same = tb == sb;
        pr = same ? 0.f : pr;
        pi = same ? 0.f : pi;
      }
      gr[st] = pr;
      gi[st] = pi;
    }
  };
  // the 64 MFMAs of one tile (4 k-steps x 4 blocks of 16 right-hand sides x 4 real products)
  auto mfma_tile = [&](int buf, const float* gr, const float* gi) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const float ngi = -gi[st];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const c64 qq = qt[buf][4 * st + (lane >> 4)][16 * b + (lane & 15)];
        accR[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr[st], qq.re, accR[b], 0, 0, 0);
        accR[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ngi, qq.im, accR[b], 0, 0, 0);
        accI[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr[st], qq.im, accI[b], 0, 0, 0);
        accI[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi[st], qq.re, accI[b], 0, 0, 0);
      }
    }
  };

  if (c0 < c1) {
    c64 qreg[4];
    float gr[4], gi[4];
    load_q(c0, qreg);
    store_q(0, qreg);
    gen_phi(c0, body_setup(c0), gr, gi);
    __syncthreads();
    int buf = 0;
    for (int64_t jb = c0; jb < c1; jb += (int64_t)kMfmaSrc * kMfmaFlush) {
      const int64_t je = min(c1, jb + (int64_t)kMfmaSrc * kMfmaFlush);
      for (int64_t j0 = jb; j0 < je; j0 += kMfmaSrc) {
        const int64_t jn = j0 + kMfmaSrc;
        const bool more = jn < c1;
        bool far_next = false;
        if (more) {
          load_q(jn, qreg);  // in flight during the matrix-core work below
          far_next = body_setup(jn);
        }
        float gn[4], gm[4];
        if (more && far_next) {
          // straight-line block: the scheduler interleaves the next tile's phi with this tile's MFMAs
          mfma_tile(buf, gr, gi);
          gen_phi(jn, true, gn, gm);
#pragma unroll
          for (int i = 0; i < 56; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // two VALU
          }
        } else {
          mfma_tile(buf, gr, gi);
          if (more) gen_phi(jn, false, gn, gm);
        }
        if (more) {
          store_q(buf ^ 1, qreg);
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            gr[st] = gn[st];
            gi[st] = gm[st];
          }
        }
        __syncthreads();
        buf ^= 1;
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sumR[b][i] += (double)accR[b][i];
          sumI[b][i] += (double)accI[b][i];
          accR[b][i] = 0.f;
          accI[b][i] = 0.f;
        }
    }
  }
  // output layout of the 16x16 MFMA: lane l, register i -> row 4 (l / 16) + i, column l % 16
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int r = r0 + 16 * b + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t t = tbase + 4 * (lane >> 4) + i;
      if (r < R && t < N)
        partial[((int64_t)blockIdx.y * R + r) * N + t] = c64{(float)sumR[b][i], (float)sumI[b][i]};
    }
  }
}

// ---------------------------------------------------------------------------
// Many right-hand sides on the FP16 matrix cores, operands split in two.
//
// Each FP32 operand x is carried as two FP16 numbers, x ~ hi + lo with hi = x rounded to FP16 and
// lo = x - hi rounded again (both toward zero: |x - hi| < 2^-10 |x|, and lo keeps 11 bits of it).
// A product is then a_hi b_hi + a_hi b_lo + a_lo b_hi, leaving out a_lo b_lo; each is within
// 3 2^-20 of the exact product at worst and ~2^-22 on average, below the ~1e-6 phase error of the
// FP32 phi.  FP16 products are exact in the FP32 accumulators.  Per 32 sources, 16 targets and 64
// right-hand sides this takes 48 FP16 16x16x32 products of 16 cycles against 128 FP32 16x16x4
// products of 32 cycles: under a fifth of the matrix-core time.  This is the
// single-precision recovery with low-precision matrix units of Ootomo and Yokota (2022) (Markidis
// et al. 2018 before them).  The matrix cores keep FP16 subnormal inputs (checked on the hardware),
// so lo needs no extra scaling.
//
// Scaling keeps the parts in range: each right-hand side is scaled by the power of two that puts
// its largest component in [2^13, 2^14); phi by 2^sA with sA chosen per scene so that
// 2^sA |phi| < 2^13 (in 2D |phi| < 16 always; in 3D from the smallest distance between two bodies'
// points).  Far-field amplitudes carry 2^sA in their constants, so the scaling costs nothing there.
//
// A block of 4 waves owns 64 targets and 64 right-hand sides; sources come 32 at a time
// (v_mfma_f32_16x16x32_f16: lane l holds row l%16 and 8 consecutive k values of group l/16, for A
// (phi: targets x sources) and B (charges: sources x right-hand sides) alike, so lane l evaluates
// phi for sources 8 (l/16) .. 8 (l/16) + 7 of the tile, all in one 16-point half and so in one
// body).  The FP32 accumulators are added into FP32 sums every 8 tiles (256 sources): the sums take
// at most a few hundred additions (~3e-7 relative), and the registers this saves over FP64 sums let
// three waves share a SIMD, so that one wave's phi evaluation overlaps another's products.
// ---------------------------------------------------------------------------
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __fp16 h2pk __attribute__((ext_vector_type(2)));
constexpr int kM16Src = 32;                          // sources per tile (the k of one MFMA)
constexpr int kM16Flush = 8;                         // tiles between flushes of the accumulators
constexpr int kM16TileChunks = 4 * 4 * kMfmaRhs;     // 16-byte chunks of one split tile (16 KB)
constexpr int kM16QExp = 14;                         // largest scaled charge component below 2^14


// x[0..7] (times s) -> hi and lo = x s - hi, two values per conversion (round toward zero; x s - hi
// is exact in FP32)
__device__ __forceinline__ void split8(const float* x, float s, uint4& hi, uint4& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float x0 = x[2 * m] * s, x1 = x[2 * m + 1] * s;
    const h2pk a = __builtin_amdgcn_cvt_pkrtz(x0, x1);
    const h2pk b = __builtin_amdgcn_cvt_pkrtz(x0 - (float)a.x, x1 - (float)a.y);
    h[m] = __builtin_bit_cast(uint32_t, a);
    l[m] = __builtin_bit_cast(uint32_t, b);
  }
  hi = uint4{h[0], h[1], h[2], h[3]};
  lo = uint4{l[0], l[1], l[2], l[3]};
}

__device__ __forceinline__ v8h as_v8h(const uint4& u) { return __builtin_bit_cast(v8h, u); }

// lane I of each 16-lane row to the whole row (DPP row_newbcast)
template <int I>
__device__ __forceinline__ float row_bcast(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x150 + I, 0xF, 0xF, false));
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// E[r]: the largest |Re q| or |Im q| of right-hand side r is f 2^E[r] with f in [0.5, 1) (0: zero column).
__global__ __launch_bounds__(256) void qsplit_exp_kernel(const c64* __restrict__ q, int64_t N, int R,
                                                         int32_t* __restrict__ E) {
  const int r = blockIdx.x;
  float m = 0.f;
  if (r < R)
    for (int64_t j = threadIdx.x; j < N; j += 256) {
      const c64 v = q[(int64_t)r * N + j];
      m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int e = 0;
    if (m > 0.f) frexpf(m, &e);
    E[r] = e;
  }
}

// Charges -> the split tile layout: right-hand-side block rb, tile t (32 sources), component c
// (Re hi, Im hi, Re lo, Im lo), group g, right-hand side rr: the 8 halves of sources
// 32 t + 8 g + 0..7, 16 bytes, at chunk (((rb ntiles + t) 4 + c) 4 + g) 64 + rr.  Sources >= N and
// right-hand sides >= R are zero.
__global__ __launch_bounds__(256) void qsplit_kernel(const c64* __restrict__ q, int64_t N, int R, int64_t ntiles,
                                                     const int32_t* __restrict__ E, uint4* __restrict__ out) {
  const int64_t t = blockIdx.x;
  const int rb = blockIdx.y;
  const int g = threadIdx.x >> 6, rr = threadIdx.x & 63;
  const int r = rb * kMfmaRhs + rr;
  const int64_t j0 = t * kM16Src + 8 * g;
  const int sh = r < R ? kM16QExp - E[r] : 0;
  float re[8], im[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t j = j0 + e;
    const c64 v = (r < R && j < N) ? q[(int64_t)r * N + j] : c64{0.f, 0.f};
    re[e] = ldexpf(v.re, sh);
    im[e] = ldexpf(v.im, sh);
  }
  uint4 rh, rl, ih, il;
  split8(re, 1.0f, rh, rl);
  split8(im, 1.0f, ih, il);
  uint4* dst = out + ((int64_t)rb * ntiles + t) * kM16TileChunks;
  dst[(0 * 4 + g) * kMfmaRhs + rr] = rh;
  dst[(1 * 4 + g) * kMfmaRhs + rr] = ih;
  dst[(2 * 4 + g) * kMfmaRhs + rr] = rl;
  dst[(3 * 4 + g) * kMfmaRhs + rr] = il;
}

struct M16Lds {
  uint4 q[2][kM16TileChunks];  // [buffer][(component * 4 + group) * 64 + right-hand side]
  float4 geo[2][kM16Src];      // [buffer][source]: body-local offset (l0, l1, l2) and |l|^2
  int sb[2][2];                // [buffer][half]: body of the tile's two 16-point halves
};

template <int DIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void ghat_mfma16_kernel(
    BodyPhaseConsts k, BodyPhaseConsts kf, const float* __restrict__ l0, const float* __restrict__ l1,
    const float* __restrict__ l2, const float* __restrict__ lsq, const double* __restrict__ cen,
    const int32_t* __restrict__ body_of, const uint4* __restrict__ qs, const int32_t* __restrict__ qexp, int64_t N,
    int64_t ntiles, int R, int64_t chunk_len, float a_scale, int a_shift, c64* __restrict__ partial) {
  __shared__ M16Lds lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int grp = lane >> 4;   // k group: sources 8 grp .. 8 grp + 7 of the tile
  const int half = lane >> 5;  // the tile half those sources lie in
  const int col = lane & 15;
  const int64_t tbase = (int64_t)blockIdx.x * kMfmaTargets + 16 * wave;
  const int r0 = blockIdx.z * kMfmaRhs;
  const int64_t Ns = ntiles * kM16Src;
  const int64_t c0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t c1 = min(Ns, c0 + chunk_len);
  const uint4* qtiles = qs + (int64_t)blockIdx.z * ntiles * kM16TileChunks;

  // target of this lane in the A layout (row l % 16)
  const int64_t tg = tbase + col;
  const int64_t tgc = tg < N ? tg : N - 1;
  float lt[DIM];
  lt[0] = l0[tgc];
  lt[1] = l1[tgc];
  if constexpr (DIM == 3) lt[2] = l2[tgc];
  const int tb = tg < N ? body_of[tgc] : -1;
  double ct[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) ct[d] = cen[(int64_t)body_of[tgc] * DIM + d];

  v4f tr[4], ti[4];
  float sumR[4][4], sumI[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    tr[b] = ti[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) sumR[b][i] = sumI[b][i] = 0.f;
  }
  int cur_sb = -1;
  bool same = false;
  float A = 0.f, D = 0.f, D2 = 0.f, ph0 = 0.f, P[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) P[d] = 0.f;

  // Staging of tile t into buffer t % 2, one tile ahead: thread tid moves charge chunks tid + 256 u
  // (component u); threads below 128 one geometry value each; threads 128 and 129 the bodies of
  // the two halves.
  const float* garr = tid < 32 ? l0 : tid < 64 ? l1 : tid < 96 ? l2 : lsq;
  const bool gstage = tid < 128 && (DIM == 3 || tid < 64 || tid >= 96);
  uint4 q0, q1, q2, q3;
  float gv = 0.f;
  int sbv = 0;
  auto load_q = [&](int64_t j) __attribute__((always_inline)) {
    const uint4* src = qtiles + (j / kM16Src) * kM16TileChunks + tid;
    q0 = src[0];
    q1 = src[256];
    q2 = src[512];
    q3 = src[768];
  };
  auto load_geo = [&](int64_t j) __attribute__((always_inline)) {
    if (gstage) gv = garr[min(j + (tid & 31), N - 1)];
    if (tid >= 128 && tid < 130) sbv = body_of[min(j + 16 * (tid - 128), N - 1)];
  };
  auto stage_store = [&](int buf) __attribute__((always_inline)) {
    uint4* dst = lds.q[buf] + tid;
    dst[0] = q0;
    dst[256] = q1;
    dst[512] = q2;
    dst[768] = q3;
    if (tid < 128) reinterpret_cast<float*>(lds.geo[buf])[(tid & 31) * 4 + (tid >> 5)] = gv;
    else if (tid < 130) lds.sb[buf][tid - 128] = sbv;
  };
  // per (target, source body) quantities for this lane's half of the tile in buffer g; returns 2
  // where every pair of the wave takes the very-far branch (2D), 1 the far branch, 0 otherwise
  auto setup = [&](int g) __attribute__((always_inline)) -> int {
    const int sb = lds.sb[g][half];
    if (sb != cur_sb) {
      cur_sb = sb;
      double dd2 = 0.0;
      float Ai = 0.f;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dc = ct[d] - cen[(int64_t)sb * DIM + d];
        dd2 = fma(dc, dc, dd2);
        const float dcf = (float)dc;
        Ai = fmaf(lt[d], lt[d] + 2.0f * dcf, Ai);
        P[d] = -2.0f * (lt[d] + dcf);
      }
      const double dd = sqrt(dd2);
      const double ph = dd * k.kappa_rev64;
      A = Ai;
      D = (float)dd;
      D2 = (float)dd2;
      ph0 = (float)(ph - floor(ph)) - (DIM == 2 ? 0.125f : 0.0f);
    }
    same = tb == sb;
    if (DIM == 2 && __all(tb < 0 || (!same && D >= k.vfar_D))) return 2;
    return __all(tb < 0 || (!same && D >= k.far_D)) ? 1 : 0;
  };
  // phi (times 2^sA) for this lane's 8 sources of the tile in buffer g, split into A operands; the
  // geometry is read once per lane (source 8 grp + l % 8) and broadcast along the 16-lane rows
  auto gen = [&](int g, int regime, uint4& rh, uint4& rl, uint4& ih, uint4& il) __attribute__((always_inline)) {
    float pr[8], pi[8];
    const float4 gmine = lds.geo[g][8 * grp + (lane & 7)];
    static_for<0, 8>([&](auto ic) __attribute__((always_inline)) {
      constexpr int i = decltype(ic)::value;
      float u = A + row_bcast<i>(gmine.w);
      u = fmaf(P[0], row_bcast<i>(gmine.x), u);
      u = fmaf(P[1], row_bcast<i>(gmine.y), u);
      if constexpr (DIM == 3) u = fmaf(P[2], row_bcast<i>(gmine.z), u);
      if (regime == 2) {
        bp_phi<DIM, 2>(kf, u, D, D2, ph0, pr[i], pi[i]);
      } else if (regime == 1) {
        bp_phi<DIM, 1>(kf, u, D, D2, ph0, pr[i], pi[i]);
      } else {
        bp_phi<DIM>(k, u, D, D2, ph0, pr[i], pi[i]);
        pr[i] = same ? 0.f : pr[i] * a_scale;
        pi[i] = same ? 0.f : pi[i] * a_scale;
      }
    });
    split8(pr, 1.0f, rh, rl);
    split8(pi, 1.0f, ih, il);
  };
  // the 48 products of one tile: Re += Gr Qr - Gi Qi, Im += Gr Qi + Gi Qr, each over hi hi, hi lo
  // and lo hi
  auto tile = [&](int buf, const uint4& grh, const uint4& grl, const uint4& gih, const uint4& gil)
                  __attribute__((always_inline)) {
    const v8h Grh = as_v8h(grh), Grl = as_v8h(grl), Gih = as_v8h(gih), Gil = as_v8h(gil);
    const v8h nGih = -Gih, nGil = -Gil;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint4* qb = lds.q[buf] + 16 * b + col + grp * kMfmaRhs;
      const v8h Qrh = as_v8h(qb[0 * 256]), Qih = as_v8h(qb[1 * 256]);
      const v8h Qrl = as_v8h(qb[2 * 256]), Qil = as_v8h(qb[3 * 256]);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grh, Qrh, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grh, Qih, ti[b], 0, 0, 0);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nGih, Qih, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Gih, Qrh, ti[b], 0, 0, 0);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grh, Qrl, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grh, Qil, ti[b], 0, 0, 0);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nGih, Qil, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Gih, Qrl, ti[b], 0, 0, 0);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grl, Qrh, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Grl, Qih, ti[b], 0, 0, 0);
      tr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nGil, Qih, tr[b], 0, 0, 0);
      ti[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Gil, Qrh, ti[b], 0, 0, 0);
    }
  };

  if (c0 < c1) {
    load_q(c0);
    load_geo(c0);
    stage_store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t jb = c0; jb < c1; jb += (int64_t)kM16Src * kM16Flush) {
      const int64_t je = min(c1, jb + (int64_t)kM16Src * kM16Flush);
      for (int64_t j0 = jb; j0 < je; j0 += kM16Src) {
        const bool more = j0 + kM16Src < c1;
        if (more) {  // in flight during this tile's work
          load_q(j0 + kM16Src);
          load_geo(j0 + kM16Src);
        }
        uint4 grh, grl, gih, gil;
        const int rg = setup(buf);
        if (rg == 2) gen(buf, 2, grh, grl, gih, gil);
        else if (rg == 1) gen(buf, 1, grh, grl, gih, gil);
        else gen(buf, 0, grh, grl, gih, gil);
        tile(buf, grh, grl, gih, gil);
        if (more) stage_store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sumR[b][i] += tr[b][i];
          sumI[b][i] += ti[b][i];
          tr[b][i] = ti[b][i] = 0.f;
        }
    }
  }
  // output layout of the 16x16 MFMA: lane l, register i -> row 4 (l / 16) + i, column l % 16;
  // the charges of right-hand side r were scaled by 2^(14 - E[r]), phi by 2^a_shift
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int r = r0 + 16 * b + col;
    if (r >= R) continue;
    const int sh = qexp[r] - kM16QExp - a_shift;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t t = tbase + 4 * (lane >> 4) + i;
      if (t < N)
        partial[((int64_t)blockIdx.y * R + r) * N + t] = c64{ldexpf(sumR[b][i], sh), ldexpf(sumI[b][i], sh)};
    }
  }
}

// ---------------------------------------------------------------------------
// Many right-hand sides in FP64 (the residuals of the mixed solve, the FP64 solve): the same
// contraction on the FP64 matrix cores, phi evaluated once per pair for all 64 right-hand sides of a
// block instead of once per 4 in the vector-unit kernel.  phi in FP64 from the absolute FP64
// coordinates (the FP64 Hankel function of phi.h; no body-centre split is needed at this
// precision), FP64 products and accumulation throughout.  A block of 4 waves owns 64 targets and 64
// right-hand sides; sources come 16 at a time (four k-steps of v_mfma_f64_16x16x4f64: A and B lanes
// as in the FP32 form, but D row 4 v + l/16, column l % 16 in register v of lane l).  Every body
// holds a multiple of 16 points, so a tile lies in one body.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kM64Src = 16;

template <int DIM>
__global__ __launch_bounds__(256) void ghat_mfma64_kernel(double kappa, const double* __restrict__ x0,
                                                          const double* __restrict__ x1,
                                                          const double* __restrict__ x2,
                                                          const int32_t* __restrict__ body_of,
                                                          const c128* __restrict__ q, int64_t N, int R,
                                                          int64_t chunk_len, c128* __restrict__ partial) {
  __shared__ c128 qt[2][kM64Src][kMfmaRhs];  // charge tiles, double-buffered
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tbase = (int64_t)blockIdx.x * kMfmaTargets + 16 * wave;
  const int r0 = blockIdx.z * kMfmaRhs;
  const int64_t c0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t c1 = min(N, c0 + chunk_len);
  const int64_t tg = tbase + (lane & 15);
  const int64_t tgc = tg < N ? tg : N - 1;
  double xt[DIM];
  xt[0] = x0[tgc];
  xt[1] = x1[tgc];
  if constexpr (DIM == 3) xt[2] = x2[tgc];
  const int tb = tg < N ? body_of[tgc] : -1;
  v4d accR[4], accI[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) accR[b] = accI[b] = v4d{0.0, 0.0, 0.0, 0.0};
  // staging: thread tid moves right-hand side tid / 4, sources 4 (tid % 4) .. + 3 of the tile
  const int rr = tid >> 2, sg = (tid & 3) * 4;
  const int rq = r0 + rr;
  c128 qreg[4];
  auto load_q = [&](int64_t j0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) qreg[u] = rq < R ? q[(int64_t)rq * N + j0 + sg + u] : c128{0.0, 0.0};
  };
  auto store_q = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 4; ++u) qt[buf][sg + u][rr] = qreg[u];
  };
  if (c0 < c1) {
    load_q(c0);
    store_q(0);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = c0; j0 < c1; j0 += kM64Src) {
      const bool more = j0 + kM64Src < c1;
      if (more) load_q(j0 + kM64Src);  // in flight during this tile's work
      const bool same = tb == body_of[j0];
#pragma unroll 1
      for (int st = 0; st < 4; ++st) {  // not unrolled: one copy of the FP64 Hankel function
        const int64_t j = j0 + 4 * st + (lane >> 4);
        double r2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double dx = xt[d] - (d == 0 ? x0[j] : d == 1 ? x1[j] : x2[j]);
          r2 = fma(dx, dx, r2);
        }
        double pr = 0.0, pi = 0.0;
        if (!same && tb >= 0) {
          if constexpr (DIM == 2) phi2d_f64(sqrt(r2), kappa, pr, pi);
          else phi3d_f64(sqrt(r2), kappa, pr, pi);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const c128 qq = qt[buf][4 * st + (lane >> 4)][16 * b + (lane & 15)];
          accR[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, qq.re, accR[b], 0, 0, 0);
          accR[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi, qq.im, accR[b], 0, 0, 0);
          accI[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, qq.im, accI[b], 0, 0, 0);
          accI[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, qq.re, accI[b], 0, 0, 0);
        }
      }
      if (more) store_q(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int r = r0 + 16 * b + (lane & 15);
    if (r >= R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t t = tbase + 4 * v + (lane >> 4);
      if (t < N) partial[((int64_t)blockIdx.y * R + r) * N + t] = c128{accR[b][v], accI[b][v]};
    }
  }
}

template <int DIM>
static hipError_t launch_mfma64(const SceneDev& s, const c128* q, int R, c128* partial, int nchunks,
                                hipStream_t st) {
  int64_t chunk_len = (s.N + nchunks - 1) / nchunks;
  chunk_len = (chunk_len + kM64Src - 1) / kM64Src * kM64Src;
  dim3 grid((unsigned)((s.N + kMfmaTargets - 1) / kMfmaTargets), (unsigned)nchunks,
            (unsigned)((R + kMfmaRhs - 1) / kMfmaRhs));
  hipLaunchKernelGGL((ghat_mfma64_kernel<DIM>), grid, dim3(256), 0, st, s.kappa, s.x64[0], s.x64[1], s.x64[2],
                     s.body_of, q, s.N, R, chunk_len, partial);
  return hipGetLastError();
}

hipError_t launch_ghat_mc64(const SceneDev& s, const c128* q, int R, c128* partial, int nchunks, hipStream_t st) {
  return s.dim == 2 ? launch_mfma64<2>(s, q, R, partial, nchunks, st) : launch_mfma64<3>(s, q, R, partial, nchunks, st);
}

template <int DIM>
static hipError_t launch_mfma(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks, hipStream_t st) {
  int64_t chunk_len = (s.N + nchunks - 1) / nchunks;
  chunk_len = (chunk_len + kMfmaSrc - 1) / kMfmaSrc * kMfmaSrc;
  dim3 grid((unsigned)((s.N + kMfmaTargets - 1) / kMfmaTargets), (unsigned)nchunks,
            (unsigned)((R + kMfmaRhs - 1) / kMfmaRhs));
  hipLaunchKernelGGL((ghat_mfma_kernel<DIM>), grid, dim3(256), 0, st, make_bodyphase(s.kappa, s.rho_max), s.l32[0], s.l32[1],
                     s.l32[2], s.lsq32, s.centres, s.body_of, q, s.N, R, chunk_len, partial);
  return hipGetLastError();
}

// Split charges of the FP16 matrix-core kernel: tiles of 32 sources per block of 64 right-hand
// sides, 16 KB each, then the exponents E[Rpad].
static int64_t m16_tiles(const SceneDev& s) { return (s.N + kM16Src - 1) / kM16Src; }
static int m16_rblocks(int R) { return (R + kMfmaRhs - 1) / kMfmaRhs; }

size_t ghat_split_bytes(const SceneDev& s, int R) {
  return (size_t)m16_rblocks(R) * m16_tiles(s) * kM16TileChunks * sizeof(uint4) +
         (size_t)m16_rblocks(R) * kMfmaRhs * sizeof(int32_t);
}

bool ghat_uses_mfma16(const SceneDev& s, int R) { return R >= kMfmaMinRhs && s.all_k_mult16 && s.phi16_shift >= 0; }

template <int DIM>
static hipError_t launch_mfma16(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks, void* split,
                                hipStream_t st) {
  const int64_t ntiles = m16_tiles(s);
  const int nrb = m16_rblocks(R);
  uint4* qs = static_cast<uint4*>(split);
  int32_t* qexp = reinterpret_cast<int32_t*>(qs + (size_t)nrb * ntiles * kM16TileChunks);
  hipLaunchKernelGGL(qsplit_exp_kernel, dim3((unsigned)(nrb * kMfmaRhs)), dim3(256), 0, st, q, s.N, R, qexp);
  hipLaunchKernelGGL(qsplit_kernel, dim3((unsigned)ntiles, (unsigned)nrb), dim3(256), 0, st, q, s.N, R, ntiles,
                     static_cast<const int32_t*>(qexp), qs);
  int64_t chunk_len = (ntiles * kM16Src + nchunks - 1) / nchunks;
  chunk_len = (chunk_len + kM16Src - 1) / kM16Src * kM16Src;
  dim3 grid((unsigned)((s.N + kMfmaTargets - 1) / kMfmaTargets), (unsigned)nchunks, (unsigned)nrb);
  const BodyPhaseConsts k = make_bodyphase(s.kappa, s.rho_max);
  hipLaunchKernelGGL((ghat_mfma16_kernel<DIM>), grid, dim3(256), 0, st, k, scale_far_amplitude(k, s.phi16_shift),
                     s.l32[0], s.l32[1], s.l32[2], s.lsq32, s.centres, s.body_of, static_cast<const uint4*>(qs),
                     static_cast<const int32_t*>(qexp), s.N, ntiles, R, chunk_len, std::ldexp(1.0f, s.phi16_shift),
                     s.phi16_shift, partial);
  return hipGetLastError();
}

bool ghat_uses_mfma(const SceneDev& s, int R) { return R >= kMfmaMinRhs && s.all_k_mult16; }

hipError_t launch_ghat_mc(const SceneDev& s, const c64* q, int R, c64* partial, int nchunks, void* split,
                          hipStream_t st) {
  if (split && ghat_uses_mfma16(s, R))
    return s.dim == 2 ? launch_mfma16<2>(s, q, R, partial, nchunks, split, st)
                      : launch_mfma16<3>(s, q, R, partial, nchunks, split, st);
  return s.dim == 2 ? launch_mfma<2>(s, q, R, partial, nchunks, st) : launch_mfma<3>(s, q, R, partial, nchunks, st);
}

}  // namespace mfs
