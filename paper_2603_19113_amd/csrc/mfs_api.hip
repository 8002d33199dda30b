// C ABI of libmfs: scenes, the operator I + S G_hat (eq. mbody2), field evaluation and the
// GMRES / GMRES-IR driver.  Kernels live in pair_kernels.hip, sapply.hip, krylov.hip, lsq.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "mfs_internal.h"

namespace mfs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mfs_status fail(mfs_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Grow-only device buffer owned by a scene, drawn from the library's caching pool (pool.hip): a
// grown or released block goes back to the pool ordered after the work enqueued on `st`.
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

static mfs_status ensure(Buf& b, size_t bytes, size_t* total, hipStream_t st) {
  if (b.cap >= bytes) return MFS_OK;
  if (b.p) {
    pool_free(b.p, b.cap, st);
    *total -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t got = 0;
  hipError_t e = hipSuccess;
  void* p = pool_alloc(bytes, st, &got, &e);
  if (!p)
    return fail(MFS_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                   hipGetErrorString(e));
  b.p = p;
  b.cap = got;
  *total += got;
  return MFS_OK;
}

static void release(Buf& b, size_t* total, hipStream_t last) {
  if (b.p) {
    pool_free(b.p, b.cap, last);
    *total -= b.cap;
  }
  b.p = nullptr;
  b.cap = 0;
}

// ----------------------------------------------------------- kernel timing ---
struct TimingRecord {
  int kind;
  double pairs;
  hipEvent_t e0, e1;
};
// The record list is shared by every calling thread (the serving loop calls from one thread per slot).
static std::atomic<bool> g_timing_on{false};
static std::mutex g_timing_mu;
static std::vector<TimingRecord> g_timing;

TimedLaunch::TimedLaunch(int k, double p, hipStream_t s) : kind(k), pairs(p), st(s), ev0(nullptr), ev1(nullptr) {
  if (!g_timing_on) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  ev0 = a;
  ev1 = b;
  (void)hipEventRecord(a, st);
}

TimedLaunch::~TimedLaunch() {
  if (!ev0) return;
  (void)hipEventRecord(static_cast<hipEvent_t>(ev1), st);
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing.push_back(TimingRecord{kind, pairs, static_cast<hipEvent_t>(ev0), static_cast<hipEvent_t>(ev1)});
}

static void timing_clear() {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto& r : g_timing) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_timing.clear();
}

}  // namespace mfs

using namespace mfs;

struct mfs_scene {
  SceneDev dev{};
  int device = 0;  // HIP device the scene's tables live on
  int n_shapes = 0;
  int64_t kmax = 0;
  bool has_s32 = false;
  std::vector<int64_t> k_of_shape;
  size_t bytes = 0;
  hipStream_t last_stream = nullptr;  // stream of the latest call; releases are ordered after it
  // owned tables
  Buf x64, x32, l32, lsq, centres, body_of, body_ptr, shape_of, k_dev, S64_tab, S32_tab, rot;
  // padded layout for the symmetric pair kernel (bodies whose point count is not a multiple of 64)
  Buf pad_ptr, body_of_pad, l32p, lsqp, qpad;
  // workspaces
  Buf partial, q32, dirs, kry, vecs, qsplit;
  int phi16_shift_auto = -1;  // the scene's bound for the FP16 matrix-core kernel (-1: none)
  // near-field tables for the last set of reconstruction factors used with this scene
  std::vector<uint64_t> near_key;
  Buf near_tab;
  mfs::NearTables near{};
  std::vector<std::vector<int32_t>> bodies_of_shape;
  std::vector<const int32_t*> bodies_dev;
  // pair-sum launch shapes tuned on this scene, by (kernel variant, R)
  std::map<std::pair<int, int>, LaunchShape> tuned;
};

struct mfs_recon {
  mfs::ReconFactors f{};
  double psi_radius = 0.0;
  uint64_t id = 0;  // unique per handle: scenes cache tables by id, never by (reusable) address
};

static std::atomic<uint64_t> g_recon_ids{1};

// The scale 2^sA of phi for the FP16 matrix-core kernel: the largest sA with 2^sA |phi| < 2^13 for
// every pair of points on different bodies (at most 2^20), or -1 where no bound is known.  2D:
// |phi| = |H0(kappa r)| / 4 < 16 for every r the FP32 kernel can resolve (the Hankel function grows
// only logarithmically as kappa r -> 0), so sA = 9.  3D: |phi| = 1 / (4 pi r) with r at least the
// smallest distance between two body centres less 2 rho_max (closest pair of centres by a sweep over
// the centres sorted by their first coordinate).
int phi16_shift_for(int dim, int64_t T, const double* centres, double rho_max) {
  if (dim == 2) return 9;
  if (T < 2) return 20;
  std::vector<int64_t> idx(T);
  for (int64_t i = 0; i < T; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return centres[a * dim] < centres[b * dim]; });
  double best = INFINITY;
  for (int64_t a = 0; a < T; ++a) {
    const double* ca = centres + idx[a] * dim;
    for (int64_t b = a + 1; b < T; ++b) {
      const double* cb = centres + idx[b] * dim;
      if (cb[0] - ca[0] >= best) break;
      double d2 = 0.0;
      for (int d = 0; d < dim; ++d) d2 += (cb[d] - ca[d]) * (cb[d] - ca[d]);
      best = std::min(best, std::sqrt(d2));
    }
  }
  const double r_lb = best - 2.0 * rho_max;
  if (!(r_lb > 0.0)) return -1;
  const double phi_max = 1.0 / (4.0 * M_PI * r_lb);
  int sA = 20;
  while (sA >= 0 && std::ldexp(phi_max, sA) >= 8192.0) --sA;
  return sA;
}

// Scratch memory of mfs_apply_static: the pair sum's partial slices (and the padded copy of the
// charges for the symmetric kernel) live in this fixed array instead of scene workspace, so that
// call allocates nothing.  Each device holds its own copy (module globals are per device).  In host
// code `scratch` only names the symbol: its device address comes from hipGetSymbolAddress, taken
// once per device when the first scene is created there, and kept in g_scratch_addr.
static __device__ __align__(256) unsigned char scratch[MFS_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

// Address of `scratch` on `device` (which must be current), looked up on the first call per device.
static mfs_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(MFS_ERR_ARG, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MFS_ERR_HIP, std::string("static scratch address: ") + hipGetErrorString(e));
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return MFS_OK;
}

namespace {

#define MFS_TRY(expr)                  \
  do {                                 \
    mfs_status s__ = (expr);           \
    if (s__ != MFS_OK) return s__;     \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

mfs_status check_scene(const mfs_scene* s) {
  if (!s) return fail(MFS_ERR_ARG, "scene is null");
  return MFS_OK;
}

mfs_status check_prec_operator(const mfs_scene* s, mfs_prec prec) {
  if (prec != MFS_FP64 && prec != MFS_FP32)
    return fail(MFS_ERR_ARG, "operator precision must be MFS_FP64 or MFS_FP32");
  if (prec == MFS_FP32 && !s->has_s32) return fail(MFS_ERR_ARG, "scene was created without FP32 copies of S");
  return MFS_OK;
}

int tpt_for(mfs_prec prec) { return prec == MFS_FP64 ? 1 : 2; }

int tune_variant(const mfs_scene* s, bool f64, int R) {
  return f64 ? kTunePairF64 : ghat_uses_mfma(s->dev, R) ? kTunePairMfma : kTunePairF32;
}

// Launch shape of the pair sum over the scene's own points: the scene's tuned entry, else the
// process-wide table, else the heuristic (the symmetric kernel where it applies); resolved for this
// scene (sym is 0 or 1 on return, and nchunks counts distance chunks when sym is 1).
LaunchShape shape_for(const mfs_scene* s, bool f64, int R, int* source = nullptr) {
  const int v = tune_variant(s, f64, R);
  LaunchShape e;
  int src = 0;
  auto it = s->tuned.find({v, R});
  if (it != s->tuned.end()) {
    e = it->second;
    src = 2;
  } else if (tune_lookup(s->dev.dim, v, R, s->dev.N, &e)) {
    src = 1;
  }
  if (source) *source = src;
  LaunchShape ls = e;
  // untuned: the symmetric kernel up to kSymDefaultMaxRhs right-hand sides where the matrix cores
  // take FP32 products (it was 3.4x faster at 8, 1.7x at 16, 0.87x at 32), and below 8 where they
  // take split FP16 products (those evaluate phi once per pair for up to 64 right-hand sides: 148 ms
  // against 173 ms for the symmetric kernel with 8 on the 2000-body mixed scene); tuned or set: up
  // to kSymMaxRhs
  const bool sym_default = R <= kSymDefaultMaxRhs && !ghat_uses_mfma16(s->dev, R);
  const bool sym_ok = v != kTunePairF64 && ghat_sym_possible(s->dev, R) && (e.sym == 1 || sym_default);
  if (sym_ok && e.sym != 0) {
    ls.sym = 1;
    // a slice count tuned for the other kernel does not carry over
    if (e.sym != 1 || e.nchunks <= 0) {
      const int64_t NS = sym_view(s->dev).N;
      ls.nchunks = sym_plan(NS, 0, sym_block_waves(NS, R)).nchunks_d;
    }
  } else {
    ls.sym = 0;
    if (e.sym == 1 || e.nchunks <= 0) ls.nchunks = pair_chunks_for(s->dev.N, s->dev.N, tpt_for(f64 ? MFS_FP64 : MFS_FP32));
  }
  return ls;
}

// Rows of a partial-sum slice with this shape: the padded layout's length for the symmetric kernel
// on bodies that are not whole tiles, else N.
int64_t f32_rows(const mfs_scene* s, const LaunchShape& ls) {
  return ls.sym == 1 && sym_padded(s->dev) ? s->dev.Npad : s->dev.N;
}

// Partial-sum slices the FP32 pair sum writes with this shape for R right-hand sides.
int f32_slices(const mfs_scene* s, const LaunchShape& ls, int R) {
  if (ls.sym != 1) return ls.nchunks;
  const int64_t rows = f32_rows(s, ls);
  return sym_plan(rows, ls.nchunks, sym_block_waves(rows, R)).slices;
}

// Where the FP32 pair sum left its partial sums: `slices` slices of R rows of NP entries, body b's
// entries from pptr[b] (pptr null: the packed layout).
struct PartialF32 {
  c64* part;
  int slices;
  const int64_t* pptr;
  int64_t NP;
};

// The FP32 pair sum of q32 ([R][N] complex64) into the scene's partial buffer.
mfs_status pair_f32(mfs_scene* s, const c64* q32, int R, hipStream_t st, PartialF32* out) {
  const LaunchShape ls = shape_for(s, false, R);
  const bool padded = ls.sym == 1 && sym_padded(s->dev);
  const int64_t rows = f32_rows(s, ls);
  const int nch = f32_slices(s, ls, R);
  MFS_TRY(ensure(s->partial, (size_t)nch * R * rows * sizeof(c64), &s->bytes, st));
  c64* part = static_cast<c64*>(s->partial.p);
  const c64* qs = q32;
  if (padded) {
    MFS_TRY(ensure(s->qpad, (size_t)R * rows * sizeof(c64), &s->bytes, st));
    MFS_HIP_TRY(launch_gather_pad(s->dev, q32, R, static_cast<c64*>(s->qpad.p), st));
    qs = static_cast<c64*>(s->qpad.p);
  }
  void* split = nullptr;
  if (ls.sym != 1 && ghat_uses_mfma16(s->dev, R)) {
    MFS_TRY(ensure(s->qsplit, ghat_split_bytes(s->dev, R), &s->bytes, st));
    split = s->qsplit.p;
  }
  {
    TimedLaunch tl(MFS_KERNEL_PAIR_F32, s->dev.offbody_pairs * R, st);
    if (ls.sym == 1) MFS_HIP_TRY(launch_ghat_f32_sym(sym_view(s->dev), qs, R, part, ls.nchunks, ls.rt, st));
    else MFS_HIP_TRY(launch_ghat_f32(s->dev, q32, R, part, ls.nchunks, st, ls.rt, split));
  }
  *out = PartialF32{part, nch, padded ? s->dev.pad_ptr : nullptr, padded ? rows : 0};
  return MFS_OK;
}

// y = q + S G_hat q in FP64 (all operands complex128).
mfs_status apply_f64(mfs_scene* s, const c128* q, c128* y, int R, hipStream_t st, double beta = 1.0) {
  const int nch = ghat_f64_slices(s->dev, R, shape_for(s, true, R).nchunks);
  MFS_TRY(ensure(s->partial, (size_t)nch * R * s->dev.N * sizeof(c128), &s->bytes, st));
  c128* part = static_cast<c128*>(s->partial.p);
  {
    TimedLaunch tl(MFS_KERNEL_PAIR_F64, s->dev.offbody_pairs * R, st);
    MFS_HIP_TRY(launch_ghat_f64(s->dev, q, R, part, nch, st));
  }
  MFS_HIP_TRY(launch_sapply_f64(s->dev, part, nch, q, beta, y, R, (int)s->kmax, st));
  return MFS_OK;
}

// y = q + S G_hat q in FP32 (complex64 in and out).
mfs_status apply_f32(mfs_scene* s, const c64* q, c64* y, int R, hipStream_t st) {
  PartialF32 p;
  MFS_TRY(pair_f32(s, q, R, st, &p));
  MFS_HIP_TRY(launch_sapply_f32(s->dev, p.part, p.slices, q, 1.0f, y, R, (int)s->kmax, st, p.pptr, p.NP));
  return MFS_OK;
}

// y = q + S G_hat q with q, y complex128 and the pair sum and S product in FP32: the identity
// part stays exact in FP64, only S G_hat q carries single-precision error.
mfs_status apply_mixed(mfs_scene* s, const c128* q, c128* y, int R, hipStream_t st, double beta = 1.0) {
  const int64_t NR = s->dev.N * R;
  MFS_TRY(ensure(s->q32, (size_t)NR * sizeof(c64), &s->bytes, st));
  c64* q32 = static_cast<c64*>(s->q32.p);
  MFS_HIP_TRY(launch_to_c64(q, q32, NR, st));
  PartialF32 p;
  MFS_TRY(pair_f32(s, q32, R, st, &p));
  MFS_HIP_TRY(launch_sapply_mixed(s->dev, p.part, p.slices, q, beta, y, R, (int)s->kmax, st, p.pptr, p.NP));
  return MFS_OK;
}

// Device tables tying the scene's bodies to the reconstruction factors of their shapes; rebuilt
// when the factors passed in change.  Synchronous on the first call with a new set.
mfs_status prepare_near(mfs_scene* s, const mfs_recon* const* recon, hipStream_t st) {
  if (!recon) return fail(MFS_ERR_ARG, "reconstruction factors: null array");
  if (s->dev.T > 65535) return fail(MFS_ERR_ARG, "near-field calls support at most 65535 bodies (one grid row each)");
  const int ns = s->n_shapes;
  bool same = (int)s->near_key.size() == ns;
  for (int i = 0; i < ns; ++i) {
    const mfs_recon* r = recon[i];
    if (!r) return fail(MFS_ERR_ARG, "reconstruction factors: null handle for shape " + std::to_string(i));
    if (r->f.dim != s->dev.dim || r->f.k != s->k_of_shape[i] ||
        std::fabs(r->f.kappa - s->dev.kappa) > 1e-12 * s->dev.kappa)
      return fail(MFS_ERR_ARG, "reconstruction factors of shape " + std::to_string(i) +
                                   " do not match the scene (dim, k or kappa)");
    same = same && s->near_key[i] == r->id;
  }
  if (same) return MFS_OK;
  const int64_t T = s->dev.T;
  std::vector<int32_t> shape_of(T);
  MFS_HIP_TRY(hipMemcpyAsync(shape_of.data(), s->shape_of.p, sizeof(int32_t) * T, hipMemcpyDeviceToHost, st));
  MFS_HIP_TRY(hipStreamSynchronize(st));
  std::vector<int64_t> cptr(T + 1, 0), sptr(T + 1, 0);
  s->bodies_of_shape.assign(ns, {});
  for (int64_t b = 0; b < T; ++b) {
    const int sh = shape_of[b];
    cptr[b + 1] = cptr[b] + recon[sh]->f.m;
    sptr[b + 1] = sptr[b] + recon[sh]->f.n;
    s->bodies_of_shape[sh].push_back((int32_t)b);
  }
  std::vector<const void*> colloc(ns), src(ns), Y(ns);
  std::vector<int32_t> mm(ns), nn(ns);
  std::vector<double> psi2(ns);
  NearTables t{};
  t.mmax = t.nmax = t.kmax = 0;
  for (int i = 0; i < ns; ++i) {
    const ReconFactors& f = recon[i]->f;
    colloc[i] = f.colloc;
    src[i] = f.src;
    Y[i] = f.Y;
    mm[i] = f.m;
    nn[i] = f.n;
    psi2[i] = recon[i]->psi_radius * recon[i]->psi_radius;
    t.mmax = std::max(t.mmax, f.m);
    t.nmax = std::max(t.nmax, f.n);
    t.kmax = std::max(t.kmax, f.k);
  }
  // one host image of all tables, copied in one go
  std::vector<char> img;
  auto put = [&](const void* p, size_t bytes) {
    const size_t off = (img.size() + 255) / 256 * 256;
    img.resize(off + bytes);
    std::memcpy(img.data() + off, p, bytes);
    return off;
  };
  const size_t oC = put(colloc.data(), sizeof(void*) * ns), oS = put(src.data(), sizeof(void*) * ns),
               oY = put(Y.data(), sizeof(void*) * ns), oM = put(mm.data(), sizeof(int32_t) * ns),
               oN = put(nn.data(), sizeof(int32_t) * ns), oP = put(psi2.data(), sizeof(double) * ns),
               oCp = put(cptr.data(), sizeof(int64_t) * (T + 1)), oSp = put(sptr.data(), sizeof(int64_t) * (T + 1));
  std::vector<size_t> oB(ns);
  const int32_t none = -1;  // a shape with no bodies still gets a (never read) one-entry list
  for (int i = 0; i < ns; ++i) {
    const std::vector<int32_t>& bl = s->bodies_of_shape[i];
    oB[i] = bl.empty() ? put(&none, sizeof(int32_t)) : put(bl.data(), sizeof(int32_t) * bl.size());
  }
  MFS_TRY(ensure(s->near_tab, img.size(), &s->bytes, st));
  char* base = static_cast<char*>(s->near_tab.p);
  MFS_HIP_TRY(hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, st));
  MFS_HIP_TRY(hipStreamSynchronize(st));  // img is released on return
  t.colloc_of_shape = reinterpret_cast<const double* const*>(base + oC);
  t.src_of_shape = reinterpret_cast<const double* const*>(base + oS);
  t.Y_of_shape = reinterpret_cast<const c128* const*>(base + oY);
  t.m_of_shape = reinterpret_cast<const int32_t*>(base + oM);
  t.n_of_shape = reinterpret_cast<const int32_t*>(base + oN);
  t.psi2_of_shape = reinterpret_cast<const double*>(base + oP);
  t.cptr = reinterpret_cast<const int64_t*>(base + oCp);
  t.sptr = reinterpret_cast<const int64_t*>(base + oSp);
  t.Mtot = cptr[T];
  t.Ntot = sptr[T];
  s->bodies_dev.assign(ns, nullptr);
  for (int i = 0; i < ns; ++i) s->bodies_dev[i] = reinterpret_cast<const int32_t*>(base + oB[i]);
  s->near = t;
  s->near_key.resize(ns);
  for (int i = 0; i < ns; ++i) s->near_key[i] = recon[i]->id;
  return MFS_OK;
}
// y = S G_hat q with q already complex64 (a single-precision Krylov basis vector) and y complex128.
mfs_status apply_mixed_from32(mfs_scene* s, const c64* q32, c128* y, int R, hipStream_t st) {
  PartialF32 p;
  MFS_TRY(pair_f32(s, q32, R, st, &p));
  MFS_HIP_TRY(launch_sapply_mixed(s->dev, p.part, p.slices, nullptr, 0.0, y, R, (int)s->kmax, st, p.pptr, p.NP));
  return MFS_OK;
}

// y = q + S G_hat q with every intermediate in the caller-supplied buffer `buf` of `cap` bytes (the
// static scratch): the same kernels as apply_f64 / apply_f32, with the launch shape cut to what
// fits.  The symmetric kernel runs when the scene's shape picks it and its slices (and the padded
// charges) fit; otherwise the body-phase (or matrix-core) kernel with as many source slices as fit,
// up to the scene's own count.  Every slice a consumer reads is written by the pair kernel first,
// so nothing in `buf` needs to start at zero.  No allocation of any kind.
mfs_status apply_in_buffer(mfs_scene* s, const void* q, void* y, int R, mfs_prec prec, void* buf, size_t cap,
                           hipStream_t st) {
  const int64_t N = s->dev.N;
  if (prec == MFS_FP64) {
    const size_t per_slice = (size_t)R * N * sizeof(c128);
    const int fit = (int)std::min<size_t>(cap / per_slice, 1024);
    if (fit < 1)
      return fail(MFS_ERR_ARG, "apply_static: one FP64 partial slice needs " + std::to_string(per_slice) +
                                   " bytes (R x N x 16), more than the static scratch's " + std::to_string(cap));
    const int nch = std::min(shape_for(s, true, R).nchunks, fit);
    c128* part = static_cast<c128*>(buf);
    MFS_HIP_TRY(launch_ghat_f64(s->dev, static_cast<const c128*>(q), R, part, nch, st, false));
    MFS_HIP_TRY(launch_sapply_f64(s->dev, part, nch, static_cast<const c128*>(q), 1.0, static_cast<c128*>(y), R,
                                  (int)s->kmax, st));
    return MFS_OK;
  }
  const c64* q32 = static_cast<const c64*>(q);
  LaunchShape ls = shape_for(s, false, R);
  if (ls.sym == 1) {
    const bool padded = sym_padded(s->dev);
    const int64_t rows = f32_rows(s, ls);
    const int slices = f32_slices(s, ls, R);
    const size_t part_bytes = ((size_t)slices * R * rows * sizeof(c64) + 255) / 256 * 256;
    const size_t need = part_bytes + (padded ? (size_t)R * rows * sizeof(c64) : 0);
    if (need <= cap) {
      c64* part = static_cast<c64*>(buf);
      const c64* qs = q32;
      if (padded) {
        c64* qp = reinterpret_cast<c64*>(static_cast<char*>(buf) + part_bytes);
        MFS_HIP_TRY(launch_gather_pad(s->dev, q32, R, qp, st));
        qs = qp;
      }
      MFS_HIP_TRY(launch_ghat_f32_sym(sym_view(s->dev), qs, R, part, ls.nchunks, ls.rt, st));
      MFS_HIP_TRY(launch_sapply_f32(s->dev, part, slices, q32, 1.0f, static_cast<c64*>(y), R, (int)s->kmax, st,
                                    padded ? s->dev.pad_ptr : nullptr, padded ? rows : 0));
      return MFS_OK;
    }
    // the symmetric kernel's slices do not fit: the plain kernel, with the plain heuristic's slices
    ls.nchunks = pair_chunks_for(N, N, tpt_for(MFS_FP32));
  }
  const size_t per_slice = (size_t)R * N * sizeof(c64);
  // the FP16 matrix-core kernel's split charges sit after the partial slices when both fit (else
  // the FP32 matrix-core kernel runs)
  const size_t split_bytes = ghat_uses_mfma16(s->dev, R) ? (ghat_split_bytes(s->dev, R) + 255) / 256 * 256 : 0;
  const size_t slice_room = split_bytes && cap >= split_bytes + per_slice ? (cap - split_bytes) / 256 * 256 : cap;
  const int fit = (int)std::min<size_t>(slice_room / per_slice, 1024);
  if (fit < 1)
    return fail(MFS_ERR_ARG, "apply_static: one FP32 partial slice needs " + std::to_string(per_slice) +
                                 " bytes (R x N x 8), more than the static scratch's " + std::to_string(cap));
  const int nch = std::min(ls.nchunks, fit);
  c64* part = static_cast<c64*>(buf);
  void* split = slice_room < cap ? static_cast<char*>(buf) + slice_room : nullptr;
  MFS_HIP_TRY(launch_ghat_f32(s->dev, q32, R, part, nch, st, ls.rt, split));
  MFS_HIP_TRY(launch_sapply_f32(s->dev, part, nch, q32, 1.0f, static_cast<c64*>(y), R, (int)s->kmax, st));
  return MFS_OK;
}

// ------------------------------------------------------------- block GMRES ---
// Workspace of a block solve (carved from the scene's Krylov workspace): basis slots of N x R,
// the packed block Hessenberg matrix, Householder vectors, least-squares right side and solution,
// partial sums of the inner products, and R x R factors.
struct BlockWork {
  int64_t N = 0;
  int R = 0, m = 0;
  bool v32 = false;
  void* V = nullptr;
  c128 *Hp = nullptr, *refl = nullptr, *g = nullptr, *Y = nullptr, *h2 = nullptr, *part = nullptr;
  c128 *gram = nullptr, *F = nullptr, *Finv = nullptr, *rtot = nullptr;
  double *bnorm = nullptr, *res = nullptr, *npart = nullptr, *wn = nullptr;
  int32_t *flag = nullptr, *dep = nullptr;
  int nblk = 0;
  c128 *W = nullptr, *Wt = nullptr;  // N x R blocks
  c128 *q1 = nullptr, *coef = nullptr;  // completion of dependent columns: one vector, its coefficients
  c64 *W32 = nullptr, *coef32 = nullptr;  // complex64 copies of W and of the Gram-Schmidt coefficients
  // pinned host slots: R doubles, 2R doubles, a flag and R ints
  double* res_pin = nullptr;
  double* wn_pin = nullptr;
  double reorth_eta = 0.1;  // second Gram-Schmidt pass when some column keeps less than this of its norm
  int* n_second = nullptr;  // counts the steps that took it
  int32_t *flag_pin = nullptr, *dep_pin = nullptr;
  hipEvent_t ev = nullptr;
  size_t vbytes() const { return v32 ? sizeof(c64) : sizeof(c128); }
  void* slot(int j) const { return static_cast<char*>(V) + (size_t)j * R * N * vbytes(); }
  int64_t hoff(int j) const { return (int64_t)R * R * ((int64_t)j * (j + 3) / 2); }
  int64_t ldg() const { return (int64_t)(m + 1) * R; }
};

// Bytes of the block workspace for N, R, m block steps (basis of complex64 when v32).
// Workspace of the per-column solve (GMRES per right-hand side): the basis ((m+1) N R, complex64 with
// v32), the Hessenberg matrices, rotations, right sides and coefficient vectors, norm partials and
// the deflation vectors, each carved at 256-byte alignment.
struct ColumnWork {
  size_t V, H, cs, sn, g, h1, h2, y, beta, bn, res, hn, act, jl, wn, ro, nro, part, jdev, tol, q, cr, ee, jold, rn2,
      keep, total;
};

ColumnWork column_work_layout(int64_t N, int R, int m, bool v32) {
  const size_t NR = (size_t)N * R;
  const size_t szV = (v32 ? sizeof(c64) : sizeof(c128)) * (size_t)(m + 1) * NR;
  const size_t szH = sizeof(c128) * (size_t)R * m * (m + 1);
  const size_t szRm = sizeof(c128) * (size_t)R * m;
  const size_t szRm1 = sizeof(c128) * (size_t)R * (m + 1);
  const size_t szPart = sizeof(double) * 2 * (size_t)R * (m + 1) * krylov_part_blocks(N);
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  ColumnWork L{};
  L.V = carve(szV);
  L.H = carve(szH);
  L.cs = carve(szRm);
  L.sn = carve(szRm);
  L.g = carve(szRm1);
  L.h1 = carve(szRm1);
  L.h2 = carve(szRm1);
  L.y = carve(szRm);
  L.beta = carve(8 * R);
  L.bn = carve(8 * R);
  L.res = carve(8 * R);
  L.hn = carve(8 * R);
  L.act = carve(4 * R);
  L.jl = carve(4 * R);
  L.wn = carve(8 * R);
  L.ro = carve(4 * R);
  L.nro = carve(4 * R);
  L.part = carve(szPart);
  L.jdev = carve(sizeof(int32_t));
  L.tol = carve(sizeof(double));
  L.q = carve(szRm1);
  L.cr = carve(szRm1);
  L.ee = carve(szRm1);
  L.jold = carve(4 * R);
  L.rn2 = carve(8 * R);
  L.keep = carve(4 * R);
  L.total = off;
  return L;
}

size_t block_work_bytes(int64_t N, int R, int m, bool v32, int64_t* offs) {
  size_t off = 0;
  int idx = 0;
  auto carve = [&](size_t bytes) {
    if (offs) offs[idx] = (int64_t)off;
    ++idx;
    off += (bytes + 255) / 256 * 256;
  };
  const size_t RR = (size_t)R * R;
  carve((v32 ? sizeof(c64) : sizeof(c128)) * (size_t)(m + 1) * R * N);  // V
  carve(sizeof(c128) * RR * ((size_t)m * (m + 3) / 2));                // Hp
  carve(sizeof(c128) * (size_t)m * R * (R + 1));                       // refl
  carve(sizeof(c128) * (size_t)(m + 1) * R * R);                       // g
  carve(sizeof(c128) * (size_t)m * R * R);                             // Y
  carve(sizeof(c128) * (size_t)(m + 1) * R * R);                       // h2
  carve(sizeof(c128) * (size_t)std::max<int64_t>(kBdotsPartMax, (int64_t)(m + 1) * R) * R);  // part
  for (int i = 0; i < 4; ++i) carve(sizeof(c128) * RR);                // gram, F, Finv, rtot
  carve(sizeof(double) * R);                                           // bnorm
  carve(sizeof(double) * R);                                           // res
  carve(sizeof(double) * 2 * (size_t)R * krylov_part_blocks(N));       // norm partials
  carve(sizeof(int32_t));                                              // flag
  carve(sizeof(c128) * (size_t)R * N);                                 // W
  carve(sizeof(c128) * (size_t)R * N);                                 // Wt
  carve(sizeof(int32_t) * R);                                          // dep
  carve(sizeof(c128) * (size_t)N);                                     // q1
  carve(sizeof(c128) * (size_t)(m + 1) * R);                           // coef
  carve(sizeof(double) * 2 * R);                                       // wn: |W| before and after a pass
  carve(sizeof(c64) * (size_t)R * N);                                  // W32
  carve(sizeof(c64) * (size_t)(m + 1) * R * R);                        // coef32
  return off;
}

BlockWork block_work_at(char* base, int64_t N, int R, int m, bool v32) {
  int64_t o[32];
  block_work_bytes(N, R, m, v32, o);
  BlockWork b;
  b.N = N;
  b.R = R;
  b.m = m;
  b.v32 = v32;
  b.V = base + o[0];
  b.Hp = reinterpret_cast<c128*>(base + o[1]);
  b.refl = reinterpret_cast<c128*>(base + o[2]);
  b.g = reinterpret_cast<c128*>(base + o[3]);
  b.Y = reinterpret_cast<c128*>(base + o[4]);
  b.h2 = reinterpret_cast<c128*>(base + o[5]);
  b.part = reinterpret_cast<c128*>(base + o[6]);
  b.gram = reinterpret_cast<c128*>(base + o[7]);
  b.F = reinterpret_cast<c128*>(base + o[8]);
  b.Finv = reinterpret_cast<c128*>(base + o[9]);
  b.rtot = reinterpret_cast<c128*>(base + o[10]);
  b.bnorm = reinterpret_cast<double*>(base + o[11]);
  b.res = reinterpret_cast<double*>(base + o[12]);
  b.npart = reinterpret_cast<double*>(base + o[13]);
  b.flag = reinterpret_cast<int32_t*>(base + o[14]);
  b.W = reinterpret_cast<c128*>(base + o[15]);
  b.Wt = reinterpret_cast<c128*>(base + o[16]);
  b.dep = reinterpret_cast<int32_t*>(base + o[17]);
  b.q1 = reinterpret_cast<c128*>(base + o[18]);
  b.coef = reinterpret_cast<c128*>(base + o[19]);
  b.wn = reinterpret_cast<double*>(base + o[20]);
  b.W32 = reinterpret_cast<c64*>(base + o[21]);
  b.coef32 = reinterpret_cast<c64*>(base + o[22]);
  b.nblk = krylov_nblk(N);
  return b;
}

// q1 -= A (A^H q1) for the K columns of A (N x K, complex64 when a32): one Gram-Schmidt pass.
mfs_status project_out(const BlockWork& bw, const void* A, bool a32, int K, hipStream_t st) {
  if (K <= 0) return MFS_OK;
  const int ns = bdots_splits(bw.N, K);
  MFS_HIP_TRY(launch_bdots(A, a32, bw.N, K, bw.q1, bw.N, 1, bw.N, bw.part, ns, st));
  MFS_HIP_TRY(launch_breduce(bw.part, ns, K, 1, bw.coef, K, false, nullptr, 0, st));
  MFS_HIP_TRY(launch_bgemm_nk(A, a32, bw.N, bw.N, K, bw.coef, K, 1, -1.0, 1.0, bw.q1, bw.N, bw.q1, bw.N, st));
  return MFS_OK;
}

// Orthonormal basis of the columns of W (N x R): shifted CholeskyQR3 (Fukaya et al. 2020) with the
// columns scaled to unit norm in the first step, so that columns of very different size (right-hand
// sides at different stages of convergence) do not square the condition number.  W = Q Rtot with
// Rtot upper triangular (bw.rtot); Q is left in bw.W or bw.Wt, returned.  A column of W that lies
// in the span of the columns before it gets a zero row of Rtot; its column of Q is then completed
// with a pseudo-random vector orthogonalised (twice) against the first nprev basis columns and the
// rest of Q, so that Q stays orthonormal and W = Q Rtot still holds.
mfs_status block_qr(const BlockWork& bw, c128* W, c128** Q, int nprev, uint64_t seed, hipStream_t st) {
  const int64_t N = bw.N;
  const int R = bw.R;
  const double u = 1.1102230246251565e-16;  // 2^-53
  const double shift = 11.0 * ((double)N * R + (double)R * (R + 1)) * u * R;  // |W D^-1|_2^2 <= R
  c128* cur = W;
  c128* nxt = W == bw.W ? bw.Wt : bw.W;
  const int ns = bdots_splits(N, R);
  MFS_HIP_TRY(hipMemsetAsync(bw.flag, 0, sizeof(int32_t), st));
  for (int p = 0; p < 3; ++p) {
    MFS_HIP_TRY(launch_bdots(cur, false, N, R, cur, N, R, N, bw.part, ns, st));
    MFS_HIP_TRY(launch_breduce(bw.part, ns, R, R, bw.gram, R, false, nullptr, 0, st));
    // after the shifted first step the columns have unit norm: a pivot^2 of 1e-12 marks a column
    // that only rounding separated from the span of the others
    MFS_HIP_TRY(launch_chol(bw.gram, R, p == 0, p == 0 ? shift : 0.0, p == 0, p == 0 ? 0.0 : 1e-12, bw.F, bw.Finv,
                            bw.rtot, bw.dep, bw.flag, st));
    MFS_HIP_TRY(launch_bgemm_nk(cur, false, N, N, R, bw.Finv, R, R, 1.0, 0.0, nullptr, 0, nxt, N, st));
    std::swap(cur, nxt);
  }
  *Q = cur;
  MFS_HIP_TRY(hipMemcpyAsync(bw.flag_pin, bw.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MFS_HIP_TRY(hipMemcpyAsync(bw.dep_pin, bw.dep, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
  MFS_HIP_TRY(hipEventRecord(bw.ev, st));
  MFS_HIP_TRY(hipEventSynchronize(bw.ev));
  if (!*bw.flag_pin) return MFS_OK;
  for (int k = 0; k < R; ++k) {
    if (!bw.dep_pin[k]) continue;
    MFS_HIP_TRY(launch_fill_random(bw.q1, N, seed * 64 + (uint64_t)k, st));
    for (int pass = 0; pass < 2; ++pass) {
      MFS_TRY(project_out(bw, bw.V, bw.v32, nprev, st));
      MFS_TRY(project_out(bw, cur, false, R, st));  // column k of Q is zero until filled
    }
    MFS_HIP_TRY(launch_norms(bw.q1, N, 1, bw.npart, bw.nblk, bw.res, st));
    MFS_HIP_TRY(hipMemcpyAsync(bw.res_pin, bw.res, sizeof(double), hipMemcpyDeviceToHost, st));
    MFS_HIP_TRY(hipStreamSynchronize(st));
    const double nrm = bw.res_pin[0];
    if (!(nrm > 0.0)) return fail(MFS_ERR_HIP, "block QR: completion vector vanished");
    MFS_HIP_TRY(launch_axpby(bw.q1, bw.q1, cur + (int64_t)k * N, 1.0 / nrm, 0.0, N, st));
  }
  return MFS_OK;
}

// Store the N x R block Q into basis slot j (rounded to complex64 when the basis is).
mfs_status block_store_slot(const BlockWork& bw, int j, const c128* Q, hipStream_t st) {
  const int64_t NR = bw.N * bw.R;
  if (bw.v32) MFS_HIP_TRY(launch_to_c64(Q, static_cast<c64*>(bw.slot(j)), NR, st));
  else MFS_HIP_TRY(hipMemcpyAsync(bw.slot(j), Q, sizeof(c128) * NR, hipMemcpyDeviceToDevice, st));
  return MFS_OK;
}

// Where one block Arnoldi process keeps its state: first basis slot, packed Hessenberg matrix and
// Householder vectors (a later process's follow those of a kept one).
struct BlockProcess {
  int o = 0;
  c128* Hp = nullptr;
  c128* refl = nullptr;
};

// The first cycle's process, kept for the deflated correction cycles (GCRO, de Sturler 1996, the
// block form of the single-right-hand-side path): after k block steps K~ V_k = V_{k+1} Hbar with
// Hbar = Q [U; 0] (Q from the stored reflectors), C = V_{k+1} Q_{:, 0:kR} is an orthonormal basis of
// K~ V_k, and C C^H = V_{k+1} (I - q q^H) V_{k+1}^H with q the last R columns of Q.
struct KeptSpace {
  int k = 0;  // block steps (slots 0..k)
  const c128* Hp = nullptr;
  const c128* refl = nullptr;
};

// Y = U^{-1} rhs for the first J column blocks of a process's triangular factor (block back
// substitution; rhs, leading dimension ldr, is overwritten).
mfs_status block_backsolve(const BlockWork& bw, const c128* Hp, int J, c128* rhs, int64_t ldr, hipStream_t st) {
  const int R = bw.R;
  for (int i = J - 1; i >= 0; --i) {
    const c128* Ui = Hp + bw.hoff(i);
    const int64_t ldu = (int64_t)(i + 2) * R;
    MFS_HIP_TRY(launch_btrsm_diag(Ui + (int64_t)i * R, ldu, rhs + (int64_t)i * R, ldr, bw.Y + (int64_t)i * R,
                                  (int64_t)bw.m * R, R, st));
    if (i > 0)
      MFS_HIP_TRY(launch_bgemm_nk(Ui, false, ldu, (int64_t)i * R, R, bw.Y + (int64_t)i * R, (int64_t)bw.m * R, R,
                                  -1.0, 1.0, rhs, ldr, rhs, ldr, st));
  }
  return MFS_OK;
}

// a <- (I - q q^H) a for the first (k+1)R rows of the R columns of a (leading dimension lda): Q^H,
// zero the last R rows, Q.
mfs_status project_kept(const BlockWork& bw, const KeptSpace& kp, c128* a, int64_t lda, hipStream_t st) {
  const int R = bw.R;
  const int64_t kR = (int64_t)kp.k * R;
  MFS_HIP_TRY(launch_bhess_apply(kp.refl, R, 0, kR, a, lda, R, st));
  MFS_HIP_TRY(hipMemset2DAsync(a + kR, sizeof(c128) * lda, 0, sizeof(c128) * R, R, st));
  MFS_HIP_TRY(launch_bhess_apply_rev(kp.refl, R, 0, kR, a, lda, R, st));
  return MFS_OK;
}

// One block GMRES cycle on the residual block r (N x R), at most mlim block steps, stopping when
// every column's residual estimate |g_{j+1,c}| falls to ktol times that column's starting norm;
// x += the correction.  `apply(slot)` computes bw.W = S G_hat V_slot and `apply_vec(v)` computes
// bw.W = S G_hat v for an N x R complex128 block (the operator without its identity, which goes onto
// the Hessenberg diagonal).  With a kept space (kp.k > 0) the process runs on (I - C C^H) K~ from
// (I - C C^H) r with its basis from slot pr.o, and the correction is W y + V_k U^{-1} C^H (r - K~ W y).
template <typename Apply, typename ApplyVec>
mfs_status block_cycle(const BlockWork& bw, const BlockProcess& pr, const KeptSpace& kp, const c128* r, c128* x,
                       double ktol, int mlim, Apply apply, ApplyVec apply_vec, int verbose, int* steps_out,
                       double* est_out, hipStream_t st) {
  const int64_t N = bw.N;
  const int R = bw.R;
  const int64_t ldg = bw.ldg();
  const int o = pr.o;
  const bool defl = kp.k > 0;
  const int ko = defl ? kp.k + 1 : 0;  // kept basis blocks
  // Gram-Schmidt on the FP32 matrix cores when the basis is complex64 (the mixed solve): its
  // rounding (~3e-7 of the norms) is below the FP32 operator's own error
  const bool gs32 = bw.v32;
  MFS_HIP_TRY(launch_norms(r, N, R, bw.npart, bw.nblk, bw.bnorm, st));
  // starting block: r (projected off C with a kept space), a pseudo-random vector for a zero column
  MFS_HIP_TRY(hipMemcpyAsync(bw.W, r, sizeof(c128) * N * R, hipMemcpyDeviceToDevice, st));
  if (defl) {
    const int K = ko * R;
    const int ns = bdots_splits(N, K);
    MFS_HIP_TRY(launch_bdots(bw.V, bw.v32, N, K, bw.W, N, R, N, bw.part, ns, st));
    MFS_HIP_TRY(launch_breduce(bw.part, ns, K, R, bw.h2, ldg, false, nullptr, 0, st));
    MFS_TRY(project_kept(bw, kp, bw.h2, ldg, st));
    MFS_HIP_TRY(launch_bgemm_nk(bw.V, bw.v32, N, N, K, bw.h2, ldg, R, -1.0, 1.0, bw.W, N, bw.W, N, st));
  }
  MFS_HIP_TRY(launch_fill_zero_columns(bw.W, N, R, bw.bnorm, st));
  c128* Q = nullptr;
  MFS_TRY(block_qr(bw, bw.W, &Q, defl ? ko * R : 0, (uint64_t)o << 20, st));
  MFS_TRY(block_store_slot(bw, o, Q, st));
  // g = [B0; 0]: the starting block's coefficients, zero for the zero columns; the estimate is
  // relative to |r|, not to |(I - C C^H) r|
  MFS_HIP_TRY(hipMemsetAsync(bw.g, 0, sizeof(c128) * ldg * R, st));
  MFS_HIP_TRY(hipMemcpy2DAsync(bw.g, sizeof(c128) * ldg, bw.rtot, sizeof(c128) * R, sizeof(c128) * R, R,
                               hipMemcpyDeviceToDevice, st));
  MFS_HIP_TRY(launch_mask_zero_columns(bw.g, ldg, R, R, bw.bnorm, st));
  int J = 0;
  double est = 1.0;
  for (int j = 0; j < mlim && o + j + 1 <= bw.m; ++j) {
    MFS_TRY(apply(o + j));  // bw.W = S G_hat V_{o+j}
    const int K = (o + j + 1) * R;  // every basis block so far (kept and this process's)
    c128* hcol = pr.Hp + bw.hoff(j);
    const int64_t ldh = (int64_t)(j + 2) * R;
    const int ns = bdots_splits(N, K);
    // block classical Gram-Schmidt, two passes.  Without a kept space: H(0..j, j) = V^H W, W -= V H.
    // With one, the coefficients on the kept vectors are replaced by their part along C (the rest
    // of the kept space stays in W) and only this process's coefficients enter its Hessenberg matrix.
    MFS_HIP_TRY(launch_norms(bw.W, N, R, bw.npart, bw.nblk, bw.wn, st));
    // inner products V^H W (FP32 matrix cores on complex64 copies of W when gs32)
    auto dots = [&]() -> mfs_status {
      if (gs32) {
        MFS_HIP_TRY(launch_to_c64(bw.W, bw.W32, N * R, st));
        MFS_HIP_TRY(launch_bdots32_b64(static_cast<const c64*>(bw.V), N, K, bw.W32, N, R, N, bw.part, ns, st));
      } else {
        MFS_HIP_TRY(launch_bdots(bw.V, bw.v32, N, K, bw.W, N, R, N, bw.part, ns, st));
      }
      return MFS_OK;
    };
    // W -= V C for the K x R coefficients C (leading dimension ldc)
    auto update = [&](const c128* C, int64_t ldc) -> mfs_status {
      if (gs32) {
        MFS_HIP_TRY(launch_to_c64_2d(C, ldc, K, R, bw.coef32, K, st));
        MFS_HIP_TRY(launch_bgemm32_c64(static_cast<const c64*>(bw.V), N, N, K, bw.coef32, K, R, -1.0, 1.0, bw.W, N,
                                       bw.W, N, st));
      } else {
        MFS_HIP_TRY(launch_bgemm_nk(bw.V, bw.v32, N, N, K, C, ldc, R, -1.0, 1.0, bw.W, N, bw.W, N, st));
      }
      return MFS_OK;
    };
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        // second pass only where the first cancelled: some column kept less than eta of its norm
        MFS_HIP_TRY(launch_norms(bw.W, N, R, bw.npart, bw.nblk, bw.wn + R, st));
        MFS_HIP_TRY(hipMemcpyAsync(bw.wn_pin, bw.wn, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, st));
        MFS_HIP_TRY(hipEventRecord(bw.ev, st));
        MFS_HIP_TRY(hipEventSynchronize(bw.ev));
        bool again = false;
        for (int c = 0; c < R; ++c) again = again || !(bw.wn_pin[R + c] >= bw.reorth_eta * bw.wn_pin[c]);
        if (!again) break;
        if (bw.n_second) ++*bw.n_second;
      }
      MFS_TRY(dots());
      if (!defl) {
        MFS_HIP_TRY(launch_breduce(bw.part, ns, K, R, hcol, ldh, pass == 1, pass == 1 ? bw.h2 : nullptr, ldg, st));
        if (pass == 0) MFS_TRY(update(hcol, ldh));
        else MFS_TRY(update(bw.h2, ldg));
      } else {
        MFS_HIP_TRY(launch_breduce(bw.part, ns, K, R, bw.h2, ldg, false, nullptr, 0, st));
        // this process's rows go to its Hessenberg column (set, then accumulated); its basis follows
        // the kept blocks directly (o = k + 1)
        MFS_HIP_TRY(launch_copy2d(bw.h2 + (int64_t)o * R, ldg, (int64_t)(j + 1) * R, R, hcol, ldh, pass == 1, st));
        MFS_TRY(project_kept(bw, kp, bw.h2, ldg, st));
        MFS_TRY(update(bw.h2, ldg));
      }
    }
    // W = V_{o+j+1} H(j+1, j)
    MFS_TRY(block_qr(bw, bw.W, &Q, K, ((uint64_t)o << 20) + (uint64_t)j + 1, st));
    MFS_TRY(block_store_slot(bw, o + j + 1, Q, st));
    MFS_HIP_TRY(hipMemcpy2DAsync(hcol + (int64_t)(j + 1) * R, sizeof(c128) * ldh, bw.rtot, sizeof(c128) * R,
                                 sizeof(c128) * R, R, hipMemcpyDeviceToDevice, st));
    MFS_HIP_TRY(launch_add_identity(hcol, ldh, (int64_t)j * R, R, st));
    // QR of the Hessenberg matrix: earlier reflectors on the new column block, then its own
    MFS_HIP_TRY(launch_bhess_apply(pr.refl, R, 0, (int64_t)j * R, hcol, ldh, R, st));
    MFS_HIP_TRY(launch_bhess_newqr(pr.refl, R, (int64_t)j * R, hcol, ldh, st));
    MFS_HIP_TRY(launch_bhess_apply(pr.refl, R, (int64_t)j * R, (int64_t)(j + 1) * R, bw.g, ldg, R, st));
    MFS_HIP_TRY(launch_bres(bw.g, ldg, (int64_t)(j + 1) * R, R, bw.bnorm, bw.res, st));
    MFS_HIP_TRY(hipMemcpyAsync(bw.res_pin, bw.res, sizeof(double) * R, hipMemcpyDeviceToHost, st));
    MFS_HIP_TRY(hipEventRecord(bw.ev, st));
    MFS_HIP_TRY(hipEventSynchronize(bw.ev));
    J = j + 1;
    est = 0.0;
    for (int c = 0; c < R; ++c) est = std::max(est, bw.res_pin[c]);
    if (verbose > 1 && (J % 50 == 0))
      std::fprintf(stderr, "[mfs_solve block] step %d of cycle, max estimate %.3e\n", J, est);
    if (est <= ktol) break;
  }
  // W y: Y = U^{-1} g (block back substitution), then x += V_{o..o+J-1} Y
  MFS_TRY(block_backsolve(bw, pr.Hp, J, bw.g, ldg, st));
  if (!defl) {
    if (J > 0)
      MFS_HIP_TRY(launch_bgemm_nk(bw.slot(o), bw.v32, N, N, J * R, bw.Y, (int64_t)bw.m * R, R, 1.0, 1.0, x, N, x, N,
                                  st));
  } else {
    // d1 = W y into Wt; x += d1; u = r - K~ d1 = r - d1 - S G_hat d1; z = Q^H V_{0..k}^H u;
    // x += V_{0..k-1} U^{-1} z_{0..kR-1}
    MFS_HIP_TRY(launch_bgemm_nk(bw.slot(o), bw.v32, N, N, J * R, bw.Y, (int64_t)bw.m * R, R, 1.0, 0.0, nullptr, 0,
                                bw.Wt, N, st));
    MFS_HIP_TRY(launch_axpby(x, bw.Wt, x, 1.0, 1.0, N * R, st));
    MFS_TRY(apply_vec(bw.Wt));  // bw.W = S G_hat d1
    MFS_HIP_TRY(launch_axpby(r, bw.W, bw.W, 1.0, -1.0, N * R, st));
    MFS_HIP_TRY(launch_axpby(bw.W, bw.Wt, bw.W, 1.0, -1.0, N * R, st));
    const int K = ko * R;
    const int ns = bdots_splits(N, K);
    MFS_HIP_TRY(launch_bdots(bw.V, bw.v32, N, K, bw.W, N, R, N, bw.part, ns, st));
    MFS_HIP_TRY(launch_breduce(bw.part, ns, K, R, bw.h2, ldg, false, nullptr, 0, st));
    MFS_HIP_TRY(launch_bhess_apply(kp.refl, R, 0, (int64_t)kp.k * R, bw.h2, ldg, R, st));
    MFS_TRY(block_backsolve(bw, kp.Hp, kp.k, bw.h2, ldg, st));
    MFS_HIP_TRY(launch_bgemm_nk(bw.V, bw.v32, N, N, kp.k * R, bw.Y, (int64_t)bw.m * R, R, 1.0, 1.0, x, N, x, N, st));
  }
  *steps_out = J;
  *est_out = est;
  return MFS_OK;
}

// The block solve behind mfs_solve with opts->block (2 <= R <= 64): one block Krylov space for the
// R right-hand sides.  MFS_MIXED: each cycle runs on the FP32 operator (basis in complex64 with
// basis32) on the current FP64 residual and asks for the reduction the outer tolerance still
// needs (at most down to inner_tol), then the FP64 residual is formed (iterative refinement).
// MFS_FP64: cycles of restarted block GMRES with the FP64 operator, the FP64 residual checked after
// each.  Converged right-hand sides stay in the block (their residuals keep shrinking).
mfs_status solve_block(mfs_scene* s, const c128* vhat, int R, const mfs_solve_opts* opts, c128* x,
                       mfs_solve_info* info, hipStream_t st, std::chrono::steady_clock::time_point t0) {
  if (R > 64) return fail(MFS_ERR_ARG, "solve: block GMRES takes at most 64 right-hand sides");
  const mfs_prec prec = opts->prec;
  const int64_t N = s->dev.N, NR = N * R;
  const int m = opts->restart;
  const bool v32 = prec == MFS_MIXED && opts->basis32 != 0;
  MFS_TRY(ensure(s->kry, block_work_bytes(N, R, m, v32, nullptr), &s->bytes, st));
  BlockWork bw = block_work_at(static_cast<char*>(s->kry.p), N, R, m, v32);
  MFS_TRY(ensure(s->vecs, 3 * sizeof(c128) * (size_t)NR + 256, &s->bytes, st));
  c128* b = static_cast<c128*>(s->vecs.p);
  c128* r = b + NR;
  c128* w = r + NR;
  size_t pin_bytes = 0;
  hipError_t pin_err = hipSuccess;
  char* pin = static_cast<char*>(
      pinned_alloc(sizeof(double) * 3 * R + sizeof(int32_t) * (R + 2) + 64, &pin_bytes, &pin_err));
  if (!pin) return fail(MFS_ERR_NOMEM, std::string("pinned host allocation failed: ") + hipGetErrorString(pin_err));
  struct PinGuard {
    void* p;
    size_t n;
    hipEvent_t ev;
    ~PinGuard() {
      if (ev) {
        (void)hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
      }
      pinned_free(p, n);
    }
  } guard{pin, pin_bytes, nullptr};
  MFS_HIP_TRY(hipEventCreateWithFlags(&guard.ev, hipEventDisableTiming));
  double* res_pin = reinterpret_cast<double*>(pin);
  bw.res_pin = res_pin;
  bw.wn_pin = res_pin + R;
  bw.flag_pin = reinterpret_cast<int32_t*>(pin + sizeof(double) * 3 * R);
  bw.dep_pin = bw.flag_pin + 1;
  bw.ev = guard.ev;

  std::vector<double> bnorm(R), relres(R, 1.0);
  auto read_norms = [&](const c128* v, std::vector<double>& out) -> mfs_status {
    MFS_HIP_TRY(launch_norms(v, N, R, bw.npart, bw.nblk, bw.res, st));
    MFS_HIP_TRY(hipMemcpyAsync(res_pin, bw.res, sizeof(double) * R, hipMemcpyDeviceToHost, st));
    MFS_HIP_TRY(hipStreamSynchronize(st));
    out.assign(res_pin, res_pin + R);
    return MFS_OK;
  };
  int n32 = 0, n64 = 0, n_refine = 0, n_restart = 0, total = 0;
  auto residual = [&]() -> mfs_status {  // r = b - A64 x, relres per column
    MFS_TRY(apply_f64(s, x, w, R, st));
    ++n64;
    MFS_HIP_TRY(launch_axpby(b, w, r, 1.0, -1.0, NR, st));
    std::vector<double> rn;
    MFS_TRY(read_norms(r, rn));
    for (int c = 0; c < R; ++c) relres[c] = bnorm[c] > 0.0 ? rn[c] / bnorm[c] : 0.0;
    return MFS_OK;
  };
  auto max_relres = [&]() {
    double mx = 0.0;
    for (double v : relres) mx = std::max(mx, v);
    return mx;
  };
  auto apply = [&](int j) -> mfs_status {  // bw.W = S G_hat V_j
    if (prec == MFS_MIXED) {
      if (v32) MFS_TRY(apply_mixed_from32(s, static_cast<const c64*>(bw.slot(j)), bw.W, R, st));
      else MFS_TRY(apply_mixed(s, static_cast<const c128*>(bw.slot(j)), bw.W, R, st, 0.0));
      ++n32;
    } else {
      MFS_TRY(apply_f64(s, static_cast<const c128*>(bw.slot(j)), bw.W, R, st, 0.0));
      ++n64;
    }
    return MFS_OK;
  };
  auto apply_vec = [&](const c128* v) -> mfs_status {  // bw.W = S G_hat v, v an N x R complex128 block
    if (prec == MFS_MIXED) {
      MFS_TRY(apply_mixed(s, v, bw.W, R, st, 0.0));
      ++n32;
    } else {
      MFS_TRY(apply_f64(s, v, bw.W, R, st, 0.0));
      ++n64;
    }
    return MFS_OK;
  };
  int n_second = 0;
  bw.n_second = &n_second;
  BlockProcess first{0, bw.Hp, bw.refl};
  KeptSpace kept{};
  BlockProcess later = first;

  // b = S vhat (eq. mbody2)
  MFS_HIP_TRY(launch_sapply_f64(s->dev, vhat, 1, nullptr, 0.0, b, R, (int)s->kmax, st));
  MFS_TRY(read_norms(b, bnorm));
  if (opts->use_x0) {
    MFS_TRY(residual());
  } else {
    MFS_HIP_TRY(hipMemsetAsync(x, 0, sizeof(c128) * NR, st));
    MFS_HIP_TRY(hipMemcpyAsync(r, b, sizeof(c128) * NR, hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < R; ++c) relres[c] = bnorm[c] > 0.0 ? 1.0 : 0.0;
  }
  const int max_cycles = prec == MFS_MIXED ? opts->max_refine : 1 << 30;
  while (max_relres() > opts->tol && n_refine < max_cycles && total < opts->maxit) {
    // reduction still needed by the worst column, relative to each column's current residual
    double ktol = opts->tol / std::max(max_relres(), 1e-300);
    if (prec == MFS_MIXED) ktol = std::min(std::max(opts->inner_tol, 0.3 * ktol), 0.5);
    const int mlim = std::min(m - (kept.k > 0 ? later.o : 0), opts->maxit - total);
    int steps = 0;
    double est = 0.0;
    const bool use_kept = kept.k > 0;
    MFS_TRY(block_cycle(bw, use_kept ? later : first, kept, r, x, ktol, mlim, apply, apply_vec, opts->verbose, &steps,
                        &est, st));
    // keep the first cycle's space for the correction cycles when there is room for 8 more blocks
    if (!use_kept && opts->deflate && prec == MFS_MIXED && n_refine == 0 && steps > 0 && steps + 1 + 8 <= m) {
      kept = KeptSpace{steps, bw.Hp, bw.refl};
      later = BlockProcess{steps + 1, bw.Hp + bw.hoff(steps), bw.refl + (int64_t)steps * R * (R + 1)};
    }
    total += steps;
    ++n_refine;
    ++n_restart;
    MFS_TRY(residual());
    if (opts->verbose)
      std::fprintf(stderr, "[mfs_solve block %s] cycle %d  block steps %d (total %d)  estimate %.3e  max relres %.3e\n",
                   prec == MFS_MIXED ? "mixed" : "fp64", n_refine, steps, total, est, max_relres());
    if (steps == 0) break;
  }
  MFS_HIP_TRY(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->n_reorth = n_second;  // block steps that took the second Gram-Schmidt pass
    info->n_matvec32 = n32;
    info->n_matvec64 = n64;
    info->n_refine = prec == MFS_MIXED ? n_refine : 0;
    info->n_restart = n_restart;
    info->relres_max = max_relres();
    info->t_total_s = std::chrono::duration<double>(t1 - t0).count();
  }
  if (max_relres() > opts->tol)
    return fail(MFS_ERR_NOCONV, "block solve: relative residual " + std::to_string(max_relres()) + " above tol after " +
                                    std::to_string(total) + " block steps");
  return MFS_OK;
}

}  // namespace

extern "C" {

const char* mfs_last_error(void) { return g_last_error.c_str(); }

int mfs_version(void) { return 100; }

mfs_status mfs_build_S(const mfs_shape_desc* desc, void* S64_dev, void* S32_dev, int64_t* k_out,
                       int64_t* skel_idx_out, double* diag_out, void* stream) {
  g_last_error.clear();
  return build_S_impl(desc, S64_dev, S32_dev, k_out, skel_idx_out, diag_out, as_stream(stream));
}

// Length of the padded layout the symmetric kernel gets (bodies padded to whole 64-point tiles), or
// 0 where none is made: only for bodies that are not all multiples of 64 (3D sub-blocks aside), and
// only while the padded pair count stays within 1.4 times the real one.
int64_t sym_pad_length(const SceneDev& d, const std::vector<int64_t>& body_ptr) {
  if (!sym_padded(d)) return 0;
  int64_t NP = 0;
  for (size_t t = 0; t + 1 < body_ptr.size(); ++t) NP += (body_ptr[t + 1] - body_ptr[t] + 63) / 64 * 64;
  const double N = (double)body_ptr.back();
  return (double)NP * (double)NP <= 1.4 * N * N && NP <= 0x7fffffff ? NP : 0;
}

mfs_status mfs_scene_create(int32_t dim, double kappa, int64_t T, const int32_t* shape_of, const double* centres,
                            const double* rotations, int32_t n_shapes, const int64_t* k_of_shape, const double* const* eq_template,
                            const void* const* S64_dev, const void* const* S32_dev, mfs_scene** out) {
  g_last_error.clear();
  if (!out) return fail(MFS_ERR_ARG, "out is null");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(MFS_ERR_ARG, "dim must be 2 or 3");
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(MFS_ERR_ARG, "kappa must be positive and finite");
  if (T < 1) return fail(MFS_ERR_ARG, "T must be >= 1");
  if (n_shapes < 1) return fail(MFS_ERR_ARG, "n_shapes must be >= 1");
  if (!shape_of || !centres || !k_of_shape || !eq_template || !S64_dev)
    return fail(MFS_ERR_ARG, "null table pointer");
  int64_t kmax = 0;
  for (int s = 0; s < n_shapes; ++s) {
    if (k_of_shape[s] < 1 || k_of_shape[s] > 4096)
      return fail(MFS_ERR_ARG, "k_of_shape[" + std::to_string(s) + "] must be in 1..4096");
    if (!eq_template[s] || !S64_dev[s]) return fail(MFS_ERR_ARG, "null template or S for shape " + std::to_string(s));
    if (S32_dev && !S32_dev[s]) return fail(MFS_ERR_ARG, "null S32 for shape " + std::to_string(s));
    kmax = std::max(kmax, k_of_shape[s]);
  }
  std::vector<int64_t> body_ptr(T + 1, 0);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t t = 0; t < T; ++t) {
    const int s = shape_of[t];
    if (s < 0 || s >= n_shapes) return fail(MFS_ERR_ARG, "shape_of[" + std::to_string(t) + "] out of range");
    body_ptr[t + 1] = body_ptr[t] + k_of_shape[s];
    if (rotations) {
      // a proper orthogonal matrix: R R^T = I to rounding, det > 0
      const double* Rt = rotations + t * dim * dim;
      double worst = 0.0;
      for (int a = 0; a < dim; ++a)
        for (int b2 = 0; b2 < dim; ++b2) {
          double dot = 0.0;
          for (int e = 0; e < dim; ++e) dot += Rt[a * dim + e] * Rt[b2 * dim + e];
          worst = std::max(worst, std::fabs(dot - (a == b2 ? 1.0 : 0.0)));
        }
      const double det = dim == 2 ? Rt[0] * Rt[3] - Rt[1] * Rt[2]
                                  : Rt[0] * (Rt[4] * Rt[8] - Rt[5] * Rt[7]) - Rt[1] * (Rt[3] * Rt[8] - Rt[5] * Rt[6]) +
                                        Rt[2] * (Rt[3] * Rt[7] - Rt[4] * Rt[6]);
      if (!(worst < 1e-10) || !(det > 0.0))
        return fail(MFS_ERR_ARG, "rotations[" + std::to_string(t) + "] is not a proper rotation");
    }
    for (int d = 0; d < dim; ++d) {
      const double c = centres[t * dim + d];
      if (!std::isfinite(c)) return fail(MFS_ERR_ARG, "non-finite centre");
      lo[d] = std::min(lo[d], c);
      hi[d] = std::max(hi[d], c);
    }
  }
  const int64_t N = body_ptr[T];
  if (N > 0x7fffffff) return fail(MFS_ERR_ARG, "N exceeds 2^31-1");
  double same_body_pairs = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    const double kt = (double)(body_ptr[t + 1] - body_ptr[t]);
    same_body_pairs += kt * kt;
  }
  std::vector<int64_t> tmpl_ptr(n_shapes + 1, 0);
  for (int s = 0; s < n_shapes; ++s) tmpl_ptr[s + 1] = tmpl_ptr[s] + k_of_shape[s];
  std::vector<double> tmpl(tmpl_ptr[n_shapes] * dim);
  for (int s = 0; s < n_shapes; ++s)
    std::memcpy(&tmpl[tmpl_ptr[s] * dim], eq_template[s], sizeof(double) * k_of_shape[s] * dim);
  double origin[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; ++d) origin[d] = 0.5 * (lo[d] + hi[d]);

  int device = 0;
  {
    const hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail(MFS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    void* scr = nullptr;
    MFS_TRY(scratch_address(device, &scr));  // once per device: mfs_apply_static then only reads the table
  }
  mfs_scene* sc = new mfs_scene();
  sc->device = device;
  sc->n_shapes = n_shapes;
  sc->kmax = kmax;
  sc->has_s32 = S32_dev != nullptr;
  sc->k_of_shape.assign(k_of_shape, k_of_shape + n_shapes);
  auto cleanup = [&](mfs_status st) {
    mfs_scene_destroy(sc);
    return st;
  };
  // Packing runs on the calling thread's private non-blocking stream, so creating a scene neither
  // waits for nor delays requests running on other streams.
  hipError_t pe = hipSuccess;
  hipStream_t ps = private_stream(&pe);
  if (pe != hipSuccess) return cleanup(fail(MFS_ERR_HIP, std::string("stream creation: ") + hipGetErrorString(pe)));
  sc->last_stream = ps;
  Buf tmpl_d, tmpl_ptr_d;
  size_t tmp_bytes = 0;
  mfs_status st;
  if ((st = ensure(sc->x64, sizeof(double) * dim * N, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->x32, sizeof(float) * dim * N, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->l32, sizeof(float) * dim * N, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->lsq, sizeof(float) * N, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->centres, sizeof(double) * dim * T, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->body_of, sizeof(int32_t) * N, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->body_ptr, sizeof(int64_t) * (T + 1), &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->shape_of, sizeof(int32_t) * T, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->k_dev, sizeof(int64_t) * n_shapes, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->S64_tab, sizeof(void*) * n_shapes, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(sc->S32_tab, sizeof(void*) * n_shapes, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
  if (rotations && (st = ensure(sc->rot, sizeof(double) * T * dim * dim, &sc->bytes, ps)) != MFS_OK)
    return cleanup(st);
  if ((st = ensure(tmpl_d, sizeof(double) * tmpl.size(), &tmp_bytes, ps)) != MFS_OK) return cleanup(st);
  if ((st = ensure(tmpl_ptr_d, sizeof(int64_t) * tmpl_ptr.size(), &tmp_bytes, ps)) != MFS_OK) return cleanup(st);

  std::vector<const void*> s32v(n_shapes, nullptr);
  if (S32_dev)
    for (int s = 0; s < n_shapes; ++s) s32v[s] = S32_dev[s];
  hipError_t e = hipSuccess;
  auto cp = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, ps);
  };
  cp(sc->body_ptr.p, body_ptr.data(), sizeof(int64_t) * (T + 1));
  cp(sc->shape_of.p, shape_of, sizeof(int32_t) * T);
  cp(sc->k_dev.p, k_of_shape, sizeof(int64_t) * n_shapes);
  cp(sc->S64_tab.p, S64_dev, sizeof(void*) * n_shapes);
  cp(sc->S32_tab.p, s32v.data(), sizeof(void*) * n_shapes);
  cp(sc->centres.p, centres, sizeof(double) * T * dim);
  if (rotations) cp(sc->rot.p, rotations, sizeof(double) * T * dim * dim);
  cp(tmpl_d.p, tmpl.data(), sizeof(double) * tmpl.size());
  cp(tmpl_ptr_d.p, tmpl_ptr.data(), sizeof(int64_t) * tmpl_ptr.size());
  if (e == hipSuccess)
    e = launch_pack_scene(dim, T, static_cast<int32_t*>(sc->shape_of.p), static_cast<double*>(sc->centres.p),
                          rotations ? static_cast<double*>(sc->rot.p) : nullptr, static_cast<int64_t*>(tmpl_ptr_d.p), static_cast<double*>(tmpl_d.p),
                          static_cast<int64_t*>(sc->body_ptr.p), origin, static_cast<double*>(sc->x64.p),
                          static_cast<float*>(sc->x32.p), static_cast<float*>(sc->l32.p),
                          static_cast<float*>(sc->lsq.p), static_cast<int32_t*>(sc->body_of.p), N, ps);
  if (e == hipSuccess) e = hipStreamSynchronize(ps);
  release(tmpl_d, &tmp_bytes, ps);
  release(tmpl_ptr_d, &tmp_bytes, ps);
  if (e != hipSuccess) return cleanup(fail(MFS_ERR_HIP, std::string("scene packing: ") + hipGetErrorString(e)));

  SceneDev& d = sc->dev;
  d.dim = dim;
  d.N = N;
  d.T = T;
  d.kappa = kappa;
  for (int i = 0; i < 3; ++i) {
    d.origin[i] = origin[i];
    d.x64[i] = i < dim ? static_cast<double*>(sc->x64.p) + (size_t)i * N : nullptr;
    d.x32[i] = i < dim ? static_cast<float*>(sc->x32.p) + (size_t)i * N : nullptr;
    d.l32[i] = i < dim ? static_cast<float*>(sc->l32.p) + (size_t)i * N : nullptr;
  }
  d.centres = static_cast<double*>(sc->centres.p);
  d.rot = rotations ? static_cast<double*>(sc->rot.p) : nullptr;
  d.lsq32 = static_cast<float*>(sc->lsq.p);
  d.body_of = static_cast<int32_t*>(sc->body_of.p);
  d.body_ptr = static_cast<int64_t*>(sc->body_ptr.p);
  d.shape_of = static_cast<int32_t*>(sc->shape_of.p);
  d.k_of_shape = static_cast<int64_t*>(sc->k_dev.p);
  d.S64 = static_cast<const void* const*>(sc->S64_tab.p);
  d.S32 = static_cast<const void* const*>(sc->S32_tab.p);
  d.offbody_pairs = (double)N * (double)N - same_body_pairs;
  d.rho_max = 0.0;
  for (size_t i = 0; i < tmpl.size() / dim; ++i) {
    double r2 = 0.0;
    for (int dd = 0; dd < dim; ++dd) r2 += tmpl[i * dim + dd] * tmpl[i * dim + dd];
    d.rho_max = std::max(d.rho_max, std::sqrt(r2));
  }
  d.all_k_mult16 = d.all_k_mult64 = true;
  for (int s2 = 0; s2 < n_shapes; ++s2) {
    d.all_k_mult16 = d.all_k_mult16 && (k_of_shape[s2] % 16 == 0);
    d.all_k_mult64 = d.all_k_mult64 && (k_of_shape[s2] % 64 == 0);
  }
  d.sym16 = dim == 3 && d.all_k_mult16 && !d.all_k_mult64;
  d.phi16_shift = sc->phi16_shift_auto = phi16_shift_for(dim, T, centres, d.rho_max);
  d.Npad = N;
  d.pad_ptr = nullptr;
  d.body_of_pad = nullptr;
  d.lsqp = nullptr;
  for (int i = 0; i < 3; ++i) d.l32p[i] = nullptr;
  if (sym_pad_length(d, body_ptr) > 0) {
    // bodies padded to whole 64-point tiles, made only where the symmetric kernel would pay
    std::vector<int64_t> pad_ptr(T + 1, 0);
    for (int64_t t = 0; t < T; ++t) pad_ptr[t + 1] = pad_ptr[t] + (body_ptr[t + 1] - body_ptr[t] + 63) / 64 * 64;
    const int64_t NP = pad_ptr[T];
    {
      std::vector<int32_t> body_of_pad(NP);
      for (int64_t t = 0; t < T; ++t)
        for (int64_t i = pad_ptr[t]; i < pad_ptr[t + 1]; ++i) body_of_pad[i] = (int32_t)t;
      if ((st = ensure(sc->pad_ptr, sizeof(int64_t) * (T + 1), &sc->bytes, ps)) != MFS_OK) return cleanup(st);
      if ((st = ensure(sc->body_of_pad, sizeof(int32_t) * NP, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
      if ((st = ensure(sc->l32p, sizeof(float) * dim * NP, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
      if ((st = ensure(sc->lsqp, sizeof(float) * NP, &sc->bytes, ps)) != MFS_OK) return cleanup(st);
      d.Npad = NP;
      d.pad_ptr = static_cast<int64_t*>(sc->pad_ptr.p);
      d.body_of_pad = static_cast<int32_t*>(sc->body_of_pad.p);
      d.lsqp = static_cast<float*>(sc->lsqp.p);
      for (int i = 0; i < dim; ++i) d.l32p[i] = static_cast<float*>(sc->l32p.p) + (size_t)i * NP;
      cp(sc->pad_ptr.p, pad_ptr.data(), sizeof(int64_t) * (T + 1));
      cp(sc->body_of_pad.p, body_of_pad.data(), sizeof(int32_t) * NP);
      if (e == hipSuccess) e = launch_pad_scene(d, static_cast<float*>(sc->l32p.p), static_cast<float*>(sc->lsqp.p), ps);
      if (e == hipSuccess) e = hipStreamSynchronize(ps);  // the host tables are released on return
      if (e != hipSuccess) return cleanup(fail(MFS_ERR_HIP, std::string("scene padding: ") + hipGetErrorString(e)));
    }
  }
  *out = sc;
  return MFS_OK;
}

mfs_status mfs_scene_destroy(mfs_scene* s) {
  if (!s) return MFS_OK;
  Buf* all[] = {&s->x64,     &s->x32,     &s->l32,      &s->lsq,     &s->centres,    &s->body_of,
                &s->body_ptr, &s->shape_of, &s->k_dev,   &s->S64_tab, &s->S32_tab,    &s->rot,
                &s->partial,  &s->q32,      &s->dirs,    &s->kry,     &s->vecs,       &s->near_tab,
                &s->pad_ptr,  &s->body_of_pad, &s->l32p, &s->lsqp,    &s->qpad,       &s->qsplit};
  for (Buf* b : all) release(*b, &s->bytes, s->last_stream);
  delete s;
  return MFS_OK;
}

mfs_status mfs_scene_size(const mfs_scene* s, int64_t* N_out, int64_t* T_out, size_t* bytes_out) {
  MFS_TRY(check_scene(s));
  if (N_out) *N_out = s->dev.N;
  if (T_out) *T_out = s->dev.T;
  if (bytes_out) *bytes_out = s->bytes;
  return MFS_OK;
}

mfs_status mfs_solve_footprint(int32_t dim, int64_t T, const int32_t* shape_of, int32_t n_shapes,
                               const int64_t* k_of_shape, int32_t rotations, int32_t R, const mfs_solve_opts* opts,
                               int64_t n_targets, size_t* bytes_out) {
  g_last_error.clear();
  if (!bytes_out) return fail(MFS_ERR_ARG, "solve_footprint: bytes_out is null");
  *bytes_out = 0;
  if (dim != 2 && dim != 3) return fail(MFS_ERR_ARG, "solve_footprint: dim must be 2 or 3");
  if (T < 1 || n_shapes < 1 || !shape_of || !k_of_shape || !opts)
    return fail(MFS_ERR_ARG, "solve_footprint: T, n_shapes >= 1 and non-null tables and options required");
  if (R < 1 || opts->restart < 1 || n_targets < 0)
    return fail(MFS_ERR_ARG, "solve_footprint: R >= 1, restart >= 1 and n_targets >= 0 required");
  if (opts->block && (R < 2 || R > 64)) return fail(MFS_ERR_ARG, "solve_footprint: block GMRES takes 2..64 right-hand sides");
  int64_t kmax = 0;
  for (int s = 0; s < n_shapes; ++s) {
    if (k_of_shape[s] < 1 || k_of_shape[s] > 4096) return fail(MFS_ERR_ARG, "solve_footprint: k_of_shape out of range");
    kmax = std::max(kmax, k_of_shape[s]);
  }
  std::vector<int64_t> body_ptr(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    if (shape_of[t] < 0 || shape_of[t] >= n_shapes) return fail(MFS_ERR_ARG, "solve_footprint: shape_of out of range");
    body_ptr[t + 1] = body_ptr[t] + k_of_shape[shape_of[t]];
  }
  const int64_t N = body_ptr[T];
  if (N > 0x7fffffff) return fail(MFS_ERR_ARG, "solve_footprint: N exceeds 2^31-1");
  // a scene with the layout and flags mfs_scene_create would give (no device memory): the launch
  // shapes and workspace sizes below come from the same functions a solve uses
  mfs_scene sh;
  SceneDev& d = sh.dev;
  d.dim = dim;
  d.N = N;
  d.T = T;
  d.all_k_mult16 = d.all_k_mult64 = true;
  for (int s = 0; s < n_shapes; ++s) {
    d.all_k_mult16 = d.all_k_mult16 && k_of_shape[s] % 16 == 0;
    d.all_k_mult64 = d.all_k_mult64 && k_of_shape[s] % 64 == 0;
  }
  d.sym16 = dim == 3 && d.all_k_mult16 && !d.all_k_mult64;
  const int64_t NP = sym_pad_length(d, body_ptr);
  static const int64_t kNonNull = 0;
  d.Npad = NP > 0 ? NP : N;
  d.pad_ptr = NP > 0 ? &kNonNull : nullptr;
  d.phi16_shift = 0;  // the split charges are counted wherever the matrix cores may run (a bound)
  sh.kmax = kmax;
  auto blk = [](size_t b) { return b ? pool_block_size(b) : 0; };
  size_t total = 0;
  // scene tables (mfs_scene_create)
  total += blk(sizeof(double) * dim * N) + 2 * blk(sizeof(float) * dim * N) + blk(sizeof(float) * N) +
           blk(sizeof(double) * dim * T) + blk(sizeof(int32_t) * N) + blk(sizeof(int64_t) * (T + 1)) +
           blk(sizeof(int32_t) * T) + blk(sizeof(int64_t) * n_shapes) + 2 * blk(sizeof(void*) * n_shapes);
  if (rotations) total += blk(sizeof(double) * T * dim * dim);
  if (NP > 0)
    total += blk(sizeof(int64_t) * (T + 1)) + blk(sizeof(int32_t) * NP) + blk(sizeof(float) * dim * NP) +
             blk(sizeof(float) * NP);
  // pair partial sums (one grow-only buffer: the largest of the FP32 sum, the FP64 residual and the
  // FP64 field evaluation), padded charges, split charges, FP32 charges
  const mfs_prec prec = opts->prec;
  size_t part = 0, qpad = 0, split = 0, q32 = 0;
  if (prec != MFS_FP64) {
    const LaunchShape ls = shape_for(&sh, false, R);
    part = (size_t)f32_slices(&sh, ls, R) * R * f32_rows(&sh, ls) * sizeof(c64);
    if (ls.sym == 1 && NP > 0) qpad = (size_t)R * NP * sizeof(c64);
    if (ls.sym != 1 && ghat_uses_mfma16(d, R)) split = ghat_split_bytes(d, R);
    if (dim == 3 && ls.sym != 1 && R <= kSymDefaultMaxRhs && ghat_sym_possible(d, R)) {
      // in 3D the split-FP16 kernel's bound on |phi| comes from the centres, which the footprint
      // does not see: where it fails the symmetric kernel runs, so count its slices too (a bound)
      LaunchShape lsym = ls;
      lsym.sym = 1;
      const int64_t NS = sym_view(d).N;
      lsym.nchunks = sym_plan(NS, 0, sym_block_waves(NS, R)).nchunks_d;
      part = std::max(part, (size_t)f32_slices(&sh, lsym, R) * R * f32_rows(&sh, lsym) * sizeof(c64));
      if (NP > 0) qpad = (size_t)R * NP * sizeof(c64);
    }
    q32 = (size_t)R * N * sizeof(c64);
  }
  part = std::max(part, (size_t)ghat_f64_slices(d, R, shape_for(&sh, true, R).nchunks) * R * N * sizeof(c128));
  if (n_targets > 0)
    part = std::max(part, (size_t)pair_chunks_for(N, n_targets, tpt_for(MFS_FP64)) * R * n_targets * sizeof(c128));
  total += blk(part) + blk(qpad) + blk(split) + blk(q32) + blk(sizeof(double) * R * dim);
  // Krylov workspace and solver vectors
  const bool v32 = prec == MFS_MIXED && opts->basis32 != 0 && !(opts->fp64_until > 0.0);
  const size_t kry = opts->block ? block_work_bytes(N, R, opts->restart, prec == MFS_MIXED && opts->basis32 != 0, nullptr)
                                 : column_work_layout(N, R, opts->restart, v32).total;
  total += blk(kry) + blk(3 * sizeof(c128) * (size_t)N * R + 256);
  *bytes_out = total;
  return MFS_OK;
}

mfs_status mfs_scene_points(const mfs_scene* s, double* xhat_host) {
  MFS_TRY(check_scene(s));
  if (!xhat_host) return fail(MFS_ERR_ARG, "xhat_host is null");
  const int dim = s->dev.dim;
  const int64_t N = s->dev.N;
  std::vector<double> soa((size_t)dim * N);
  MFS_HIP_TRY(hipMemcpy(soa.data(), s->x64.p, sizeof(double) * soa.size(), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < N; ++i)
    for (int d = 0; d < dim; ++d) xhat_host[i * dim + d] = soa[(size_t)d * N + i];
  return MFS_OK;
}

mfs_status mfs_plane_wave(const mfs_scene* sc, const double* dirs_host, int32_t R, void* vhat_dev, void* stream) {
  MFS_TRY(check_scene(sc));
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  if (R < 1 || !dirs_host || !vhat_dev) return fail(MFS_ERR_ARG, "plane wave: bad R or null pointer");
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  MFS_TRY(ensure(s->dirs, sizeof(double) * R * s->dev.dim, &s->bytes, st));
  MFS_HIP_TRY(hipMemcpyAsync(s->dirs.p, dirs_host, sizeof(double) * R * s->dev.dim, hipMemcpyHostToDevice, st));
  MFS_HIP_TRY(hipStreamSynchronize(st));  // dirs_host may be released by the caller on return
  MFS_HIP_TRY(launch_plane_wave(s->dev, static_cast<double*>(s->dirs.p), R, static_cast<c128*>(vhat_dev), st));
  return MFS_OK;
}

mfs_status mfs_ghat_apply(const mfs_scene* sc, const void* q_dev, void* t_dev, int32_t R, mfs_prec prec,
                          void* stream) {
  MFS_TRY(check_scene(sc));
  MFS_TRY(check_prec_operator(sc, prec == MFS_FP32 ? MFS_FP64 : prec));
  if (R < 1 || !q_dev || !t_dev || q_dev == t_dev) return fail(MFS_ERR_ARG, "ghat: bad R or pointers");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  if (prec == MFS_FP64) {
    const int nch = ghat_f64_slices(s->dev, R, shape_for(s, true, R).nchunks);
    MFS_TRY(ensure(s->partial, (size_t)nch * R * s->dev.N * sizeof(c128), &s->bytes, st));
    c128* part = static_cast<c128*>(s->partial.p);
    {
      TimedLaunch tl(MFS_KERNEL_PAIR_F64, s->dev.offbody_pairs * R, st);
      MFS_HIP_TRY(launch_ghat_f64(s->dev, static_cast<const c128*>(q_dev), R, part, nch, st));
    }
    MFS_HIP_TRY(launch_reduce_partials_f64(part, nch, s->dev.N, R, static_cast<c128*>(t_dev), st));
  } else {
    PartialF32 p;
    MFS_TRY(pair_f32(s, static_cast<const c64*>(q_dev), R, st, &p));
    if (p.pptr) MFS_HIP_TRY(launch_reduce_partials_padded(s->dev, p.part, p.slices, R, static_cast<c64*>(t_dev), st));
    else MFS_HIP_TRY(launch_reduce_partials_f32(p.part, p.slices, s->dev.N, R, static_cast<c64*>(t_dev), st));
  }
  return MFS_OK;
}

mfs_status mfs_s_apply(const mfs_scene* sc, const void* q_dev, const void* t_dev, void* y_dev, double beta,
                       int32_t R, mfs_prec prec, void* stream) {
  MFS_TRY(check_scene(sc));
  MFS_TRY(check_prec_operator(sc, prec));
  if (R < 1 || !t_dev || !y_dev || (beta != 0.0 && !q_dev)) return fail(MFS_ERR_ARG, "s_apply: bad R or pointers");
  if (t_dev == y_dev) return fail(MFS_ERR_ARG, "s_apply: y must not alias t");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  if (prec == MFS_FP64) {
    MFS_HIP_TRY(launch_sapply_f64(s->dev, static_cast<const c128*>(t_dev), 1, static_cast<const c128*>(q_dev), beta,
                                  static_cast<c128*>(y_dev), R, (int)s->kmax, st));
  } else {
    MFS_HIP_TRY(launch_sapply_f32(s->dev, static_cast<const c64*>(t_dev), 1, static_cast<const c64*>(q_dev),
                                  (float)beta, static_cast<c64*>(y_dev), R, (int)s->kmax, st));
  }
  return MFS_OK;
}

mfs_status mfs_apply(const mfs_scene* sc, const void* q_dev, void* y_dev, int32_t R, mfs_prec prec, void* stream) {
  MFS_TRY(check_scene(sc));
  MFS_TRY(check_prec_operator(sc, prec));
  if (R < 1 || !q_dev || !y_dev || q_dev == y_dev) return fail(MFS_ERR_ARG, "apply: bad R or pointers");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  if (prec == MFS_FP64) return apply_f64(s, static_cast<const c128*>(q_dev), static_cast<c128*>(y_dev), R, st);
  return apply_f32(s, static_cast<const c64*>(q_dev), static_cast<c64*>(y_dev), R, st);
}

mfs_status mfs_apply_static(const mfs_scene* sc, const void* q_dev, void* y_dev, int32_t R, mfs_prec prec,
                            void* stream) {
  MFS_TRY(check_scene(sc));
  MFS_TRY(check_prec_operator(sc, prec));
  if (R < 1 || !q_dev || !y_dev || q_dev == y_dev) return fail(MFS_ERR_ARG, "apply_static: bad R or pointers");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  void* buf = nullptr;
  {
    // the address was taken when the scene was created; this only reads the table
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    buf = (s->device >= 0 && s->device < kMaxDevices) ? g_scratch_addr[s->device] : nullptr;
  }
  if (!buf) return fail(MFS_ERR_ARG, "apply_static: no static scratch address for the scene's device");
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  return apply_in_buffer(s, q_dev, y_dev, R, prec, buf, (size_t)MFS_STATIC_SCRATCH_BYTES, st);
}

mfs_status mfs_eval_field(const mfs_scene* sc, const void* qhat_dev, int32_t R, const double* targets_dev, int64_t M,
                          void* u_dev, mfs_prec prec, void* stream) {
  MFS_TRY(check_scene(sc));
  MFS_TRY(check_prec_operator(sc, prec == MFS_FP32 ? MFS_FP64 : prec));
  if (R < 1 || M < 0 || !qhat_dev || !u_dev || (M > 0 && !targets_dev))
    return fail(MFS_ERR_ARG, "eval_field: bad sizes or pointers");
  if (M == 0) return MFS_OK;
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  const int nch = pair_chunks_for(s->dev.N, M, tpt_for(prec));
  if (prec == MFS_FP64) {
    MFS_TRY(ensure(s->partial, (size_t)nch * R * M * sizeof(c128), &s->bytes, st));
    c128* part = static_cast<c128*>(s->partial.p);
    {
      TimedLaunch tl(MFS_KERNEL_PAIR_F64, (double)M * s->dev.N * R, st);
      MFS_HIP_TRY(launch_eval_f64(s->dev, static_cast<const c128*>(qhat_dev), R, targets_dev, M, part, nch, st));
    }
    MFS_HIP_TRY(launch_reduce_partials_f64(part, nch, M, R, static_cast<c128*>(u_dev), st));
  } else {
    MFS_TRY(ensure(s->partial, (size_t)nch * R * M * sizeof(c64), &s->bytes, st));
    c64* part = static_cast<c64*>(s->partial.p);
    {
      TimedLaunch tl(MFS_KERNEL_PAIR_F32, (double)M * s->dev.N * R, st);
      MFS_HIP_TRY(launch_eval_f32(s->dev, static_cast<const c64*>(qhat_dev), R, targets_dev, M, part, nch, st));
    }
    MFS_HIP_TRY(launch_reduce_partials_f32(part, nch, M, R, static_cast<c64*>(u_dev), st));
  }
  return MFS_OK;
}

// ------------------------------------------------------------------- solve ---
mfs_status mfs_solve(const mfs_scene* sc, const void* vhat_dev, int32_t R, const mfs_solve_opts* opts,
                     void* qhat_dev, mfs_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  MFS_TRY(check_scene(sc));
  if (!opts || !vhat_dev || !qhat_dev || R < 1) return fail(MFS_ERR_ARG, "solve: null pointer or R < 1");
  const mfs_prec prec = opts->prec;
  if (prec != MFS_FP64 && prec != MFS_MIXED) return fail(MFS_ERR_ARG, "solve: prec must be MFS_FP64 or MFS_MIXED");
  if (prec == MFS_MIXED && !sc->has_s32) return fail(MFS_ERR_ARG, "solve: MFS_MIXED needs FP32 copies of S");
  if (!(opts->tol > 0.0) || opts->maxit < 1 || opts->restart < 1 || opts->restart > 32768)
    return fail(MFS_ERR_ARG, "solve: need tol > 0, maxit >= 1, 1 <= restart <= 32768");
  if (prec == MFS_MIXED && (opts->max_refine < 1 || !(opts->inner_tol > 0.0) || !(opts->inner_tol < 1.0)))
    return fail(MFS_ERR_ARG, "solve: MFS_MIXED needs max_refine >= 1 and 0 < inner_tol < 1");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  if (opts->block != 0 && R > 1) {
    if (opts->fp64_until > 0.0 || opts->use_graph)
      return fail(MFS_ERR_ARG, "solve: block GMRES does not take fp64_until or use_graph");
    return solve_block(s, static_cast<const c128*>(vhat_dev), R, opts, static_cast<c128*>(qhat_dev), info, st, t0);
  }
  const int64_t N = s->dev.N;
  const int64_t NR = N * R;
  const int m = opts->restart;

  // ---- Krylov state and vectors in two grow-only scene workspaces
  KrylovDev k{};
  k.N = N;
  k.R = R;
  k.m = m;
  k.nblk = krylov_nblk(N);
  // single-precision basis: inner solves that use the FP32 operator throughout
  const bool v32 = prec == MFS_MIXED && opts->basis32 != 0 && !(opts->fp64_until > 0.0);
  const ColumnWork L = column_work_layout(N, R, m, v32);
  const size_t oV = L.V, oH = L.H, ocs = L.cs, osn = L.sn, og = L.g, oh1 = L.h1, oh2 = L.h2, oy = L.y,
               obeta = L.beta, obn = L.bn, ores = L.res, ohn = L.hn, oact = L.act, ojl = L.jl, own = L.wn,
               oro = L.ro, onro = L.nro, opart = L.part, ojdev = L.jdev, otol = L.tol, oq = L.q, ocr = L.cr,
               oee = L.ee, ojold = L.jold, orn2 = L.rn2, okeep = L.keep;
  MFS_TRY(ensure(s->kry, L.total, &s->bytes, st));
  char* base = static_cast<char*>(s->kry.p);
  k.V = base + oV;
  k.v32 = v32;
  k.H = reinterpret_cast<c128*>(base + oH);
  k.cs = reinterpret_cast<c128*>(base + ocs);
  k.sn = reinterpret_cast<c128*>(base + osn);
  k.g = reinterpret_cast<c128*>(base + og);
  k.hcol = reinterpret_cast<c128*>(base + oh1);
  k.h2 = reinterpret_cast<c128*>(base + oh2);
  k.y = reinterpret_cast<c128*>(base + oy);
  k.beta = reinterpret_cast<double*>(base + obeta);
  k.bnorm = reinterpret_cast<double*>(base + obn);
  k.res = reinterpret_cast<double*>(base + ores);
  k.hnorm = reinterpret_cast<double*>(base + ohn);
  k.active = reinterpret_cast<int32_t*>(base + oact);
  k.jlen = reinterpret_cast<int32_t*>(base + ojl);
  k.part = reinterpret_cast<double*>(base + opart);
  k.wn = reinterpret_cast<double*>(base + own);
  k.reorth = reinterpret_cast<int32_t*>(base + oro);
  k.n_reorth = reinterpret_cast<int32_t*>(base + onro);
  const bool use_graph = opts->use_graph != 0;
  k.jdev = use_graph ? reinterpret_cast<int32_t*>(base + ojdev) : nullptr;
  k.tol_dev = use_graph ? reinterpret_cast<double*>(base + otol) : nullptr;
  c128* qdef = reinterpret_cast<c128*>(base + oq);      // deflation: q = G^H e_kold
  c128* cdef = reinterpret_cast<c128*>(base + ocr);     // V_old^H r of the correction's residual
  c128* edef = reinterpret_cast<c128*>(base + oee);     // coefficient work vector
  int32_t* jold = reinterpret_cast<int32_t*>(base + ojold);
  double* rn2 = reinterpret_cast<double*>(base + orn2);
  int32_t* keepdev = reinterpret_cast<int32_t*>(base + okeep);  // columns a correction solve works on
  MFS_HIP_TRY(hipMemsetAsync(k.n_reorth, 0, sizeof(int32_t) * R, st));
  // Second Gram-Schmidt pass when ||w'|| < 0.1 ||w||.  Measured: on 1000 starfish the median ratio
  // is 0.26 and eta = 0.2 takes the second pass on 26% of steps (93% for eta = 1/sqrt(2)); on 2000
  // starfish eta = 0.2 takes it on 34% and eta = 0.1 on none, each with the same iteration count and
  // final FP64 residual.  The refinement checks the true residual, so this trades no accuracy.
  k.reorth_eta = 0.1;
  k.ratio_log = opts->verbose > 2 ? reinterpret_cast<double*>(k.y) : nullptr;

  MFS_TRY(ensure(s->vecs, 3 * sizeof(c128) * (size_t)NR + 256, &s->bytes, st));
  c128* b = static_cast<c128*>(s->vecs.p);
  c128* r = b + NR;
  c128* w = r + NR;
  c128* x = static_cast<c128*>(qhat_dev);
  double* bnorm_dev = k.bnorm;

  std::vector<double> bnorm(R), rnorm(R), relres(R, 1.0);
  std::vector<int32_t> active(R);

  int n64 = 0, n32 = 0, n_refine = 0, n_restart = 0, total_it = 0;

  auto read_doubles = [&](const double* dev, std::vector<double>& host) -> mfs_status {
    MFS_HIP_TRY(hipMemcpyAsync(host.data(), dev, sizeof(double) * R, hipMemcpyDeviceToHost, st));
    MFS_HIP_TRY(hipStreamSynchronize(st));
    return MFS_OK;
  };
  auto residual = [&]() -> mfs_status {  // r = b - A64 x, relres per column
    MFS_TRY(apply_f64(s, x, w, R, st));
    ++n64;
    MFS_HIP_TRY(launch_axpby(b, w, r, 1.0, -1.0, NR, st));
    MFS_HIP_TRY(launch_norms(r, N, R, k.part, k.nblk, k.hnorm, st));
    MFS_TRY(read_doubles(k.hnorm, rnorm));
    for (int c = 0; c < R; ++c) relres[c] = bnorm[c] > 0.0 ? rnorm[c] / bnorm[c] : 0.0;
    return MFS_OK;
  };
  auto max_relres = [&]() {
    double mx = 0.0;
    for (double v : relres) mx = std::max(mx, v);
    return mx;
  };
  auto set_active_from_relres = [&]() -> mfs_status {
    for (int c = 0; c < R; ++c) active[c] = relres[c] > opts->tol ? 1 : 0;
    MFS_HIP_TRY(hipMemcpyAsync(k.active, active.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, st));
    return MFS_OK;
  };
  // Convergence flags and estimates come back through pinned slots with a lag: the host enqueues
  // step j while the device still runs the steps before it, and reads the flags of step j - lag,
  // so small systems are not bound by one host round trip per step.  Close to the target (estimate
  // within 16x of the tolerance) it reads every step.  Steps enqueued past convergence leave the
  // solution unchanged: converged columns are frozen by the Givens kernel (jlen stops growing).
  constexpr int kSlots = 3;
  size_t pin_bytes = 0;
  hipError_t pin_err = hipSuccess;
  char* pin = static_cast<char*>(pinned_alloc((size_t)kSlots * R * (sizeof(int32_t) + sizeof(double)), &pin_bytes,
                                              &pin_err));
  if (!pin) return fail(MFS_ERR_NOMEM, std::string("pinned host allocation failed: ") + hipGetErrorString(pin_err));
  struct PinGuard {
    void* p;
    size_t n;
    hipEvent_t ev[kSlots];
    ~PinGuard() {
      for (hipEvent_t e : ev)
        if (e) {
          (void)hipEventSynchronize(e);
          (void)hipEventDestroy(e);
        }
      pinned_free(p, n);
    }
  } guard{pin, pin_bytes, {nullptr, nullptr, nullptr}};
  for (int i = 0; i < kSlots; ++i)
    MFS_HIP_TRY(hipEventCreateWithFlags(&guard.ev[i], hipEventDisableTiming));
  int32_t* pin_act = reinterpret_cast<int32_t*>(pin);
  double* pin_res = reinterpret_cast<double*>(pin + ((sizeof(int32_t) * kSlots * R + 7) & ~size_t(7)));

  // Graph replay of the Krylov part of a step.  Graph b holds the launches of one step sized for
  // the largest step of bucket b; it is captured on first use (on this thread's private stream, in
  // thread-local capture mode) and replayed on st for every step of the bucket in every cycle of
  // this call.  What a replay bakes in is fixed for the call: workspace addresses, R, N and the
  // norm the estimate refers to (prec is fixed per call); the step index and tolerance are read
  // from device memory.
  struct GraphSet {
    std::vector<hipGraphExec_t> exec;
    ~GraphSet() {
      for (hipGraphExec_t e : exec)
        if (e) (void)hipGraphExecDestroy(e);
    }
  } graphs;
  if (use_graph) graphs.exec.assign((m + kStepBucket - 1) / kStepBucket, nullptr);
  auto krylov_step = [&](const KrylovDev& kk, int j, double ktol) -> mfs_status {
    if (!use_graph || !kk.jdev) {
      MFS_HIP_TRY(launch_arnoldi_orth(kk, j, w, st));
      MFS_HIP_TRY(launch_arnoldi_finish(kk, j, w, ktol, st));
      return MFS_OK;
    }
    hipGraphExec_t& ex = graphs.exec[j / kStepBucket];
    if (!ex) {
      hipError_t e = hipSuccess;
      hipStream_t cs = private_stream(&e);
      if (e != hipSuccess) return fail(MFS_ERR_HIP, std::string("stream creation: ") + hipGetErrorString(e));
      MFS_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipError_t e1 = launch_arnoldi_orth(kk, j, w, cs);
      hipError_t e2 = e1 == hipSuccess ? launch_arnoldi_finish(kk, j, w, ktol, cs) : e1;
      hipGraph_t g = nullptr;
      hipError_t e3 = hipStreamEndCapture(cs, &g);  // always leave capture mode
      if (e2 != hipSuccess || e3 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(MFS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e2 != hipSuccess ? e2 : e3));
      }
      hipError_t e4 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e4 != hipSuccess) {
        ex = nullptr;
        return fail(MFS_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(e4));
      }
    }
    MFS_HIP_TRY(hipGraphLaunch(ex, st));
    return MFS_OK;
  };

  // one GMRES cycle from the residual in r; x += V y.  Returns after mlim steps, convergence of all
  // active columns to ktol (relative to kk.bnorm), or the iteration budget.
  auto cycle = [&](KrylovDev kk, double ktol, bool mixed, int mlim) -> mfs_status {
    kk.tol = ktol;
    MFS_HIP_TRY(launch_start_cycle(kk, r, st));
    double est_max = 1.0;
    int read_j = -1;  // last step whose flags the host has read
    bool stop = false;
    const int64_t slot0 = kk.joff;
    for (int j = 0; j < mlim && !stop; ++j) {
      // Arnoldi on the compact part K = S G_hat: w = K v_j, and H(I + K) = H(K) + I (the shift is
      // added in the Givens kernel); the identity's large projection on v_j never enters w.
      if (kk.v32) {
        MFS_TRY(apply_mixed_from32(s, static_cast<const c64*>(kk.V) + (slot0 + j) * NR, w, R, st));
        ++n32;
      } else if (mixed && (opts->fp64_until <= 0.0 || !(est_max > opts->fp64_until))) {
        c128* Vj = static_cast<c128*>(kk.V) + (slot0 + j) * NR;
        MFS_TRY(apply_mixed(s, Vj, w, R, st, 0.0));
        ++n32;
      } else {
        c128* Vj = static_cast<c128*>(kk.V) + (slot0 + j) * NR;
        MFS_TRY(apply_f64(s, Vj, w, R, st, 0.0));
        ++n64;
      }
      MFS_TRY(krylov_step(kk, j, ktol));
      ++total_it;
      const int slot = j % kSlots;
      MFS_HIP_TRY(hipMemcpyAsync(pin_act + slot * R, kk.active, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
      MFS_HIP_TRY(hipMemcpyAsync(pin_res + slot * R, kk.res, sizeof(double) * R, hipMemcpyDeviceToHost, st));
      MFS_HIP_TRY(hipEventRecord(guard.ev[slot], st));
      const bool last = j + 1 == mlim || total_it >= opts->maxit;
      const int lag = (last || !(est_max > 16.0 * ktol)) ? 0 : kSlots - 1;
      while (read_j < j - lag && !stop) {
        ++read_j;
        const int rs = read_j % kSlots;
        MFS_HIP_TRY(hipEventSynchronize(guard.ev[rs]));
        int na = 0;
        est_max = 0.0;
        for (int c = 0; c < R; ++c) {
          na += pin_act[rs * R + c];
          if (pin_act[rs * R + c]) est_max = std::max(est_max, pin_res[rs * R + c]);
        }
        if (opts->verbose > 1 && (read_j + 1) % 250 == 0)
          std::fprintf(stderr, "[mfs_solve] step %d of cycle, %d total, active %d, estimate %.3e, fp32 %d fp64 %d\n",
                       read_j + 1, total_it, na, est_max, n32, n64);
        if (na == 0) stop = true;
      }
      if (total_it >= opts->maxit) stop = true;
    }
    if (kk.ratio_log) {  // diagnostics: distribution of ||w'|| / ||w|| over the cycle (column 0)
      std::vector<double> rl((size_t)m);
      MFS_HIP_TRY(hipMemcpyAsync(rl.data(), kk.ratio_log, sizeof(double) * m, hipMemcpyDeviceToHost, st));
      MFS_HIP_TRY(hipStreamSynchronize(st));
      std::vector<double> v;
      for (int i = 0; i < m && i < total_it; ++i)
        if (rl[i] > 0.0) v.push_back(rl[i]);
      const int len = (int)v.size();
      std::sort(v.begin(), v.end());
      if (len > 0)
        std::fprintf(stderr, "[mfs_solve] ||w'||/||w|| over %d steps: p5 %.3f p25 %.3f p50 %.3f p75 %.3f p95 %.3f\n",
                     len, v[len / 20], v[len / 4], v[len / 2], v[3 * len / 4], v[19 * len / 20]);
    }
    MFS_HIP_TRY(launch_gmres_update_x(kk, x, st));
    return MFS_OK;
  };

  // b = S vhat (eq. mbody2), x0 = 0, r0 = b
  MFS_HIP_TRY(launch_sapply_f64(s->dev, static_cast<const c128*>(vhat_dev), 1, nullptr, 0.0, b, R, (int)s->kmax, st));
  MFS_HIP_TRY(launch_norms(b, N, R, k.part, k.nblk, bnorm_dev, st));
  MFS_TRY(read_doubles(bnorm_dev, bnorm));
  if (opts->use_x0) {
    MFS_TRY(residual());  // r = b - A x0 in FP64
  } else {
    MFS_HIP_TRY(hipMemsetAsync(x, 0, sizeof(c128) * NR, st));
    MFS_HIP_TRY(hipMemcpyAsync(r, b, sizeof(c128) * NR, hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < R; ++c) relres[c] = bnorm[c] > 0.0 ? 1.0 : 0.0;
  }

  if (prec == MFS_FP64) {
    while (max_relres() > opts->tol && total_it < opts->maxit) {
      MFS_TRY(set_active_from_relres());
      MFS_TRY(cycle(k, opts->tol, false, m));
      ++n_restart;
      MFS_TRY(residual());
      if (opts->verbose)
        std::fprintf(stderr, "[mfs_solve fp64] cycle %d  iters %d  max relres %.3e\n", n_restart, total_it,
                     max_relres());
    }
  } else {
    // Deflated correction solves (GCRO, de Sturler 1996): the first inner solve's kold Arnoldi
    // steps give K~ V_k = V_{k+1} Hbar with Hbar = G^H [Rk; 0].  A later correction solve keeps them:
    // C = V_{k+1} Q (Q the first k columns of G^H) is an orthonormal basis of K~ V_k, and
    // U = V_k Rk^{-1} satisfies K~ U = C.  The new process runs on (I - C C^H) K~ from
    // (I - C C^H) r, its basis stored after the kept vectors; the correction is
    // d = W y + U C^H (r - K~ W y).  The new steps thus work only on what the first Krylov space
    // has not resolved, instead of rebuilding it from scratch.  Each column keeps its own k; the
    // new processes share the first free slot after the longest.
    const bool deflate = opts->deflate != 0;
    int o = 0;  // first basis slot of a correction solve's process, 0 while no space is kept
    auto keep_space = [&]() -> mfs_status {
      std::vector<int32_t> jl(R);
      MFS_HIP_TRY(hipMemcpyAsync(jl.data(), k.jlen, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
      MFS_HIP_TRY(hipStreamSynchronize(st));
      int kmax = 0;
      for (int32_t v : jl) kmax = std::max(kmax, (int)v);
      // room for at least 64 new steps after the kept vectors
      if (kmax < 1 || kmax + 1 + 64 > m) return MFS_OK;
      o = kmax + 1;
      MFS_HIP_TRY(hipMemcpyAsync(jold, k.jlen, sizeof(int32_t) * R, hipMemcpyDeviceToDevice, st));
      MFS_HIP_TRY(launch_givens_last_column(k, jold, qdef, st));
      return MFS_OK;
    };
    auto deflated_cycle = [&](double ktol) -> mfs_status {
      const size_t coeff_bytes = sizeof(c128) * (size_t)R * (m + 1);
      KrylovDev kd = k;
      kd.joff = o;
      kd.qdef = qdef;
      kd.kold = jold;
      kd.jdev = nullptr;
      kd.tol_dev = nullptr;
      kd.bnorm = rn2;  // estimate relative to the correction's own residual, before the projection
      // columns already converged get no correction at all
      MFS_HIP_TRY(hipMemcpyAsync(keepdev, active.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, st));
      MFS_HIP_TRY(launch_norms(r, N, R, k.part, k.nblk, rn2, st));
      // c = V^H r over the kept slots;  r <- r - V (c - q q^H c) = (I - C C^H) r
      MFS_HIP_TRY(launch_basis_dots(k, r, o, cdef, st));
      MFS_HIP_TRY(hipMemcpyAsync(edef, cdef, coeff_bytes, hipMemcpyDeviceToDevice, st));
      MFS_HIP_TRY(launch_deflate_coeffs(qdef, o, jold, edef, R, m + 1, keepdev, st));
      MFS_HIP_TRY(launch_basis_axpy(k, edef, o, r, st));
      MFS_TRY(cycle(kd, ktol, true, m - o));  // x += W y
      // x += U C^H (r - K~ W y) = V_k Rk^{-1} [G (c - V^H K~ W y)]_{0..k-1}
      MFS_HIP_TRY(hipMemsetAsync(r, 0, sizeof(c128) * NR, st));
      MFS_HIP_TRY(launch_update_from_y(kd, r, st));  // r = W y
      MFS_TRY(apply_mixed(s, r, w, R, st, 0.0));     // w = K~ W y
      ++n32;
      MFS_HIP_TRY(launch_basis_dots(k, w, o, edef, st));
      MFS_HIP_TRY(launch_axpby(cdef, edef, edef, 1.0, -1.0, (int64_t)R * (m + 1), st));
      // zero the columns left out (projecting q out changes nothing below: G q = e_k)
      MFS_HIP_TRY(launch_deflate_coeffs(qdef, o, jold, edef, R, m + 1, keepdev, st));
      MFS_HIP_TRY(launch_givens_apply(k, jold, edef, st));
      KrylovDev kz = k;
      kz.g = edef;
      kz.jlen = jold;
      MFS_HIP_TRY(launch_gmres_update_x(kz, x, st));
      return MFS_OK;
    };
    while (max_relres() > opts->tol && n_refine < opts->max_refine && total_it < opts->maxit) {
      MFS_TRY(set_active_from_relres());
      KrylovDev kk = k;
      kk.bnorm = kk.beta;  // inner estimate relative to the current residual
      // ask each inner solve for no more reduction than the outer tolerance still needs
      const double itol = std::max(opts->inner_tol, 0.3 * opts->tol / std::max(max_relres(), 1e-300));
      if (o > 0) {
        MFS_TRY(deflated_cycle(std::min(itol, 0.5)));
      } else {
        MFS_TRY(cycle(kk, std::min(itol, 0.5), true, m));
        if (deflate && n_refine == 0) MFS_TRY(keep_space());  // only the first inner solve is kept
      }
      ++n_refine;
      ++n_restart;
      MFS_TRY(residual());
      if (opts->verbose)
        std::fprintf(stderr, "[mfs_solve mixed] refine %d  iters %d  max relres %.3e\n", n_refine, total_it,
                     max_relres());
    }
  }
  std::vector<int32_t> nro(R);
  MFS_HIP_TRY(hipMemcpyAsync(nro.data(), k.n_reorth, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
  MFS_HIP_TRY(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    int32_t mx = 0;
    for (int32_t v : nro) mx = std::max(mx, v);
    info->n_reorth = mx;
    info->n_matvec32 = n32;
    info->n_matvec64 = n64;
    info->n_refine = n_refine;
    info->n_restart = n_restart;
    info->relres_max = max_relres();
    info->t_total_s = std::chrono::duration<double>(t1 - t0).count();
  }
  if (max_relres() > opts->tol)
    return fail(MFS_ERR_NOCONV, "solve: relative residual " + std::to_string(max_relres()) + " above tol after " +
                                    std::to_string(total_it) + " iterations");
  return MFS_OK;
}

// ---------------------------------------------------------- reconstruction ---
mfs_status mfs_recon_create(const mfs_shape_desc* desc, double psi_radius, mfs_recon** out, void* stream) {
  g_last_error.clear();
  if (!out) return fail(MFS_ERR_ARG, "recon_create: out is null");
  *out = nullptr;
  if (!(psi_radius > 0.0) || !std::isfinite(psi_radius))
    return fail(MFS_ERR_ARG, "recon_create: psi_radius must be positive and finite");
  mfs_recon* r = new mfs_recon();
  r->psi_radius = psi_radius;
  r->id = g_recon_ids.fetch_add(1);
  const mfs_status st = build_recon_impl(desc, &r->f, as_stream(stream));
  if (st != MFS_OK) {
    delete r;
    return st;
  }
  *out = r;
  return MFS_OK;
}

mfs_status mfs_recon_destroy(mfs_recon* r) {
  if (!r) return MFS_OK;
  (void)hipDeviceSynchronize();  // kernels on any stream may still read the factors
  pool_free(r->f.block, r->f.block_bytes, nullptr);
  delete r;
  return MFS_OK;
}

mfs_status mfs_recon_size(const mfs_recon* r, int64_t* m, int64_t* n, int64_t* k, int64_t* rank) {
  if (!r) return fail(MFS_ERR_ARG, "recon_size: null handle");
  if (m) *m = r->f.m;
  if (n) *n = r->f.n;
  if (k) *k = r->f.k;
  if (rank) *rank = r->f.rank;
  return MFS_OK;
}

mfs_status mfs_near_sizes(const mfs_scene* sc, const mfs_recon* const* recon, int64_t* colloc_total,
                          int64_t* src_total) {
  MFS_TRY(check_scene(sc));
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  MFS_TRY(prepare_near(s, recon, s->last_stream));
  if (colloc_total) *colloc_total = s->near.Mtot;
  if (src_total) *src_total = s->near.Ntot;
  return MFS_OK;
}

mfs_status mfs_plane_wave_colloc(const mfs_scene* sc, const mfs_recon* const* recon, const double* dirs_host,
                                 int32_t R, void* v_dev, void* stream) {
  MFS_TRY(check_scene(sc));
  if (R < 1 || !dirs_host || !v_dev) return fail(MFS_ERR_ARG, "plane_wave_colloc: bad R or null pointer");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  MFS_TRY(prepare_near(s, recon, st));
  MFS_TRY(ensure(s->dirs, sizeof(double) * R * s->dev.dim, &s->bytes, st));
  MFS_HIP_TRY(hipMemcpyAsync(s->dirs.p, dirs_host, sizeof(double) * R * s->dev.dim, hipMemcpyHostToDevice, st));
  MFS_HIP_TRY(hipStreamSynchronize(st));
  MFS_HIP_TRY(launch_plane_wave_colloc(s->dev, s->near, static_cast<double*>(s->dirs.p), R, static_cast<c128*>(v_dev),
                                       st));
  return MFS_OK;
}

mfs_status mfs_reconstruct(const mfs_scene* sc, const mfs_recon* const* recon, const void* v_colloc_dev,
                           const void* qhat_dev, int32_t R, void* qmfs_dev, void* stream) {
  MFS_TRY(check_scene(sc));
  if (R < 1 || !v_colloc_dev || !qhat_dev || !qmfs_dev) return fail(MFS_ERR_ARG, "reconstruct: bad R or null pointer");
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  MFS_TRY(prepare_near(s, recon, st));
  const int64_t N = s->dev.N;
  const NearTables& t = s->near;
  // w_hat = G_hat qhat (FP64): the field of the other bodies at each body's equivalent points
  const int nch = ghat_f64_slices(s->dev, R, shape_for(s, true, R).nchunks);
  MFS_TRY(ensure(s->partial, (size_t)nch * R * N * sizeof(c128), &s->bytes, st));
  size_t gw = 0, gv = 0;
  hipError_t e = hipSuccess;
  c128* what = static_cast<c128*>(pool_alloc(sizeof(c128) * (size_t)R * N, st, &gw, &e));
  if (!what) return fail(MFS_ERR_NOMEM, std::string("reconstruct: ") + hipGetErrorString(e));
  c128* vs = static_cast<c128*>(pool_alloc(sizeof(c128) * (size_t)R * t.Mtot, st, &gv, &e));
  if (!vs) {
    pool_free(what, gw, st);
    return fail(MFS_ERR_NOMEM, std::string("reconstruct: ") + hipGetErrorString(e));
  }
  struct Temps {
    void *a, *b;
    size_t na, nb;
    hipStream_t st;
    ~Temps() {
      pool_free(a, na, st);
      pool_free(b, nb, st);
    }
  } temps{what, vs, gw, gv, st};
  {
    TimedLaunch tl(MFS_KERNEL_PAIR_F64, s->dev.offbody_pairs * R, st);
    MFS_HIP_TRY(launch_ghat_f64(s->dev, static_cast<const c128*>(qhat_dev), R, static_cast<c128*>(s->partial.p), nch,
                                st));
  }
  MFS_HIP_TRY(launch_reduce_partials_f64(static_cast<c128*>(s->partial.p), nch, N, R, what, st));
  // A^+ v per body: Householder reflectors then back substitution, shape by shape, in place on a copy
  MFS_HIP_TRY(hipMemcpyAsync(vs, v_colloc_dev, sizeof(c128) * (size_t)R * t.Mtot, hipMemcpyDeviceToDevice, st));
  for (int sh = 0; sh < s->n_shapes; ++sh) {
    const int nb = (int)s->bodies_of_shape[sh].size();
    if (nb == 0) continue;
    const ReconFactors& f = recon[sh]->f;
    ColMap cm;
    cm.bodies = s->bodies_dev[sh];
    cm.nb = nb;
    cm.ptr_in = t.cptr;
    cm.ld_in = t.Mtot;
    cm.ptr_out = t.sptr;
    cm.ld_out = t.Ntot;
    const int ncols = nb * R;
    MFS_HIP_TRY(launch_qr_reflect(f.QA, f.m, f.m, f.tau, f.rank, vs, 0, ncols, cm, st));
    MFS_HIP_TRY(launch_backsub(f.QA, f.m, f.alpha, f.rank, vs, 0, f.perm, f.n, static_cast<c128*>(qmfs_dev), 0,
                               ncols, cm, st));
  }
  // q_mfs -= (A^+ U) w_hat
  MFS_HIP_TRY(launch_recon_combine(s->dev, t, what, R, static_cast<c128*>(qmfs_dev), st));
  return MFS_OK;
}

mfs_status mfs_eval_field_near(const mfs_scene* sc, const mfs_recon* const* recon, const void* qhat_dev,
                               const void* qmfs_dev, int32_t R, const double* targets_dev, int64_t M, void* u_dev,
                               void* stream) {
  MFS_TRY(check_scene(sc));
  if (R < 1 || M < 0 || !qhat_dev || !qmfs_dev || !u_dev || (M > 0 && !targets_dev))
    return fail(MFS_ERR_ARG, "eval_field_near: bad sizes or pointers");
  if (M == 0) return MFS_OK;
  mfs_scene* s = const_cast<mfs_scene*>(sc);
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  MFS_TRY(prepare_near(s, recon, st));
  const int nch = near_chunks_for(s->dev.T, M);
  MFS_TRY(ensure(s->partial, (size_t)nch * R * M * sizeof(c128), &s->bytes, st));
  c128* part = static_cast<c128*>(s->partial.p);
  MFS_HIP_TRY(launch_eval_near(s->dev, s->near, static_cast<const c128*>(qhat_dev), static_cast<const c128*>(qmfs_dev),
                               R, targets_dev, M, part, nch, st));
  MFS_HIP_TRY(launch_reduce_partials_f64(part, nch, M, R, static_cast<c128*>(u_dev), st));
  return MFS_OK;
}

mfs_status mfs_pool_query(mfs_pool_stats* out) {
  if (!out) return fail(MFS_ERR_ARG, "pool_query: null output");
  pool_query(&out->hits, &out->misses, &out->cached_bytes, &out->live_bytes, &out->limit_bytes);
  return MFS_OK;
}

mfs_status mfs_pool_set_limit(int64_t max_cached_bytes) {
  if (max_cached_bytes < 0) return fail(MFS_ERR_ARG, "pool_set_limit: negative limit");
  pool_set_limit((size_t)max_cached_bytes);
  return MFS_OK;
}

mfs_status mfs_pool_trim(void) {
  pool_trim();
  return MFS_OK;
}

mfs_status mfs_sym_slice_budget(int64_t bytes, int64_t* previous) {
  const int64_t old = sym_slice_budget(bytes);
  if (previous) *previous = old > 0 ? old : kSymSliceBudget;
  return MFS_OK;
}

mfs_status mfs_autotune(mfs_scene* s, int32_t R, mfs_prec prec, int32_t reps, mfs_tune_result* out, void* stream) {
  MFS_TRY(check_scene(s));
  if (prec != MFS_FP64 && prec != MFS_FP32 && prec != MFS_MIXED)
    return fail(MFS_ERR_ARG, "autotune: precision must be MFS_FP64, MFS_FP32 or MFS_MIXED");
  if (prec != MFS_FP64 && !s->has_s32) return fail(MFS_ERR_ARG, "scene was created without FP32 copies of S");
  if (R < 1 || reps < 1 || reps > 1000) return fail(MFS_ERR_ARG, "autotune: need R >= 1 and 1 <= reps <= 1000");
  hipStream_t st = as_stream(stream);
  s->last_stream = st;
  mfs_tune_result res{};
  const int64_t N = s->dev.N;
  if (N == 0) {
    if (out) *out = res;
    return MFS_OK;
  }
  const bool f64 = prec == MFS_FP64;
  const int v = tune_variant(s, f64, R);
  const std::pair<int, int> key{v, R};
  const size_t part_elem = f64 ? sizeof(c128) : sizeof(c64);
  const int maxc = (int)std::min<int64_t>(kTuneMaxChunks, std::max<int64_t>(1, N / 16));

  // candidates, the untuned shape first: slice counts from h/4 to 4h around each kernel's heuristic
  // (capped so that the partial sums stay within max(2 GiB, the heuristic's)), times 1, 2 or 4
  // right-hand sides per thread on the VALU kernel, and the symmetric kernel where it applies
  std::vector<LaunchShape> cands;
  auto add = [&](LaunchShape c) {
    for (const LaunchShape& o : cands)
      if (o.nchunks == c.nchunks && o.rt == c.rt && o.sym == c.sym) return;
    cands.push_back(c);
  };
  const bool sym_ok = v != kTunePairF64 && ghat_sym_possible(s->dev, R);
  const int h = pair_chunks_for(N, N, tpt_for(f64 ? MFS_FP64 : MFS_FP32));
  const int h_rt = v == kTunePairF32 ? ghat_default_rt(R) : 0;
  const size_t cap = std::max<size_t>((size_t)2 << 30, (size_t)h * R * N * part_elem);
  auto plain = [&]() {
    std::vector<int> rset{h_rt};
    if (v == kTunePairF32)
      for (int rt : {1, 2, 4})
        if (rt != h_rt && (rt == 1 || rt / 2 < R)) rset.push_back(rt);
    for (int f : {0, -2, -1, 1, 2}) {
      int c = f < 0 ? (h >> -f) : (h << f);
      c = std::max(1, std::min(c, maxc));
      if (f != 0 && (size_t)c * R * N * part_elem > cap) continue;
      for (int rt : rset) add(LaunchShape{c, rt, 0});
    }
  };
  if (sym_ok) {
    const int64_t NS = sym_view(s->dev).N;
    const int W = sym_block_waves(NS, R);
    const SymPlan hp = sym_plan(NS, 0, W);
    std::vector<int> rset{ghat_default_rt(R)};
    for (int rt : {1, 2, 4})
      if (rt != rset[0] && (rt == 1 || rt / 2 < R)) rset.push_back(rt);
    for (int f : {0, -2, -1, 1, 2}) {
      const int c = f < 0 ? (hp.nchunks_d >> -f) : (hp.nchunks_d << f);
      for (int rt : rset) add(LaunchShape{sym_plan(NS, std::max(1, std::min(c, kTuneMaxChunks)), W).nchunks_d, rt, 1});
    }
  }
  plain();

  const size_t vec = (prec == MFS_FP32 ? sizeof(c64) : sizeof(c128)) * (size_t)R * N;
  struct Scratch {
    void* p[2] = {nullptr, nullptr};
    size_t n[2] = {0, 0};
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t st;
    ~Scratch() {
      for (int i = 0; i < 2; ++i) {
        if (p[i]) pool_free(p[i], n[i], st);
        if (ev[i]) (void)hipEventDestroy(ev[i]);
      }
    }
  } sc;
  sc.st = st;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2; ++i) {
    sc.p[i] = pool_alloc(vec, st, &sc.n[i], &e);
    if (!sc.p[i]) return fail(MFS_ERR_NOMEM, std::string("autotune: ") + hipGetErrorString(e));
    MFS_HIP_TRY(hipEventCreate(&sc.ev[i]));
  }
  MFS_HIP_TRY(hipMemsetAsync(sc.p[0], 0x3c, vec, st));  // charges of modest size (no denormals)
  auto run = [&]() -> mfs_status {
    if (prec == MFS_FP64) return apply_f64(s, static_cast<const c128*>(sc.p[0]), static_cast<c128*>(sc.p[1]), R, st);
    if (prec == MFS_FP32) return apply_f32(s, static_cast<const c64*>(sc.p[0]), static_cast<c64*>(sc.p[1]), R, st);
    return apply_mixed(s, static_cast<const c128*>(sc.p[0]), static_cast<c128*>(sc.p[1]), R, st);
  };
  auto prior = s->tuned.find(key);
  const bool had = prior != s->tuned.end();
  const LaunchShape before = had ? prior->second : LaunchShape{};
  auto restore = [&]() {
    if (had) s->tuned[key] = before;
    else s->tuned.erase(key);
  };
  double best = 0.0, ms_h = 0.0, ms_plain = -1.0;
  LaunchShape best_ls = cands.front();
  for (size_t i = 0; i < cands.size(); ++i) {
    s->tuned[key] = cands[i];
    mfs_status rc = run();  // warm-up; sizes the partial sums
    if (rc == MFS_OK && hipEventRecord(sc.ev[0], st) != hipSuccess) rc = fail(MFS_ERR_HIP, "autotune: event record");
    for (int r = 0; rc == MFS_OK && r < reps; ++r) rc = run();
    float ms = 0.0f;
    if (rc == MFS_OK && (hipEventRecord(sc.ev[1], st) != hipSuccess || hipEventSynchronize(sc.ev[1]) != hipSuccess ||
                         hipEventElapsedTime(&ms, sc.ev[0], sc.ev[1]) != hipSuccess))
      rc = fail(MFS_ERR_HIP, "autotune: event timing failed");
    if (rc != MFS_OK) {
      restore();
      return rc;
    }
    const double t = (double)ms / reps;
    if (i == 0) ms_h = t;
    if (cands[i].sym == 0 && ms_plain < 0.0) ms_plain = t;  // the plain kernel's heuristic shape
    // another shape replaces the untuned one only when it is clearly faster (2%), so that timing
    // noise does not make the choice wander between runs
    if (i == 0 || (t < best && t < 0.98 * ms_h)) {
      best = t;
      best_ls = cands[i];
    }
  }
  s->tuned[key] = best_ls;
  tune_store(s->dev.dim, v, R, N, best_ls);
  // the largest candidate may have grown the partial-sum buffer well past what the winner needs
  const size_t need = f64 ? (size_t)best_ls.nchunks * R * N * part_elem
                          : (size_t)f32_slices(s, best_ls, R) * R * f32_rows(s, best_ls) * part_elem;
  if (s->partial.cap > 2 * need) release(s->partial, &s->bytes, st);
  res.nchunks = best_ls.nchunks;
  res.rhs_per_thread = (v == kTunePairF32 || best_ls.sym == 1) ? (best_ls.rt ? best_ls.rt : ghat_default_rt(R)) : 0;
  res.ms = best;
  res.ms_heuristic = ms_h;
  res.n_tried = (int32_t)cands.size();
  res.uses_mfma = v == kTunePairMfma && best_ls.sym != 1 ? 1 : 0;
  res.symmetric = best_ls.sym == 1 ? 1 : 0;
  res.ms_plain = ms_plain;
  if (out) *out = res;
  return MFS_OK;
}

mfs_status mfs_tune_get(const mfs_scene* s, int32_t R, mfs_prec prec, int32_t* nchunks, int32_t* rhs_per_thread,
                        int32_t* symmetric, int32_t* source) {
  MFS_TRY(check_scene(s));
  if (R < 1) return fail(MFS_ERR_ARG, "tune_get: R must be >= 1");
  const bool f64 = prec == MFS_FP64;
  const int v = tune_variant(s, f64, R);
  int src = 0;
  const LaunchShape ls = shape_for(s, f64, R, &src);
  if (nchunks) *nchunks = ls.nchunks;
  if (rhs_per_thread)
    *rhs_per_thread = (v == kTunePairF32 || ls.sym == 1) ? (ls.rt ? ls.rt : ghat_default_rt(R)) : 0;
  if (symmetric) *symmetric = ls.sym == 1 ? 1 : 0;
  if (source) *source = src;
  return MFS_OK;
}

mfs_status mfs_pair_kernel(const mfs_scene* s, int32_t R, mfs_prec prec, int32_t* kind) {
  MFS_TRY(check_scene(s));
  if (R < 1) return fail(MFS_ERR_ARG, "pair_kernel: R must be >= 1");
  if (!kind) return fail(MFS_ERR_ARG, "pair_kernel: kind is null");
  if (prec == MFS_FP64) {
    *kind = ghat_uses_mfma(s->dev, R) ? MFS_PAIR_MC_F64 : MFS_PAIR_F64;
    return MFS_OK;
  }
  const LaunchShape ls = shape_for(s, false, R);
  if (ls.sym == 1) {
    const bool shared = sym_block_waves(f32_rows(s, ls), R) > 1;
    *kind = s->dev.sym16 ? (shared ? MFS_PAIR_F32_SYM16_SHARED : MFS_PAIR_F32_SYM16)
                         : (shared ? MFS_PAIR_F32_SYM_SHARED : MFS_PAIR_F32_SYM);
  }
  else if (ghat_uses_mfma16(s->dev, R)) *kind = MFS_PAIR_MC_F16X3;
  else if (ghat_uses_mfma(s->dev, R)) *kind = MFS_PAIR_MC_F32;
  else *kind = MFS_PAIR_F32;
  return MFS_OK;
}

mfs_status mfs_scene_set_split_fp16(mfs_scene* s, int32_t enable) {
  MFS_TRY(check_scene(s));
  if (enable != 0 && enable != 1) return fail(MFS_ERR_ARG, "scene_set_split_fp16: enable must be 0 or 1");
  if (enable && s->phi16_shift_auto < 0)
    return fail(MFS_ERR_ARG, "scene_set_split_fp16: no bound on |phi| is known for this scene (bodies too close)");
  s->dev.phi16_shift = enable ? s->phi16_shift_auto : -1;
  return MFS_OK;
}

mfs_status mfs_tune_set(mfs_scene* s, int32_t R, mfs_prec prec, int32_t nchunks, int32_t rhs_per_thread,
                        int32_t symmetric) {
  MFS_TRY(check_scene(s));
  if (R < 1) return fail(MFS_ERR_ARG, "tune_set: R must be >= 1");
  if (nchunks < 0 || nchunks > kTuneMaxChunks)
    return fail(MFS_ERR_ARG, "tune_set: nchunks must be in 0.." + std::to_string(kTuneMaxChunks));
  if (rhs_per_thread != 0 && rhs_per_thread != 1 && rhs_per_thread != 2 && rhs_per_thread != 4)
    return fail(MFS_ERR_ARG, "tune_set: rhs_per_thread must be 0, 1, 2 or 4");
  if (symmetric < -1 || symmetric > 1) return fail(MFS_ERR_ARG, "tune_set: symmetric must be -1, 0 or 1");
  const std::pair<int, int> key{tune_variant(s, prec == MFS_FP64, R), R};
  if (nchunks == 0) s->tuned.erase(key);
  else s->tuned[key] = LaunchShape{nchunks, rhs_per_thread, symmetric};
  return MFS_OK;
}

mfs_status mfs_tune_save(const char* path) {
  if (!path) return fail(MFS_ERR_ARG, "tune_save: null path");
  std::string err;
  return tune_save(path, &err) ? MFS_OK : fail(MFS_ERR_ARG, err);
}

mfs_status mfs_tune_load(const char* path) {
  if (!path) return fail(MFS_ERR_ARG, "tune_load: null path");
  std::string err;
  return tune_load(path, &err) ? MFS_OK : fail(MFS_ERR_ARG, err);
}

mfs_status mfs_tune_clear(void) {
  tune_clear();
  return MFS_OK;
}

mfs_status mfs_tune_table_size(int64_t* entries) {
  if (!entries) return fail(MFS_ERR_ARG, "tune_table_size: null output");
  *entries = tune_size();
  return MFS_OK;
}

mfs_status mfs_timing_enable(int32_t on) {
  timing_clear();
  g_timing_on = on != 0;
  return MFS_OK;
}

mfs_status mfs_timing_read(mfs_kernel_kind kind, double* total_ms, int64_t* launches, double* pairs) {
  double ms = 0.0, pr = 0.0;
  int64_t n = 0;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto& r : g_timing) {
    if (r.kind != (int)kind) continue;
    MFS_HIP_TRY(hipEventSynchronize(r.e1));
    float t = 0.0f;
    MFS_HIP_TRY(hipEventElapsedTime(&t, r.e0, r.e1));
    ms += t;
    pr += r.pairs;
    ++n;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (pairs) *pairs = pr;
  return MFS_OK;
}

}  // extern "C"
