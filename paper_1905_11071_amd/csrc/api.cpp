// C ABI of libslista: argument checks, workspace layout and the stream-ordered
// sequence of launches for the forward and reverse passes of Step-LISTA.
//
// Forward (Section 4, Eq. (14)), z^(0) = 0:
//   prep     c = D^T x (FP32 MFMA product with D^T), ||x||^2 (FP64)
//   layer 0  z^(1) = ST(a_0 c, lam a_0)                       (elementwise)
//   layer t  z^(t+1) = ST(z^t - a_t (G z^t - c), lam a_t)     (fused MFMA kernel)
//   final    F(z^T) from G z^T                                (fused MFMA kernel)
// Reverse (hand-derived; the paper differentiates by autodiff, Appendix D):
//   seed     v^{T-1} = [z^T != 0] (dF (G z^T - c + lam sign z^T) + dZ)
//   layer t  dJ/da_t = -(1/a_t) sum v^t (z^t - z^{t+1});
//            v^{t-1} = [z^t != 0] (v^t - a_t G v^t)           (fused MFMA kernel)
//   layer 0  dJ/da_0 from v^0 and z^(1) only                  (elementwise)
// With checkpointing every k layers the forward keeps z^k, z^2k, ... and z^T;
// the reverse pass recomputes each segment's interior before walking it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/slista.h"
#include "common.hpp"
#include "persist.hpp"
#include "lista_persist.hpp"

struct slista_dict {
  slista::Dict d;
};

struct slista_batch {
  int P = 0, T = 0, prec = 0, k = 1;
  int base = 0, tail = 0;              // precision schedule (see parse_sched)
  std::vector<slista_problem> probs;
  std::vector<size_t> offset;          // workspace offset of each problem
  size_t total = 0;
  // buckets of the persistent kernels; per contraction precision (index
  // slista::kF32 / kBF16) a tile variant and a work list
  struct Bucket {
    int np = 0, max_m_pad = 0, rows_total = 0;
    int variant[2] = {0, 0}, nwork[2] = {0, 0};
    std::vector<int> problems;
    size_t work_off[2] = {0, 0};        // index of the bucket's first work item
    size_t small_off = 0;               // index of its first entry in d_small (and d_corr)
    size_t tstart_off = 0;              // index of its tile-start prefix sums in d_tstart
    int corr_tiles = 0;                 // correlation-product tiles of its problems
    int max_N = 0;                      // largest N of its problems
    size_t max_group_elems = 0;         // largest row-group copy of c (float4 count)
  };
  std::vector<Bucket> buckets;
  std::vector<int> rows[2];             // tile rows per problem
  bool uses[2] = {false, false};        // precisions the schedule runs
  // device tables (owned)
  slista::PersistArgs* d_args[2] = {nullptr, nullptr};
  int2* d_work = nullptr;
  size_t work_cap = 0;                  // entries d_work holds
  slista::BatchSmall* d_small = nullptr;  // [P] small-kernel table, bucket by bucket
  slista::GemmArgs* d_corr = nullptr;     // [P] correlation-product arguments, same order
  int* d_tstart = nullptr;                // per bucket: tile-start prefix sums
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // one stream per bucket (default priority), forked from and joined into
  // the caller's stream with events, so that the buckets run concurrently
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;  // [0]: fork; [1 + bi]: bucket bi done
};

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(SLISTA_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// ---------------------------------------------------------------- timing
// Event pairs around every launch while recording is on (slista_profile_*).
enum Kind { kKCorr = 0, kKFwd = 1, kKFinal = 2, kKSeed = 3, kKBwd = 4, kKOther = 5 };
constexpr size_t kMaxRecords = 65536;

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, size_t>> recs;
  int dropped = 0;
};
Profiler g_prof;

struct ProfScope {
  size_t idx = (size_t)-1;
  int kind;
  hipStream_t s;
  ProfScope(int k, hipStream_t st) : kind(k), s(st) {
    if (!g_prof.on) return;
    if (g_prof.recs.size() >= kMaxRecords) {
      ++g_prof.dropped;
      return;
    }
    const size_t i = 2 * g_prof.recs.size();
    while (g_prof.pool.size() < i + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      g_prof.pool.push_back(e);
    }
    if (hipEventRecord(g_prof.pool[i], s) == hipSuccess) idx = i;
  }
  ~ProfScope() {
    if (idx == (size_t)-1) return;
    if (hipEventRecord(g_prof.pool[idx + 1], s) == hipSuccess) g_prof.recs.emplace_back(kind, idx);
  }
};

#define LAUNCH(kind, stream, expr)     \
  do {                                 \
    ProfScope ps_((kind), (stream));   \
    HIP_TRY(expr);                     \
  } while (0)

// Kernel family: 0 = automatic (persistent kernels when m_pad <= 2048),
// 1 = per-layer kernels, 2 = persistent kernels (falls back to per-layer
// where they do not apply). Set through slista_set_option.
int g_kernel_family = 0;
// Tile variant of the persistent kernels (0 = default; see persist_rows).
int g_persist_variant = 0;
// Finite-value checks of inputs and outputs (SLISTA_OPT_CHECK_FINITE).
int g_check_finite = 0;
// Autotuned variants: (precision, column-pass bucket, floor(log2 N)) -> variant,
// shared by all threads (g_tuned_mu guards it).
std::map<std::tuple<int, int, int>, int> g_tuned;
std::mutex g_tuned_mu;
// The autotuners run their timing calls with these per-thread overrides of
// the family and the variant, so other threads keep their settings.
thread_local int t_family_override = -1;
thread_local int t_variant_override = -1;

int kernel_family() { return t_family_override >= 0 ? t_family_override : g_kernel_family; }

int log2_bucket(int N) {
  int b = 0;
  while (N > 1) {
    N >>= 1;
    ++b;
  }
  return b;
}

// The tile variant a call uses: the forced one, else the tuned one, else 0
// (the kernels' built-in default).
int variant_for(int prec, int m_pad, int N) {
  if (t_variant_override >= 0) return t_variant_override;
  if (g_persist_variant != 0) return g_persist_variant;
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  const auto it = g_tuned.find(std::make_tuple(prec, slista::persist_np(m_pad), log2_bucket(N)));
  return it == g_tuned.end() ? 0 : it->second;
}

void record_tuned(int prec, int np, int nbucket, int variant) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  g_tuned[std::make_tuple(prec, np, nbucket)] = variant;
}

constexpr int kMaxN = 1 << 26;
constexpr int kMaxT = 100000;
constexpr int kMaxM = 8192;
constexpr int kMaxn = 65536;
constexpr int kTileRows = 128;  // rows of the fused kernel's workgroup tile
constexpr int kTileCols = 128;  // columns of the fused kernel's workgroup tile

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t C = 0, Cg = 0, xsq = 0, Fd = 0, fpart = 0, dpart = 0, pp = 0, ckpt = 0, seg = 0, vbuf = 0;
  size_t total = 0;
  size_t zbytes = 0;
  int k = 0, nckpt = 0, nseg = 0, col_tiles = 0, P = 0;
  bool groups = false;  // Cg is there
};

Layout make_layout(const slista::Dict& d, int N, int T, int k, bool groups = true) {
  Layout L;
  L.k = k;
  // N rounded up to whole 64-row tiles: the persistent kernels keep the
  // iterates in the accumulator's row order (four rows of a column together)
  // and load every row group of a tile unconditionally
  L.zbytes = (size_t)slista::tape_rows(N) * d.m_pad * sizeof(float);
  const int row_tiles = (N + kTileRows - 1) / kTileRows;
  L.col_tiles = (d.m_pad + kTileCols - 1) / kTileCols;
  int P = row_tiles * L.col_tiles;
  const int p0 = slista::bwd0_blocks(N, d.m_pad);
  const int pt = (N + 15) / 16;  // persistent tiles have at least 16 rows
  L.P = P > p0 ? P : p0;
  if (pt > L.P) L.P = pt;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.C = take(L.zbytes);
  L.groups = groups;
  if (groups) L.Cg = take(L.zbytes);  // c in the same row-group order, read by the persistent forward
  L.xsq = take((size_t)N * sizeof(double));
  L.Fd = take((size_t)N * sizeof(double));
  L.fpart = take((size_t)L.col_tiles * N * sizeof(double));
  if (k == 0) {
    L.pp = take(2 * L.zbytes);
  } else {
    L.nckpt = (T + k - 1) / k;
    L.nseg = k - 1;
    L.ckpt = take((size_t)L.nckpt * L.zbytes);
    L.seg = take((size_t)L.nseg * L.zbytes);
    L.vbuf = take(2 * L.zbytes);
    L.dpart = take((size_t)T * L.P * sizeof(double));
  }
  L.total = off;
  return L;
}

struct Run {
  const slista::Dict* d;
  Layout L;
  char* ws;
  int N, T;
  hipStream_t s;

  float* C() const { return (float*)(ws + L.C); }
  float* Cg() const { return L.groups ? (float*)(ws + L.Cg) : nullptr; }
  double* xsq() const { return (double*)(ws + L.xsq); }
  double* Fd() const { return (double*)(ws + L.Fd); }
  double* fpart() const { return (double*)(ws + L.fpart); }
  double* dpart() const { return (double*)(ws + L.dpart); }
  float* vbuf(int i) const { return (float*)(ws + L.vbuf + (size_t)(i & 1) * L.zbytes); }
  // Where z^(t), t >= 1, lives.
  float* slot(int t) const {
    if (L.k == 0) return (float*)(ws + L.pp + (size_t)(t & 1) * L.zbytes);
    if (t % L.k == 0 || t == T) return (float*)(ws + L.ckpt + (size_t)((t + L.k - 1) / L.k - 1) * L.zbytes);
    return (float*)(ws + L.seg + (size_t)(t % L.k - 1) * L.zbytes);
  }
};

slista::GemmArgs base_args(const Run& r, const float* alpha, float lam) {
  slista::GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.rows = r.N;
  g.ncols = r.d->m_pad;
  g.K = r.d->m_pad;
  g.lda = r.d->m_pad;
  g.ldb = r.d->m_pad;
  g.ldz = r.d->m_pad;
  g.alpha = alpha;
  g.lam = lam;
  g.C = r.C();
  g.m = r.d->m;
  slista::gemm_grid(r.N, r.d->m_pad, g);
  return g;
}

const void* gram_for(const slista::Dict& d, int prec) {
  return prec == slista::kF32 ? (const void*)d.G32 : (const void*)d.Gb;
}

bool use_persist(const Run& r, int prec) {
  if (kernel_family() == 1) return false;
  return slista::persist_rows(prec, r.d->m_pad, variant_for(prec, r.d->m_pad, r.N)) > 0;
}

// ---------------------------------------------------------------- precision schedule
// The `prec` argument of the forward/backward entry points: its low byte is
// the contraction precision (SLISTA_FP32 or SLISTA_BF16); with SLISTA_BF16,
// bits 8 and up may give an FP32 tail: the last `tail` layers contract in FP32.
struct Sched {
  int base = 0, tail = 0, T = 0;
  // contraction precision of layer t (z^t -> z^{t+1})
  int at(int t) const { return (tail > 0 && t >= T - tail) ? (int)slista::kF32 : base; }
  int split() const { return tail > 0 && tail < T ? T - tail : 1 << 30; }
};

int parse_sched(int prec, int T, int ckpt_every, Sched* sc) {
  if (prec < 0) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  const int base = prec & 0xff, tail = prec >> 8;
  if (base != SLISTA_FP32 && base != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  if (tail > 0 && base != SLISTA_BF16) return fail(SLISTA_EINVAL, "an FP32 tail needs SLISTA_BF16 layers before it");
  if (tail > T) return fail(SLISTA_EINVAL, "FP32 tail of %d layers is longer than T=%d", tail, T);
  if (tail > 0 && tail < T && ckpt_every > 1 && (T - tail) % ckpt_every != 0)
    return fail(SLISTA_EINVAL, "the first FP32 layer (T - tail = %d) must be a checkpoint (ckpt_every=%d)", T - tail,
                ckpt_every);
  sc->base = base;
  sc->tail = tail;
  sc->T = T;
  return SLISTA_OK;
}

// Layer ranges that run in one precision: one span, or a BF16 span and the FP32 tail.
struct Span {
  int t0, t1, prec;
};
int spans_of(const Sched& sc, Span out[2]) {
  if (sc.tail == 0 || sc.tail >= sc.T) {
    out[0] = Span{0, sc.T, sc.tail > 0 ? (int)slista::kF32 : sc.base};
    return 1;
  }
  out[0] = Span{0, sc.T - sc.tail, sc.base};
  out[1] = Span{sc.T - sc.tail, sc.T, (int)slista::kF32};
  return 2;
}

bool use_persist(const Run& r, const Sched& sc) {
  Span sp[2];
  const int ns = spans_of(sc, sp);
  for (int i = 0; i < ns; ++i)
    if (!use_persist(r, sp[i].prec)) return false;
  return true;
}

// Tiles of the persistent kernels for precision p on this run.
int persist_tiles(const Run& r, int p) {
  const int rows = slista::persist_rows(p, r.d->m_pad, variant_for(p, r.d->m_pad, r.N));
  return (r.N + rows - 1) / rows;
}

// ---------------------------------------------------------------- tape registry
// What a forward pass left in a workspace, recorded on the host, keyed by the
// workspace's address range: a backward call uses the tape only if it was
// kept for the same arguments, kernel family and tile variants, and
// recomputes it otherwise. Every entry point that writes a caller workspace
// drops the records its range overlaps.
struct TapeTag {
  const slista::Dict* d;
  const float* X;
  const float* alpha;
  int N, T, prec, k, family, variant0, variant1;
  float lam;
  // Which of the tape's slots hold the forward's iterates: the checkpoints
  // always; the interior of the last segment (which the forward keeps) only
  // until a backward pass with several segments has recomputed the earlier
  // segments into the same slots.
  bool operator==(const TapeTag& o) const {
    return d == o.d && X == o.X && alpha == o.alpha && N == o.N && T == o.T && prec == o.prec && k == o.k &&
           family == o.family && variant0 == o.variant0 && variant1 == o.variant1 &&
           std::memcmp(&lam, &o.lam, sizeof lam) == 0;
  }
};
struct TapeRec {
  uintptr_t lo, hi;
  TapeTag tag;
  bool last_interior;
};
std::mutex g_tape_mu;
std::vector<TapeRec> g_tapes;
constexpr size_t kMaxTapes = 4096;

TapeTag tape_tag(const Run& r, const float* X, float lam, const float* alpha, int prec) {
  TapeTag t;
  std::memset(&t, 0, sizeof t);
  t.d = r.d;
  t.X = X;
  t.alpha = alpha;
  t.N = r.N;
  t.T = r.T;
  t.prec = prec;
  t.k = r.L.k;
  t.family = kernel_family();
  t.variant0 = variant_for(slista::kF32, r.d->m_pad, r.N);
  t.variant1 = variant_for(slista::kBF16, r.d->m_pad, r.N);
  t.lam = lam;
  return t;
}

void tape_forget(const void* ws, size_t bytes) {
  const uintptr_t lo = (uintptr_t)ws, hi = lo + (bytes > 0 ? bytes : 1);
  std::lock_guard<std::mutex> lock(g_tape_mu);
  g_tapes.erase(std::remove_if(g_tapes.begin(), g_tapes.end(),
                               [&](const TapeRec& t) { return t.lo < hi && lo < t.hi; }),
                g_tapes.end());
}

void tape_record(const void* ws, size_t bytes, const TapeTag& tag, bool last_interior) {
  tape_forget(ws, bytes);
  std::lock_guard<std::mutex> lock(g_tape_mu);
  if (g_tapes.size() >= kMaxTapes) g_tapes.erase(g_tapes.begin());
  g_tapes.push_back(TapeRec{(uintptr_t)ws, (uintptr_t)ws + bytes, tag, last_interior});
}

// 0: no tape of this forward in ws; 1: checkpoints only; 2: the whole tape.
int tape_state(const void* ws, const TapeTag& tag) {
  std::lock_guard<std::mutex> lock(g_tape_mu);
  for (const auto& t : g_tapes)
    if (t.lo == (uintptr_t)ws && t.tag == tag) return t.last_interior ? 2 : 1;
  return 0;
}

// Whether a backward pass over this layout leaves the last segment's interior
// in place (it recomputes the earlier segments into the same slots).
bool backward_keeps_interior(const Layout& L, int T) { return L.k <= 1 || (T + L.k - 1) / L.k <= 1; }

// ---------------------------------------------------------------- finite-value checks
// With SLISTA_OPT_CHECK_FINITE on: count NaN / Inf entries of the given
// buffers on the device and synchronise; SLISTA_ENONFINITE if any.
struct Buf {
  const float* p;
  size_t n;
};
int check_finite(const slista::Dict& d, hipStream_t s, std::initializer_list<Buf> bufs, const char* what) {
  if (!g_check_finite) return SLISTA_OK;
  LAUNCH(kKOther, s, slista::launch_zero_u32(d.flag, s));
  for (const Buf& b : bufs) LAUNCH(kKOther, s, slista::launch_count_nonfinite(b.p, b.n, d.flag, s));
  unsigned int cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, d.flag, sizeof cnt, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (cnt) return fail(SLISTA_ENONFINITE, "%u non-finite values in %s", cnt, what);
  return SLISTA_OK;
}

slista::PersistArgs persist_args(const Run& r, int prec, const float* alpha, float lam) {
  slista::PersistArgs a;
  std::memset(&a, 0, sizeof a);
  a.Gsw = prec == slista::kF32 ? (const void*)r.d->Gsf : (const void*)r.d->Gsb;
  a.m_pad = r.d->m_pad;
  a.KC = r.d->m_pad * (prec == slista::kF32 ? 4 : 2) / 64;
  a.N = r.N;
  a.m = r.d->m;
  a.Cg = r.Cg();
  a.alpha = alpha;
  a.lam = lam;
  a.ckpt = r.ws + r.L.ckpt;
  a.seg = r.ws + r.L.seg;
  a.zbytes = r.L.zbytes;
  a.k = r.L.k;
  a.T = r.T;
  a.a_last = r.L.k > 0 && r.T > 0 ? ((r.T - 1) / r.L.k) * r.L.k : 0;
  a.xsq = r.xsq();
  a.P_stride = r.L.P;
  return a;
}

// One forward layer t >= 1: z^(t+1) from z^(t).
int fwd_layer(const Run& r, int prec, const float* alpha, float lam, int t, double* fpart) {
  slista::GemmArgs g = base_args(r, alpha, lam);
  g.A = r.slot(t);
  g.Bt = gram_for(*r.d, prec);
  g.t = t;
  g.Zt = r.slot(t);
  g.Out = r.slot(t + 1);
  g.fpart = fpart;
  LAUNCH(kKFwd, r.s, slista::launch_gemm(prec, slista::kEpiFwd, false, g, r.s));
  return SLISTA_OK;
}

// Arguments of the correlation product c = D^T x for every sample (row-major).
slista::GemmArgs corr_args(const Run& r, const float* X) {
  slista::GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = X;
  g.lda = r.d->n;
  g.Bt = r.d->Dt;
  g.ldb = r.d->n;
  g.rows = r.N;
  g.ncols = r.d->m_pad;
  g.K = r.d->n;
  g.Out = r.C();
  g.ldz = r.d->m_pad;
  slista::gemm_grid(r.N, r.d->m_pad, g);
  return g;
}

int prep_corr(const Run& r, const float* X) {
  const slista::GemmArgs g = corr_args(r, X);
  LAUNCH(kKCorr, r.s, slista::launch_gemm(slista::kF32, slista::kEpiCorr, true, g, r.s));
  return SLISTA_OK;
}

// c, the norms ||x_i||^2, and, where the layout has room for it, the
// row-group copy of c that the persistent forward reads.
int prep(const Run& r, const float* X) {
  int st = prep_corr(r, X);
  if (st != SLISTA_OK) return st;
  if (r.L.groups) LAUNCH(kKOther, r.s, slista::launch_row_groups(r.C(), r.N, r.d->m_pad, r.Cg(), r.s));
  LAUNCH(kKOther, r.s, slista::launch_xsq(X, r.N, r.d->n, r.xsq(), r.s));
  return SLISTA_OK;
}

int check_common(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha, int T,
                 int prec, int ckpt_every, void* ws, size_t ws_bytes, size_t* need, Sched* sc = nullptr) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  if (T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "T=%d outside [0, %d]", T, kMaxT);
  if (!(lambda > 0.f) || !std::isfinite(lambda))
    return fail(SLISTA_EINVAL, "lambda=%g must be finite and > 0", (double)lambda);
  if (ckpt_every < 0 || ckpt_every > kMaxT)
    return fail(SLISTA_EINVAL, "ckpt_every=%d outside [0, %d]", ckpt_every, kMaxT);
  if (sc) {
    const int st = parse_sched(prec, T, ckpt_every, sc);
    if (st != SLISTA_OK) return st;
  } else if (prec != SLISTA_FP32 && prec != SLISTA_BF16) {
    return fail(SLISTA_EINVAL, "unknown precision %d (FP32 tails are not taken here)", prec);
  }
  if (N > 0 && !X) return fail(SLISTA_EINVAL, "X is NULL");
  if (T > 0 && !alpha) return fail(SLISTA_EINVAL, "alpha is NULL");
  const Layout L = make_layout(dict->d, N, T, ckpt_every);
  *need = L.total;
  if (L.total > 0) {
    if (!ws) return fail(SLISTA_EINVAL, "workspace is NULL (%zu bytes needed)", L.total);
    if (((uintptr_t)ws & 255) != 0) return fail(SLISTA_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < L.total)
      return fail(SLISTA_EINVAL, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  }
  return SLISTA_OK;
}

// Forward pass into the workspace. want_final: evaluate F(z^T) here (else
// the caller's seed contraction does it). Z may be NULL (the tape only).
int run_forward(const Run& r, const float* X, float lam, const float* alpha, const Sched& sc, float* Z, float* F,
                int f_trace, float* loss, bool want_final, float* seed_vout = nullptr, float seed_dF = 0.f) {
  const int N = r.N, T = r.T, mp = r.d->m_pad;
  int st;
  if ((st = prep(r, X)) != SLISTA_OK) return st;
  const bool want_f = (F != nullptr) || (loss != nullptr);
  if (T == 0) {
    if (Z) LAUNCH(kKOther, r.s, slista::launch_fill(Z, (size_t)N * r.d->m, 0.f, r.s));
    if (want_f) {
      LAUNCH(kKOther, r.s, slista::launch_reduce_f(r.xsq(), r.fpart(), 0, N, F, r.Fd(), r.s));
      if (loss) LAUNCH(kKOther, r.s, slista::launch_reduce_loss(r.Fd(), N, loss, r.s));
    }
    return SLISTA_OK;
  }
  if (use_persist(r, sc)) {
    Span sp[2];
    const int ns = spans_of(sc, sp);
    // without a tape, the iterate where the precision changes goes through
    // the (otherwise unused) iterate buffers of the layout
    float* handoff = (r.L.k == 0 && ns == 2) ? (float*)(r.ws + r.L.pp) : nullptr;
    for (int i = 0; i < ns; ++i) {
      const bool last = i == ns - 1;
      slista::PersistArgs a = persist_args(r, sp[i].prec, alpha, lam);
      a.t_begin = sp[i].t0;
      a.t_end = sp[i].t1;
      if (F && f_trace) {
        a.mode |= slista::kModeTrace;
        a.Ftrace = F;
      }
      if (last) {
        if (want_f && want_final) {
          a.mode |= slista::kModeF;
          a.F = F ? (f_trace ? F + (size_t)T * N : F) : nullptr;
          a.Fd = r.Fd();
        }
        a.Zuser = Z;
        if (seed_vout) {
          a.mode |= slista::kModeSeed;
          a.dF_scalar = seed_dF;
          a.Vout = seed_vout;
        }
        a.zload = i > 0 ? handoff : nullptr;
      } else {
        a.zsave = handoff;
      }
      LAUNCH(kKFwd, r.s,
             slista::launch_persist(true, sp[i].prec, a, r.s, variant_for(sp[i].prec, r.d->m_pad, r.N)));
    }
    if (loss && want_final) LAUNCH(kKOther, r.s, slista::launch_reduce_loss(r.Fd(), N, loss, r.s));
    return SLISTA_OK;
  }
  if (F && f_trace) LAUNCH(kKOther, r.s, slista::launch_reduce_f(r.xsq(), r.fpart(), 0, N, F, nullptr, r.s));
  LAUNCH(kKOther, r.s, slista::launch_layer0(r.C(), N, mp, alpha, lam, r.slot(1), r.s));
  for (int t = 1; t < T; ++t) {
    const bool tr = F && f_trace;
    if ((st = fwd_layer(r, sc.at(t), alpha, lam, t, tr ? r.fpart() : nullptr)) != SLISTA_OK) return st;
    if (tr) LAUNCH(kKOther, r.s, slista::launch_reduce_f(r.xsq(), r.fpart(), r.L.col_tiles, N, F + (size_t)t * N, nullptr, r.s));
  }
  if (Z) LAUNCH(kKOther, r.s, slista::launch_copy_out(r.slot(T), N, mp, r.d->m, Z, r.s));
  if (want_f && want_final) {
    slista::GemmArgs g = base_args(r, alpha, lam);
    g.A = r.slot(T);
    g.Bt = gram_for(*r.d, sc.at(T - 1));
    g.t = T - 1;
    g.Zt = r.slot(T);
    g.fpart = r.fpart();
    LAUNCH(kKFinal, r.s, slista::launch_gemm(sc.at(T - 1), slista::kEpiFinal, false, g, r.s));
    float* Fout = F ? (f_trace ? F + (size_t)T * N : F) : nullptr;
    LAUNCH(kKOther, r.s, slista::launch_reduce_f(r.xsq(), r.fpart(), r.L.col_tiles, N, Fout, r.Fd(), r.s));
    if (loss) LAUNCH(kKOther, r.s, slista::launch_reduce_loss(r.Fd(), N, loss, r.s));
  }
  return SLISTA_OK;
}

// Reverse pass over a workspace holding the forward tape. If seed_fpart, the
// seed contraction also produces F(z^T) (into F / loss). Layer t of the
// adjoint contracts in the precision of forward layer t.
int run_backward(const Run& r, float lam, const float* alpha, const Sched& sc, const float* dZ, const float* dF,
                 float dF_scalar, float* dalpha, bool seed_fpart, float* F, float* loss, bool seeded = false,
                 bool last_interior = true) {
  const int N = r.N, T = r.T, k = r.L.k;
  if (T == 0) return SLISTA_OK;
  int st;
  if (use_persist(r, sc)) {
    const int pT = sc.at(T - 1);
    if (!seeded) {
      slista::PersistArgs a = persist_args(r, pT, alpha, lam);
      a.t_begin = a.t_end = T;
      a.mode = slista::kModeSeed;
      a.dF = dF;
      a.dF_scalar = dF_scalar;
      a.dZ = dZ;
      a.Vout = r.vbuf(0);
      if (seed_fpart) {
        a.mode |= slista::kModeF;
        a.F = F;
        a.Fd = r.Fd();
      }
      LAUNCH(kKSeed, r.s, slista::launch_persist(true, pT, a, r.s, variant_for(pT, r.d->m_pad, r.N)));
      if (seed_fpart && loss) LAUNCH(kKOther, r.s, slista::launch_reduce_loss(r.Fd(), N, loss, r.s));
    }
    auto bwd = [&](int prec, int t_hi, int t_lo) -> int {
      slista::PersistArgs bw = persist_args(r, prec, alpha, lam);
      bw.t_hi = t_hi;
      bw.t_lo = t_lo;
      bw.Vio = r.vbuf(0);
      bw.dpart = r.dpart();
      LAUNCH(kKBwd, r.s, slista::launch_persist(false, prec, bw, r.s, variant_for(prec, r.d->m_pad, r.N)));
      return SLISTA_OK;
    };
    if (k == 1) {
      // every iterate kept: nothing is recomputed; one launch per precision span
      Span sp[2];
      const int ns = spans_of(sc, sp);
      for (int i = ns - 1; i >= 0; --i)
        if ((st = bwd(sp[i].prec, sp[i].t1 - 1, sp[i].t0)) != SLISTA_OK) return st;
    } else {
      // one recompute + one backward launch per segment (a segment never
      // straddles the first FP32 layer, which is a checkpoint)
      const int nseg = (T + k - 1) / k;
      for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int a0 = sgi * k;
        const int b = (a0 + k < T) ? a0 + k : T;
        const int prec = sc.at(a0);
        if ((sgi != nseg - 1 || !last_interior) && b - 1 > a0) {
          slista::PersistArgs f = persist_args(r, prec, alpha, lam);
          f.t_begin = a0;
          f.t_end = b - 1;
          f.store_all = 1;
          LAUNCH(kKFwd, r.s, slista::launch_persist(true, prec, f, r.s, variant_for(prec, r.d->m_pad, r.N)));
        }
        if ((st = bwd(prec, b - 1, a0)) != SLISTA_OK) return st;
      }
    }
    const int tiles_lo = persist_tiles(r, sc.at(0)), tiles_hi = persist_tiles(r, pT);
    LAUNCH(kKOther, r.s, slista::launch_reduce_dalpha(r.dpart(), T, r.L.P, tiles_lo, tiles_lo, alpha, dalpha, r.s,
                                                      sc.split(), tiles_hi));
    return SLISTA_OK;
  }
  {
    const int pT = sc.at(T - 1);
    slista::GemmArgs g = base_args(r, alpha, lam);
    g.A = r.slot(T);
    g.Bt = gram_for(*r.d, pT);
    g.t = T - 1;
    g.Zt = r.slot(T);
    g.Out = r.vbuf(T - 1);
    g.dF = dF;
    g.dF_scalar = dF_scalar;
    g.dZ = dZ;
    g.fpart = seed_fpart ? r.fpart() : nullptr;
    LAUNCH(kKSeed, r.s, slista::launch_gemm(pT, slista::kEpiSeed, false, g, r.s));
    if (seed_fpart) {
      LAUNCH(kKOther, r.s, slista::launch_reduce_f(r.xsq(), r.fpart(), r.L.col_tiles, N, F, r.Fd(), r.s));
      if (loss) LAUNCH(kKOther, r.s, slista::launch_reduce_loss(r.Fd(), N, loss, r.s));
    }
  }
  const int nseg = (T + k - 1) / k;
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const int a = sgi * k;
    const int b = (a + k < T) ? a + k : T;
    // Recompute the interior z^(a+1) .. z^(b-1) unless the forward left it.
    if (sgi != nseg - 1 || !last_interior) {
      for (int t = a + 1; t < b; ++t) {
        if (t == 1)
          LAUNCH(kKOther, r.s, slista::launch_layer0(r.C(), N, r.d->m_pad, alpha, lam, r.slot(1), r.s));
        else if ((st = fwd_layer(r, sc.at(t - 1), alpha, lam, t - 1, nullptr)) != SLISTA_OK)
          return st;
      }
    }
    for (int t = b - 1; t >= a; --t) {
      double* dp = r.dpart() + (size_t)t * r.L.P;
      if (t == 0) {
        LAUNCH(kKOther, r.s, slista::launch_bwd0(r.vbuf(0), r.slot(1), N, r.d->m_pad, dp, slista::bwd0_blocks(N, r.d->m_pad), r.s));
      } else {
        slista::GemmArgs g = base_args(r, alpha, lam);
        g.A = r.vbuf(t);
        g.Vin = r.vbuf(t);
        g.Bt = gram_for(*r.d, sc.at(t));
        g.t = t;
        g.Zt = r.slot(t);
        g.Zt1 = r.slot(t + 1);
        g.Out = r.vbuf(t - 1);
        g.dpart = dp;
        LAUNCH(kKBwd, r.s, slista::launch_gemm(sc.at(t), slista::kEpiBwd, false, g, r.s));
      }
    }
  }
  // Layer 0 wrote bwd0_blocks partials, every other layer one per tile.
  slista::GemmArgs g = base_args(r, alpha, lam);
  LAUNCH(kKOther, r.s, slista::launch_reduce_dalpha(r.dpart(), T, r.L.P, slista::bwd0_blocks(N, r.d->m_pad),
                                       g.row_tiles * g.col_tiles, alpha, dalpha, r.s));
  return SLISTA_OK;
}

// ------------------------------------------------------------- coupled LISTA
// Factored form of Eq. (11): per layer R^t = Z^t D^T - X (contraction over
// m_pad) then z^{t+1} = ST(z^t - alpha_t R^t W_t, lam beta_t) (contraction
// over n_pad). The adjoint runs Q = V W_t^T, v' = [z^t != 0](v - alpha_t Q D)
// and dW_t = -alpha_t (R^t)^T V, the last as a split contraction over sample
// chunks of chunk-major copies of R^t and V (FP32 in both precisions).
//
// Two kernel families. Persistent (default where the 32-sample tile fits in
// LDS): one forward and one backward launch for all layers; the tape holds
// R^t and v^t chunk-major and one code byte per element ([z^t != 0], sign
// z^{t+1}). Per-layer: two fused contractions per layer and direction; the
// tape holds z^0..z^T, R^0..R^T and v^0..v^{T-1} sample-major, transposed
// per layer group for the weight gradient. Both keep the operand copies of D
// and of the W stack and the padded samples.
struct ListaLayout {
  int n_pad = 0, m_pad = 0, ctn = 0, ctm = 0, Pa = 0, Pb = 0, S = 1, Kc = 0, Np = 0, opb = 4, Gl = 1, nwg = 0;
  bool tape = false, persist = false;
  size_t zbytes = 0, rbytes = 0;
  size_t Xp = 0, Dr = 0, DT = 0, Wr = 0, WT = 0, zs = 0, rs = 0, fres = 0, fl1 = 0, Fd = 0;
  size_t vb = 0, q = 0, dpa = 0, dpb = 0, RT = 0, VT = 0, wpart = 0, codes = 0, total = 0;
};

// The persistent kernels apply when their LDS tile fits and the per-layer
// family is not forced.
bool lista_persist_ok(int prec, int n_pad, int m_pad, int N, int T) {
  if (kernel_family() == 1 || N <= 0 || T <= 0) return false;
  return slista::lista_persist_lds(prec, true, n_pad, m_pad) <= slista::kListaMaxLds &&
         slista::lista_persist_lds(prec, false, n_pad, m_pad) <= slista::kListaMaxLds;
}

ListaLayout lista_layout(const slista::Dict& d, int N, int T, int prec, bool tape) {
  ListaLayout L;
  L.tape = tape;
  L.m_pad = d.m_pad;
  L.n_pad = (d.n + slista::kPadM - 1) / slista::kPadM * slista::kPadM;
  L.opb = prec == slista::kF32 ? 4 : 2;
  L.persist = lista_persist_ok(prec, L.n_pad, L.m_pad, N, T);
  L.zbytes = (size_t)N * L.m_pad * sizeof(float);
  L.rbytes = (size_t)N * L.n_pad * sizeof(float);
  const int row_tiles = (N + kTileRows - 1) / kTileRows;
  L.ctn = (L.n_pad + kTileCols - 1) / kTileCols;
  L.ctm = (L.m_pad + kTileCols - 1) / kTileCols;
  L.Pa = row_tiles * L.ctn;
  L.Pb = row_tiles * L.ctm;
  L.nwg = (N + slista::kListaRows - 1) / slista::kListaRows;
  // sample chunks of the weight-gradient contraction: enough workgroups to
  // fill the chip, at least ~256 samples (8 K steps) per chunk, Kc a
  // multiple of 64 (the transpose tile)
  const int wtiles = ((d.n + kTileRows - 1) / kTileRows) * ((d.m + kTileCols - 1) / kTileCols);
  int S = 512 / wtiles;
  const int by_n = (N + 255) / 256;
  if (S > by_n) S = by_n;
  if (S < 1) S = 1;
  const int per = (N + S - 1) / S;
  L.Kc = (per + 63) / 64 * 64;
  if (L.Kc < 64) L.Kc = 64;
  L.S = (N + L.Kc - 1) / L.Kc;
  if (L.S < 1) L.S = 1;
  L.Np = L.S * L.Kc;
  // layers per weight-gradient launch: about 1024 workgroups per launch
  const int per_layer = L.S * wtiles;
  L.Gl = (1024 + per_layer - 1) / per_layer;
  if (L.Gl > T) L.Gl = T;
  if (L.Gl < 1) L.Gl = 1;
  const size_t dmat = (size_t)L.n_pad * L.m_pad * L.opb;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes > 0 ? bytes : 1);
    return o;
  };
  L.Xp = take(L.rbytes);
  L.Dr = take(dmat);
  L.DT = take(dmat);
  L.Wr = take(dmat * (size_t)T);
  L.WT = take(dmat * (size_t)T);
  if (L.persist) {
    L.zs = take(L.zbytes);  // z^T
    L.rs = take(L.rbytes);  // R^T
    L.fres = take((size_t)N * sizeof(double));
    L.fl1 = take((size_t)N * sizeof(double));
    L.Fd = take((size_t)N * sizeof(double));
    if (tape) {
      L.RT = take((size_t)T * d.n * L.Np * sizeof(float));                       // R^t, chunk-major
      L.codes = take((size_t)T * L.nwg * (slista::kListaRows / 4) * L.m_pad * 4);  // mask / sign codes
      L.vb = take(L.zbytes);                                                     // v^{T-1} from the seed
      L.VT = take((size_t)T * d.m * L.Np * sizeof(float));                       // v^t, chunk-major
      L.dpa = take((size_t)T * L.nwg * sizeof(double));
      L.dpb = take((size_t)T * L.nwg * sizeof(double));
      L.wpart = take((size_t)L.Gl * L.S * d.n * d.m * sizeof(float));
    }
  } else {
    L.zs = take(L.zbytes * (tape ? (size_t)T + 1 : 2));
    L.rs = take(L.rbytes * (tape ? (size_t)T + 1 : 1));
    L.fres = take((size_t)L.ctn * N * sizeof(double));
    L.fl1 = take((size_t)L.ctm * N * sizeof(double));
    L.Fd = take((size_t)N * sizeof(double));
    if (tape) {
      L.vb = take(((size_t)T + 1) * L.zbytes);  // v^t for every layer (slot T: the unused v^{-1})
      L.q = take(L.rbytes);
      L.dpa = take((size_t)T * L.Pa * sizeof(double));
      L.dpb = take((size_t)T * L.Pb * sizeof(double));
      L.RT = take((size_t)L.Gl * d.n * L.Np * sizeof(float));
      L.VT = take((size_t)L.Gl * d.m * L.Np * sizeof(float));
      L.wpart = take((size_t)L.Gl * L.S * d.n * d.m * sizeof(float));
    }
  }
  L.total = off;
  return L;
}

struct ListaRun {
  const slista::Dict* d;
  ListaLayout L;
  char* ws;
  int N, T, prec;
  hipStream_t s;
  // per-layer family: z^t, R^t and v^t slots
  float* z(int t) const {
    const int slot = L.tape ? t : (t & 1);
    return (float*)(ws + L.zs + (size_t)slot * L.zbytes);
  }
  float* r(int t) const { return (float*)(ws + L.rs + (size_t)(L.tape ? t : 0) * L.rbytes); }
  float* v(int t) const { return (float*)(ws + L.vb + (size_t)(t >= 0 ? t : T) * L.zbytes); }
  // persistent family: z^T, R^T and the seed's v^{T-1}
  float* zT() const { return (float*)(ws + L.zs); }
  float* rT() const { return (float*)(ws + L.rs); }
  float* vseed() const { return (float*)(ws + L.vb); }
  const void* Wr(int t) const { return ws + L.Wr + (size_t)t * L.n_pad * L.m_pad * L.opb; }
  const void* WT(int t) const { return ws + L.WT + (size_t)t * L.n_pad * L.m_pad * L.opb; }
  float* Xp() const { return (float*)(ws + L.Xp); }
  double* fres() const { return (double*)(ws + L.fres); }
  double* fl1() const { return (double*)(ws + L.fl1); }
  double* Fd() const { return (double*)(ws + L.Fd); }
  float* RT() const { return (float*)(ws + L.RT); }
  float* VT() const { return (float*)(ws + L.VT); }
};

// Contraction with N sample rows: A [N][lda] times the K-contiguous operand Bt.
slista::GemmArgs lista_args(const ListaRun& r, const float* A, int lda, const void* Bt, int K, int ncols, float* Out) {
  slista::GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = A;
  g.lda = lda;
  g.Bt = Bt;
  g.ldb = K;
  g.K = K;
  g.rows = r.N;
  g.ncols = ncols;
  g.ldz = ncols;
  g.Out = Out;
  g.m = r.d->m;
  slista::gemm_grid(r.N, ncols, g);
  return g;
}

// R^t = Z^t D^T - X; fpart (may be NULL) gets 1/2 |R^t|^2 by column tile.
int lista_resid(const ListaRun& r, int t, double* fpart) {
  const ListaLayout& L = r.L;
  slista::GemmArgs g = lista_args(r, r.z(t), L.m_pad, r.ws + L.Dr, L.m_pad, L.n_pad, r.r(t));
  g.C = r.Xp();
  g.fpart = fpart;
  LAUNCH(kKFwd, r.s, slista::launch_gemm(r.prec, slista::kEpiResid, false, g, r.s));
  return SLISTA_OK;
}

slista::ListaPersistArgs lista_persist_args(const ListaRun& r, float lam, const float* alpha, const float* beta) {
  slista::ListaPersistArgs a;
  std::memset(&a, 0, sizeof a);
  a.N = r.N;
  a.n = r.d->n;
  a.m = r.d->m;
  a.n_pad = r.L.n_pad;
  a.m_pad = r.L.m_pad;
  a.T = r.T;
  a.Kc = r.L.Kc;
  a.Np = r.L.Np;
  a.Xp = r.Xp();
  a.Dr = r.ws + r.L.Dr;
  a.DT = r.ws + r.L.DT;
  a.Wr = r.ws + r.L.Wr;
  a.WT = r.ws + r.L.WT;
  a.alpha = alpha;
  a.beta = beta;
  a.lam = lam;
  a.nwg = r.L.nwg;
  if (r.L.tape) {
    a.rtape = r.RT();
    a.codes = (uint32_t*)(r.ws + r.L.codes);
    a.vseed = r.vseed();
    a.vtape = r.VT();
    a.dpa = (double*)(r.ws + r.L.dpa);
    a.dpb = (double*)(r.ws + r.L.dpb);
  }
  return a;
}

int lista_check(const slista_dict* dict, int N, int T, float lambda, int prec) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  if (T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "T=%d outside [0, %d]", T, kMaxT);
  if (!(lambda > 0.f) || !std::isfinite(lambda))
    return fail(SLISTA_EINVAL, "lambda=%g must be finite and > 0", (double)lambda);
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  return SLISTA_OK;
}

int lista_check_ws(const ListaLayout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(SLISTA_EINVAL, "workspace is NULL (%zu bytes needed)", L.total);
  if (((uintptr_t)ws & 255) != 0) return fail(SLISTA_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < L.total) return fail(SLISTA_EINVAL, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  return SLISTA_OK;
}

int lista_forward_run(const ListaRun& r, const float* X, float lam, const float* W, const float* alpha,
                      const float* beta, float* Z, float* F, float* loss) {
  const slista::Dict& d = *r.d;
  const ListaLayout& L = r.L;
  const int N = r.N, T = r.T;
  hipStream_t s = r.s;
  LAUNCH(kKOther, s, slista::launch_lista_pack(d.Dt, 1, d.n, d.m, d.n, 0, 1, L.n_pad, L.m_pad, r.prec, r.ws + L.Dr,
                                               r.ws + L.DT, s));
  if (T > 0)
    LAUNCH(kKOther, s, slista::launch_lista_pack(W, T, d.n, d.m, d.m, (size_t)d.n * d.m, 0, L.n_pad, L.m_pad, r.prec,
                                                 r.ws + L.Wr, r.ws + L.WT, s));
  LAUNCH(kKOther, s, slista::launch_pad_rows(X, N, d.n, L.n_pad, r.Xp(), s));
  const bool want_f = F || loss;
  int st;
  if (L.persist) {  // every layer, R^T and the objective partials in one launch
    slista::ListaPersistArgs pa = lista_persist_args(r, lam, alpha, beta);
    pa.zT = r.zT();
    pa.rT = (want_f || L.tape) ? r.rT() : nullptr;
    pa.fres = want_f ? r.fres() : nullptr;
    pa.fl1 = want_f ? r.fl1() : nullptr;
    if (L.tape)  // chunk rows past the last workgroup's tile stay zero
      LAUNCH(kKOther, s, slista::launch_zero_tape_rows(r.RT(), T, d.n, L.Kc, L.Np, L.nwg * slista::kListaRows, s));
    LAUNCH(kKFwd, s, slista::launch_lista_persist(r.prec, true, pa, s));
    LAUNCH(kKOther, s, slista::launch_copy_out(r.zT(), N, L.m_pad, d.m, Z, s));
    if (want_f) {
      LAUNCH(kKOther, s, slista::launch_lista_reduce_f(r.fres(), 1, r.fl1(), 1, N, F, r.Fd(), s));
      if (loss) LAUNCH(kKOther, s, slista::launch_reduce_loss(r.Fd(), N, loss, s));
    }
    return SLISTA_OK;
  }
  LAUNCH(kKOther, s, slista::launch_fill(r.z(0), (size_t)N * L.m_pad, 0.f, s));
  for (int t = 0; t < T; ++t) {
    if ((st = lista_resid(r, t, nullptr)) != SLISTA_OK) return st;
    slista::GemmArgs g = lista_args(r, r.r(t), L.n_pad, r.WT(t), L.n_pad, L.m_pad, r.z(t + 1));
    g.Zt = r.z(t);
    g.alpha = alpha;
    g.beta = beta;
    g.t = t;
    g.lam = lam;
    g.fpart = (want_f && t == T - 1) ? r.fl1() : nullptr;
    LAUNCH(kKFwd, s, slista::launch_gemm(r.prec, slista::kEpiLista, false, g, s));
  }
  // R^T: the residual term of F(z^T) and the backward seed's input
  if (want_f || L.tape)
    if ((st = lista_resid(r, T, want_f ? r.fres() : nullptr)) != SLISTA_OK) return st;
  LAUNCH(kKOther, s, slista::launch_copy_out(r.z(T), N, L.m_pad, d.m, Z, s));
  if (want_f) {
    LAUNCH(kKOther, s, slista::launch_lista_reduce_f(r.fres(), L.ctn, r.fl1(), T > 0 ? L.ctm : 0, N, F, r.Fd(), s));
    if (loss) LAUNCH(kKOther, s, slista::launch_reduce_loss(r.Fd(), N, loss, s));
  }
  return SLISTA_OK;
}

// dW_t = -alpha_t sum_i r_i v_i^T for g layers t0.. whose R^t and v^t are
// chunk-major at RT and VT ([g][Np / Kc][n or m][Kc]).
int lista_dw_group(const ListaRun& r, const float* RT, const float* VT, int g, const float* alpha, float* dW) {
  const slista::Dict& d = *r.d;
  const ListaLayout& L = r.L;
  slista::GemmArgs gw;
  std::memset(&gw, 0, sizeof gw);
  gw.A = RT;  // chunk s of layer b: [n][Kc] at RT + b n Np + s n Kc
  gw.lda = L.Kc;
  gw.Bt = VT;
  gw.ldb = L.Kc;
  gw.K = L.Kc;
  gw.rows = d.n;
  gw.ncols = d.m;
  gw.ldz = d.m;
  gw.Out = (float*)(r.ws + L.wpart);
  gw.ksplit = L.S;
  gw.nbatch = g;
  gw.a_split = (size_t)d.n * L.Kc;
  gw.b_split = (size_t)d.m * L.Kc;
  gw.a_batch = (size_t)d.n * L.Np;
  gw.b_batch = (size_t)d.m * L.Np;
  gw.out_split = (size_t)d.n * d.m;
  slista::gemm_grid(d.n, d.m, gw);
  LAUNCH(kKBwd, r.s, slista::launch_gemm(slista::kF32, slista::kEpiSplit, false, gw, r.s));
  LAUNCH(kKOther, r.s, slista::launch_lista_reduce_w(gw.Out, L.S, (size_t)d.n * d.m, alpha, g, dW, r.s));
  return SLISTA_OK;
}

int lista_backward_run(const ListaRun& r, float lam, const float* alpha, const float* dZ, const float* dF,
                       float dF_scalar, float* dW, float* dalpha, float* dbeta) {
  const slista::Dict& d = *r.d;
  const ListaLayout& L = r.L;
  const int N = r.N, T = r.T;
  hipStream_t s = r.s;
  if (T == 0) return SLISTA_OK;
  {  // seed v^{T-1} = [z^T != 0] (dF D^T R^T + dF lam sign z^T + dZ)
    float* vs = L.persist ? r.vseed() : r.v(T - 1);
    slista::GemmArgs g = lista_args(r, L.persist ? r.rT() : r.r(T), L.n_pad, r.ws + L.DT, L.n_pad, L.m_pad, vs);
    g.Zt = L.persist ? r.zT() : r.z(T);
    g.C = nullptr;
    g.dF = dF;
    g.dF_scalar = dF_scalar;
    g.dZ = dZ;
    g.lam = lam;
    LAUNCH(kKSeed, s, slista::launch_gemm(r.prec, slista::kEpiSeed, false, g, s));
  }
  double* dpa = (double*)(r.ws + L.dpa);
  double* dpb = (double*)(r.ws + L.dpb);
  int st;
  if (L.persist) {  // all layers back in one launch; R^t and v^t chunk-major on the tape
    slista::ListaPersistArgs pa = lista_persist_args(r, lam, alpha, nullptr);
    LAUNCH(kKOther, s, slista::launch_zero_tape_rows(r.VT(), T, d.m, L.Kc, L.Np, L.nwg * slista::kListaRows, s));
    LAUNCH(kKBwd, s, slista::launch_lista_persist(r.prec, false, pa, s));
    LAUNCH(kKOther, s, slista::launch_lista_reduce_ab(dpa, L.nwg, dpb, L.nwg, T, lam, dalpha, dbeta, s));
    for (int t0 = 0; dW && t0 < T; t0 += L.Gl) {
      const int g = T - t0 < L.Gl ? T - t0 : L.Gl;
      if ((st = lista_dw_group(r, r.RT() + (size_t)t0 * d.n * L.Np, r.VT() + (size_t)t0 * d.m * L.Np, g,
                               alpha + t0, dW + (size_t)t0 * d.n * d.m)) != SLISTA_OK)
        return st;
    }
    return SLISTA_OK;
  }
  float* q = (float*)(r.ws + L.q);
  for (int t = T - 1; t >= 0; --t) {
    const float* v = r.v(t);
    {  // Q = V W_t^T, dalpha_t partials against R^t
      slista::GemmArgs g = lista_args(r, v, L.m_pad, r.Wr(t), L.m_pad, L.n_pad, q);
      g.C = r.r(t);
      g.dpart = dpa + (size_t)t * L.Pa;
      LAUNCH(kKBwd, s, slista::launch_gemm(r.prec, slista::kEpiListaQ, false, g, s));
    }
    {  // v^{t-1} = [z^t != 0] (v^t - alpha_t Q D), dbeta_t partials
      slista::GemmArgs g = lista_args(r, q, L.n_pad, r.ws + L.DT, L.n_pad, L.m_pad, r.v(t - 1));
      g.Vin = v;
      g.Zt = r.z(t);
      g.Zt1 = r.z(t + 1);
      g.alpha = alpha;
      g.t = t;
      g.dpart = dpb + (size_t)t * L.Pb;
      LAUNCH(kKBwd, s, slista::launch_gemm(r.prec, slista::kEpiListaBwd, false, g, s));
    }
  }
  LAUNCH(kKOther, s, slista::launch_lista_reduce_ab(dpa, L.Pa, dpb, L.Pb, T, lam, dalpha, dbeta, s));
  // dW in layer groups: R^t and v^t transposed to chunk-major copies first
  for (int t0 = 0; dW && t0 < T; t0 += L.Gl) {
    const int g = T - t0 < L.Gl ? T - t0 : L.Gl;
    LAUNCH(kKOther, s, slista::launch_transpose_pad(r.r(t0), N, L.n_pad, d.n, L.Np, L.Kc, r.RT(), g,
                                                    L.rbytes / sizeof(float), (size_t)d.n * L.Np, s));
    LAUNCH(kKOther, s, slista::launch_transpose_pad(r.v(t0), N, L.m_pad, d.m, L.Np, L.Kc, r.VT(), g,
                                                    L.zbytes / sizeof(float), (size_t)d.m * L.Np, s));
    if ((st = lista_dw_group(r, r.RT(), r.VT(), g, alpha + t0, dW + (size_t)t0 * d.n * d.m)) != SLISTA_OK) return st;
  }
  return SLISTA_OK;
}

}  // namespace

// Static per-device scratch of slista_forward_scratch (for callers that cannot
// allocate device memory): the workspace of a forward pass without a tape.
// Each GPU the library runs on holds one copy of this array until the process
// ends. Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol): it uses the device address obtained with
// hipGetSymbolAddress once per device, with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up on the first
// call per device).
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SLISTA_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLISTA_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SLISTA_OK;
}

}  // namespace

extern "C" {

int slista_abi_version(void) { return SLISTA_ABI_VERSION; }

int slista_set_option(int option, int value) {
  if (option == SLISTA_OPT_KERNEL_FAMILY) {
    if (value < 0 || value > 2) return fail(SLISTA_EINVAL, "kernel family %d outside [0, 2]", value);
    g_kernel_family = value;
    return SLISTA_OK;
  }
  if (option == SLISTA_OPT_PERSIST_VARIANT) {
    if (value < 0 || value > slista::kPersistMaxVariant)
      return fail(SLISTA_EINVAL, "tile variant %d outside [0, %d]", value, slista::kPersistMaxVariant);
    g_persist_variant = value;
    return SLISTA_OK;
  }
  if (option == SLISTA_OPT_CHECK_FINITE) {
    if (value < 0 || value > 1) return fail(SLISTA_EINVAL, "check-finite flag %d outside [0, 1]", value);
    g_check_finite = value;
    return SLISTA_OK;
  }
  return fail(SLISTA_EINVAL, "unknown option %d", option);
}

int slista_profile_begin(void) {
  g_prof.on = true;
  g_prof.recs.clear();
  g_prof.dropped = 0;
  return SLISTA_OK;
}

int slista_profile_end(int* launches, double* total_ms, int* dropped) {
  if (!launches || !total_ms) return fail(SLISTA_EINVAL, "launches or total_ms is NULL");
  g_prof.on = false;
  for (int k = 0; k < SLISTA_PROFILE_KINDS; ++k) {
    launches[k] = 0;
    total_ms[k] = 0.0;
  }
  for (const auto& r : g_prof.recs) {
    HIP_TRY(hipEventSynchronize(g_prof.pool[r.second + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g_prof.pool[r.second], g_prof.pool[r.second + 1]));
    launches[r.first] += 1;
    total_ms[r.first] += ms;
  }
  if (dropped) *dropped = g_prof.dropped;
  g_prof.recs.clear();
  return SLISTA_OK;
}

const char* slista_status_string(int status) {
  switch (status) {
    case SLISTA_OK: return "ok";
    case SLISTA_EINVAL: return "invalid argument";
    case SLISTA_ENOMEM: return "device allocation failed";
    case SLISTA_EHIP: return "HIP runtime error";
    case SLISTA_ENOTSUP: return "not supported";
    case SLISTA_ENOTCONV: return "power iteration did not converge";
    case SLISTA_ENONFINITE: return "non-finite values (NaN or Inf) found by the finite-value check";
    default: return "unknown status";
  }
}

const char* slista_last_error(void) { return g_last_error.c_str(); }

int slista_dict_create(const float* D, int n, int m, void* stream, slista_dict** out) {
  if (!out) return fail(SLISTA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!D) return fail(SLISTA_EINVAL, "D is NULL");
  if (n < 1 || n > kMaxn) return fail(SLISTA_EINVAL, "n=%d outside [1, %d]", n, kMaxn);
  if (m < 1 || m > kMaxM) return fail(SLISTA_EINVAL, "m=%d outside [1, %d]", m, kMaxM);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SLISTA_ENOTSUP, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  hipStream_t s = (hipStream_t)stream;
  slista_dict* h = new (std::nothrow) slista_dict;
  if (!h) return fail(SLISTA_ENOMEM, "host allocation failed");
  slista::Dict& d = h->d;
  d.n = n;
  d.m = m;
  d.m_pad = (m + slista::kPadM - 1) / slista::kPadM * slista::kPadM;
  d.device = dev;
  d.G32 = nullptr;
  d.Gb = nullptr;
  d.Dt = nullptr;
  d.pwork = nullptr;
  d.Gsb = nullptr;
  d.Gsf = nullptr;
  d.flag = nullptr;
  const size_t mp = d.m_pad;
  bool ok = hipMalloc(&d.G32, mp * mp * sizeof(float)) == hipSuccess &&
            hipMalloc(&d.Gb, mp * mp * sizeof(uint16_t)) == hipSuccess &&
            hipMalloc(&d.Dt, mp * (size_t)n * sizeof(float)) == hipSuccess &&
            hipMalloc(&d.pwork, (2 * mp + 8) * sizeof(double)) == hipSuccess &&
            hipMalloc(&d.Gsb, mp * mp * sizeof(uint16_t)) == hipSuccess &&
            hipMalloc(&d.Gsf, mp * mp * sizeof(float)) == hipSuccess &&
            hipMalloc(&d.flag, 256) == hipSuccess;
  if (!ok) {
    (void)hipFree(d.G32);
    (void)hipFree(d.Gb);
    (void)hipFree(d.Dt);
    (void)hipFree(d.pwork);
    (void)hipFree(d.Gsb);
    (void)hipFree(d.Gsf);
    (void)hipFree(d.flag);
    delete h;
    (void)hipGetLastError();
    return fail(SLISTA_ENOMEM, "hipMalloc of the Gram matrices (m_pad=%d) failed", d.m_pad);
  }
  hipError_t e = slista::launch_gram(D, n, m, d.m_pad, d.G32, d.Gb, d.Dt, s);
  if (e == hipSuccess) e = slista::launch_swizzle(d.G32, d.m_pad, d.Gsb, d.Gsf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    slista_dict_destroy(h);
    return fail(SLISTA_EHIP, "Gram matrix: %s", hipGetErrorString(e));
  }
  const int cst = check_finite(d, s, {{D, (size_t)n * m}}, "D");
  if (cst != SLISTA_OK) {
    slista_dict_destroy(h);
    return cst;
  }
  *out = h;
  return SLISTA_OK;
}

int slista_dict_destroy(slista_dict* dict) {
  if (!dict) return SLISTA_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(dict->d.G32);
  (void)hipFree(dict->d.Gb);
  (void)hipFree(dict->d.Dt);
  (void)hipFree(dict->d.pwork);
  (void)hipFree(dict->d.Gsb);
  (void)hipFree(dict->d.Gsf);
  (void)hipFree(dict->d.flag);
  delete dict;
  return SLISTA_OK;
}

int slista_dict_dims(const slista_dict* dict, int* n, int* m, int* m_pad) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (n) *n = dict->d.n;
  if (m) *m = dict->d.m;
  if (m_pad) *m_pad = dict->d.m_pad;
  return SLISTA_OK;
}

int slista_dict_gram(const slista_dict* dict, float* G_out, void* stream) {
  if (!dict || !G_out) return fail(SLISTA_EINVAL, "dict or G_out is NULL");
  const slista::Dict& d = dict->d;
  HIP_TRY(hipMemcpy2DAsync(G_out, (size_t)d.m * sizeof(float), d.G32, (size_t)d.m_pad * sizeof(float),
                           (size_t)d.m * sizeof(float), d.m, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SLISTA_OK;
}

int slista_dict_lipschitz(slista_dict* dict, int max_iter, double rtol, double* L_out, int* iters,
                          void* stream) {
  if (!dict || !L_out) return fail(SLISTA_EINVAL, "dict or L_out is NULL");
  if (max_iter < 1 || max_iter > 10000000) return fail(SLISTA_EINVAL, "max_iter=%d outside [1, 1e7]", max_iter);
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(SLISTA_EINVAL, "rtol must be finite and >= 0");
  slista::Dict& d = dict->d;
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(kKOther, s, slista::launch_power_init(d.m, d.m_pad, d.pwork, s));
  // state: L, iterations, converged, previous quotient, zero vector
  double res[5] = {0, 0, 0, 0, 0};
  for (;;) {
    // a batch of iterations; launches after a stop condition return at once
    for (int b = 0; b < 32; ++b)
      LAUNCH(kKOther, s, slista::launch_power_step(d.G32, d.m, d.m_pad, max_iter, rtol, d.pwork, s));
    HIP_TRY(hipMemcpyAsync(res, d.pwork + 2 * (size_t)d.m_pad, sizeof res, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (res[2] != 0.0 || res[4] != 0.0 || res[1] >= (double)max_iter) break;
  }
  *L_out = res[0];
  if (iters) *iters = (int)res[1];
  if (res[2] == 0.0) return fail(SLISTA_ENOTCONV, "power iteration: %d iterations without rtol=%g", (int)res[1], rtol);
  return SLISTA_OK;
}

int slista_workspace_size(const slista_dict* dict, int N, int T, int prec, int ckpt_every, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 0 || N > kMaxN || T < 0 || T > kMaxT || ckpt_every < 0 || ckpt_every > kMaxT)
    return fail(SLISTA_EINVAL, "sizes out of range");
  Sched sc;
  const int st = parse_sched(prec, T, ckpt_every, &sc);
  if (st != SLISTA_OK) return st;
  *bytes = make_layout(dict->d, N, T, ckpt_every).total;
  return SLISTA_OK;
}

int slista_ckpt_for_budget(const slista_dict* dict, int N, int T, int prec, size_t budget, int* ckpt_every,
                           size_t* bytes) {
  if (!dict || !ckpt_every) return fail(SLISTA_EINVAL, "dict or ckpt_every is NULL");
  if (N < 0 || N > kMaxN || T < 1 || T > kMaxT) return fail(SLISTA_EINVAL, "sizes out of range");
  Sched sc;
  const int st = parse_sched(prec, T, 1, &sc);
  if (st != SLISTA_OK) return st;
  // the workspace shrinks with k until the segment buffers outgrow the
  // checkpoints (around sqrt(T)); the smallest fitting k recomputes least
  size_t best_bytes = (size_t)-1;
  for (int k = 1; k <= T; ++k) {
    const size_t b = make_layout(dict->d, N, T, k).total;
    if (b <= budget) {
      *ckpt_every = k;
      if (bytes) *bytes = b;
      return SLISTA_OK;
    }
    if (b < best_bytes) best_bytes = b;
  }
  return fail(SLISTA_ENOMEM, "no checkpoint spacing fits %zu bytes (smallest workspace %zu bytes)", budget,
              best_bytes);
}

int slista_forward(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha, int T,
                   int prec, float* Z, float* F, int f_trace, float* loss, int ckpt_every, void* ws,
                   size_t ws_bytes, void* stream) {
  size_t need = 0;
  Sched sc;
  int st = check_common(dict, X, N, lambda, alpha, T, prec, ckpt_every, ws, ws_bytes, &need, &sc);
  if (st != SLISTA_OK) return st;
  if (N > 0 && !Z) return fail(SLISTA_EINVAL, "Z is NULL");
  hipStream_t s = (hipStream_t)stream;
  tape_forget(ws, need);
  if (loss && N == 0) {
    LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    return SLISTA_OK;
  }
  if (N == 0) return SLISTA_OK;
  const slista::Dict& d = dict->d;
  if ((st = check_finite(d, s, {{X, (size_t)N * d.n}, {alpha, (size_t)T}}, "the inputs X, alpha")) != SLISTA_OK)
    return st;
  Run r{&d, make_layout(d, N, T, ckpt_every), (char*)ws, N, T, s};
  if ((st = run_forward(r, X, lambda, alpha, sc, Z, F, f_trace, loss, true)) != SLISTA_OK) return st;
  if (ckpt_every >= 1) tape_record(ws, need, tape_tag(r, X, lambda, alpha, prec), true);
  const size_t nF = F ? (f_trace ? (size_t)(T + 1) * N : (size_t)N) : 0;
  return check_finite(d, s, {{Z, (size_t)N * d.m}, {F, nF}, {loss, loss ? 1u : 0u}}, "the outputs Z, F, loss");
}

int slista_forward_scratch(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha,
                           int T, int prec, float* Z, float* F, int f_trace, float* loss, void* stream) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (g_prof.on) return fail(SLISTA_EINVAL, "kernel timing creates HIP events; switch it off for this entry point");
  if (N < 0 || N > kMaxN || T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "N=%d or T=%d out of range", N, T);
  const size_t need = make_layout(dict->d, N, T, 0).total;
  if (need > kScratchBytes)
    return fail(SLISTA_EINVAL, "N=%d, m_pad=%d needs %zu bytes of scratch; the static scratch holds %zu bytes", N,
                dict->d.m_pad, need, kScratchBytes);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != dict->d.device)
    return fail(SLISTA_EINVAL, "the current device (%d) is not the dictionary's (%d)", dev, dict->d.device);
  void* ws = nullptr;
  const int st = scratch_ptr(dev, &ws);
  if (st != SLISTA_OK) return st;
  return slista_forward(dict, X, N, lambda, alpha, T, prec, Z, F, f_trace, loss, 0, ws, kScratchBytes, stream);
}

int slista_objective(const slista_dict* dict, const float* X, int N, float lambda, const float* Z, float* F,
                     void* stream) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  if (!(lambda >= 0.f) || !std::isfinite(lambda)) return fail(SLISTA_EINVAL, "lambda must be finite and >= 0");
  if (N > 0 && (!X || !Z || !F)) return fail(SLISTA_EINVAL, "X, Z or F is NULL");
  if (dict->d.n > 512) return fail(SLISTA_ENOTSUP, "slista_objective supports n <= 512 (n=%d)", dict->d.n);
  LAUNCH(kKOther, (hipStream_t)stream,
         slista::launch_objective(X, dict->d.Dt, N, dict->d.n, dict->d.m, lambda, Z, F, (hipStream_t)stream));
  return SLISTA_OK;
}

int slista_forward_f64_workspace_size(const slista_dict* dict, int N, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  *bytes = align256((size_t)N * sizeof(double));
  return SLISTA_OK;
}

int slista_forward_f64(const slista_dict* dict, const double* X, int N, double lambda, const double* alpha, int T,
                       double* Z, double* F, int f_trace, double* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  if (T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "T=%d outside [0, %d]", T, kMaxT);
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(SLISTA_EINVAL, "lambda must be finite and > 0");
  if (N > 0 && (!X || !Z)) return fail(SLISTA_EINVAL, "X or Z is NULL");
  if (T > 0 && !alpha) return fail(SLISTA_EINVAL, "alpha is NULL");
  if (f_trace && !F) return fail(SLISTA_EINVAL, "f_trace needs F");
  const slista::Dict& d = dict->d;
  if (d.n > slista::f64_max_n())
    return fail(SLISTA_ENOTSUP, "the FP64 forward supports n <= %d (n=%d)", slista::f64_max_n(), d.n);
  hipStream_t s = (hipStream_t)stream;
  // the per-sample objectives the loss averages: F itself, the trace's last
  // row, or the workspace
  double* Fd = nullptr;
  if (loss) {
    if (F) {
      Fd = f_trace ? F + (size_t)T * N : F;
    } else if (N > 0) {
      if (!ws || ((uintptr_t)ws & 255) || ws_bytes < (size_t)N * sizeof(double))
        return fail(SLISTA_EINVAL, "the loss without F needs a 256-byte aligned workspace of %zu bytes",
                    align256((size_t)N * sizeof(double)));
      Fd = (double*)ws;
    }
  }
  if (slista::ista_f64_lds(d.n, d.m_pad) > 160 * 1024)
    return fail(SLISTA_ENOTSUP, "the FP64 forward's per-wave iterate does not fit in LDS (m_pad=%d)", d.m_pad);
  LAUNCH(kKFwd, s, slista::launch_ista_f64(d.Dt, d.n, d.m, d.m_pad, X, N, lambda, alpha, T, Z, F, f_trace, Fd, s));
  if (loss) LAUNCH(kKOther, s, slista::launch_mean_d(Fd, N, loss, s));
  return SLISTA_OK;
}

int slista_backward(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha, int T,
                    int prec, const float* dZ, const float* dF, float* dalpha, int ckpt_every, void* ws,
                    size_t ws_bytes, void* stream) {
  size_t need = 0;
  Sched sc;
  int st = check_common(dict, X, N, lambda, alpha, T, prec, ckpt_every, ws, ws_bytes, &need, &sc);
  if (st != SLISTA_OK) return st;
  if (ckpt_every < 1) return fail(SLISTA_EINVAL, "backward needs ckpt_every >= 1 (its tape)");
  if (!dZ && !dF) return fail(SLISTA_EINVAL, "dZ and dF are both NULL");
  if (T > 0 && !dalpha) return fail(SLISTA_EINVAL, "dalpha is NULL");
  if (T == 0) return SLISTA_OK;
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    LAUNCH(kKOther, s, slista::launch_fill(dalpha, T, 0.f, s));
    return SLISTA_OK;
  }
  const slista::Dict& d = dict->d;
  if ((st = check_finite(d, s, {{X, (size_t)N * d.n}, {alpha, (size_t)T}, {dZ, dZ ? (size_t)N * d.m : 0},
                                {dF, dF ? (size_t)N : 0}},
                         "the inputs X, alpha, dZ, dF")) != SLISTA_OK)
    return st;
  Run r{&d, make_layout(d, N, T, ckpt_every), (char*)ws, N, T, s};
  const TapeTag tag = tape_tag(r, X, lambda, alpha, prec);
  int state = tape_state(ws, tag);
  if (state == 0) {
    // no tape of a forward with these arguments in ws: keep one now
    if ((st = run_forward(r, X, lambda, alpha, sc, nullptr, nullptr, 0, nullptr, false)) != SLISTA_OK) return st;
    state = 2;
  }
  if ((st = run_backward(r, lambda, alpha, sc, dZ, dF, 0.f, dalpha, false, nullptr, nullptr, false, state == 2)) !=
      SLISTA_OK)
    return st;
  tape_record(ws, need, tag, state == 2 && backward_keeps_interior(r.L, T));
  return check_finite(d, s, {{dalpha, (size_t)T}}, "the output dalpha");
}

int slista_forward_backward(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha,
                            int T, int prec, float* Z, float* F, float* loss, float* dalpha, int ckpt_every,
                            void* ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  Sched sc;
  int st = check_common(dict, X, N, lambda, alpha, T, prec, ckpt_every, ws, ws_bytes, &need, &sc);
  if (st != SLISTA_OK) return st;
  if (ckpt_every < 1) return fail(SLISTA_EINVAL, "forward_backward needs ckpt_every >= 1");
  if (N > 0 && !Z) return fail(SLISTA_EINVAL, "Z is NULL");
  if (T > 0 && !dalpha) return fail(SLISTA_EINVAL, "dalpha is NULL");
  hipStream_t s = (hipStream_t)stream;
  tape_forget(ws, need);
  if (N == 0) {
    if (T > 0) LAUNCH(kKOther, s, slista::launch_fill(dalpha, T, 0.f, s));
    if (loss) LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    return SLISTA_OK;
  }
  const slista::Dict& d = dict->d;
  if ((st = check_finite(d, s, {{X, (size_t)N * d.n}, {alpha, (size_t)T}}, "the inputs X, alpha")) != SLISTA_OK)
    return st;
  Run r{&d, make_layout(d, N, T, ckpt_every), (char*)ws, N, T, s};
  if (T == 0) {
    if ((st = run_forward(r, X, lambda, alpha, sc, Z, F, 0, loss, true)) != SLISTA_OK) return st;
  } else if (use_persist(r, sc)) {
    // one persistent launch runs the forward, F(z^T) and the seed of the mean loss
    if ((st = run_forward(r, X, lambda, alpha, sc, Z, F, 0, loss, true, r.vbuf(0), (float)(1.0 / N))) != SLISTA_OK)
      return st;
    if ((st = run_backward(r, lambda, alpha, sc, nullptr, nullptr, 0.f, dalpha, false, nullptr, nullptr, true)) !=
        SLISTA_OK)
      return st;
  } else {
    if ((st = run_forward(r, X, lambda, alpha, sc, Z, nullptr, 0, nullptr, false)) != SLISTA_OK) return st;
    if ((st = run_backward(r, lambda, alpha, sc, nullptr, nullptr, (float)(1.0 / N), dalpha, F || loss, F, loss)) !=
        SLISTA_OK)
      return st;
  }
  tape_record(ws, need, tape_tag(r, X, lambda, alpha, prec), backward_keeps_interior(r.L, T));
  return check_finite(d, s, {{Z, (size_t)N * d.m}, {F, F ? (size_t)N : 0}, {loss, loss ? 1u : 0u},
                             {dalpha, (size_t)T}},
                      "the outputs Z, F, loss, dalpha");
}

// ------------------------------------------------------------- FISTA
// Workspace of slista_fista: the forward workspace without a tape (C, norms,
// objective partials, two z buffers), two y buffers and the momentum weights.
static size_t fista_offsets(const slista::Dict& d, int N, int T, size_t off[2]) {
  const Layout L = make_layout(d, N, T, 0, false);
  size_t o = align256(L.total);
  off[0] = o;  // y buffers
  o += 2 * align256(L.zbytes);
  off[1] = o;  // beta [T]
  o += align256((size_t)(T > 0 ? T : 1) * sizeof(float));
  return o;
}

int slista_fista_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 0 || N > kMaxN || T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "sizes out of range");
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  size_t off[2];
  *bytes = fista_offsets(dict->d, N, T, off);
  return SLISTA_OK;
}

int slista_fista(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha, int T, int prec,
                 float* Z, float* F, float* loss, void* ws, size_t ws_bytes, void* stream) {
  size_t need_fwd = 0;
  int st = check_common(dict, X, N, lambda, alpha, T, prec, 0, ws, ws_bytes, &need_fwd);
  if (st != SLISTA_OK) return st;
  size_t off[2];
  const size_t need = fista_offsets(dict->d, N, T, off);
  if (ws_bytes < need) return fail(SLISTA_EINVAL, "workspace must hold %zu bytes", need);
  tape_forget(ws, need);
  if (N > 0 && !Z) return fail(SLISTA_EINVAL, "Z is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    if (loss) LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    return SLISTA_OK;
  }
  const Run r{&dict->d, make_layout(dict->d, N, T, 0, false), (char*)ws, N, T, s};
  const int mp = dict->d.m_pad;
  if (T == 0) return run_forward(r, X, lambda, alpha, Sched{prec, 0, 0}, Z, F, 0, loss, true);  // Z = 0, F = |x|^2 / 2
  if ((st = prep(r, X)) != SLISTA_OK) return st;
  float* ybuf[2] = {(float*)((char*)ws + off[0]), (float*)((char*)ws + off[0] + align256(r.L.zbytes))};
  float* beta = (float*)((char*)ws + off[1]);
  LAUNCH(kKOther, s, slista::launch_fista_beta(T, beta, s));
  if (kernel_family() != 1 && slista::fista_persist_applies(mp)) {
    // one persistent launch: each tile carries z and y through all layers;
    // the first y buffer holds the row-group copy of c it reads
    float* Cg = ybuf[0];
    LAUNCH(kKOther, s, slista::launch_row_groups(r.C(), N, mp, Cg, s));
    slista::PersistArgs a = persist_args(r, prec, alpha, lambda);
    a.Cg = Cg;
    a.beta = beta;
    a.k = 0;
    a.t_begin = 0;
    a.t_end = T;
    a.mode = (F || loss) ? slista::kModeF : 0;
    a.F = F;
    a.Fd = r.Fd();
    a.Zuser = Z;
    LAUNCH(kKFwd, s, slista::launch_fista_persist(prec, a, s, variant_for(prec, mp, N)));
    if (loss) LAUNCH(kKOther, s, slista::launch_reduce_loss(r.Fd(), N, loss, s));
    return SLISTA_OK;
  }
  // layer 0: y^0 = z^0 = 0, so z^1 = ST(alpha_0 c, lam alpha_0) and y^1 = z^1 (beta_0 = 0)
  LAUNCH(kKOther, s, slista::launch_layer0(r.C(), N, mp, alpha, lambda, r.slot(1), s));
  const float* y = r.slot(1);
  for (int t = 1; t < T; ++t) {
    slista::GemmArgs g = base_args(r, alpha, lambda);
    g.A = y;
    g.Bt = gram_for(*r.d, prec);
    g.t = t;
    g.Zt = y;
    g.Zt1 = r.slot(t);
    g.Out = r.slot(t + 1);
    g.Out2 = ybuf[(t + 1) & 1];
    g.beta = beta;
    LAUNCH(kKFwd, s, slista::launch_gemm(prec, slista::kEpiFista, false, g, s));
    y = g.Out2;
  }
  LAUNCH(kKOther, s, slista::launch_copy_out(r.slot(T), N, mp, dict->d.m, Z, s));
  if (F || loss) {
    slista::GemmArgs g = base_args(r, alpha, lambda);
    g.A = r.slot(T);
    g.Bt = gram_for(*r.d, prec);
    g.t = T - 1;
    g.Zt = r.slot(T);
    g.fpart = r.fpart();
    LAUNCH(kKFinal, s, slista::launch_gemm(prec, slista::kEpiFinal, false, g, s));
    LAUNCH(kKOther, s, slista::launch_reduce_f(r.xsq(), r.fpart(), r.L.col_tiles, N, F, r.Fd(), s));
    if (loss) LAUNCH(kKOther, s, slista::launch_reduce_loss(r.Fd(), N, loss, s));
  }
  return SLISTA_OK;
}

// ------------------------------------------------------------- Oracle-ISTA
// Workspace of slista_oista: the forward workspace without a tape (C, norms,
// objective partials reused as violation counts, two z buffers), the
// gradient R [N, m_pad], the warm-start vectors V [N, m_pad], the steps [N].
static size_t oista_offsets(const slista::Dict& d, int N, int T, size_t off[3]) {
  const Layout L = make_layout(d, N, T, 0, false);
  size_t o = align256(L.total);
  off[0] = o;  // R
  o += align256(L.zbytes);
  off[1] = o;  // V
  o += align256(L.zbytes);
  off[2] = o;  // step
  o += align256((size_t)(N > 0 ? N : 1) * sizeof(float));
  return o;
}

int slista_oista_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 0 || N > kMaxN || T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "sizes out of range");
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  size_t off[3];
  *bytes = oista_offsets(dict->d, N, T, off);
  return SLISTA_OK;
}

int slista_oista(const slista_dict* dict, const float* X, int N, float lambda, double L, int T, int prec,
                 int max_power_iter, double power_rtol, float* Z, float* F, float* loss, float* steps, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (!(L > 0.0) || !std::isfinite(L)) return fail(SLISTA_EINVAL, "L must be finite and > 0");
  if (max_power_iter < 1 || max_power_iter > 1000000) return fail(SLISTA_EINVAL, "max_power_iter outside [1, 1e6]");
  if (!(power_rtol >= 0.0) || !std::isfinite(power_rtol)) return fail(SLISTA_EINVAL, "power_rtol must be >= 0");
  if (dict->d.m_pad > 2048) return fail(SLISTA_ENOTSUP, "Oracle-ISTA supports m <= 2048 (m_pad=%d)", dict->d.m_pad);
  if (slista::support_lipschitz_lds(dict->d.m_pad, dict->d.n) > 160 * 1024)
    return fail(SLISTA_ENOTSUP, "Oracle-ISTA's per-sample Lanczos does not fit in LDS (n=%d)", dict->d.n);
  if (T < 0 || T > kMaxT) return fail(SLISTA_EINVAL, "T=%d outside [0, %d]", T, kMaxT);
  size_t need_fwd = 0;  // checks N, lambda, prec, X and the workspace alignment (no step sizes here)
  int st = check_common(dict, X, N, lambda, nullptr, 0, prec, 0, ws, ws_bytes, &need_fwd);
  if (st != SLISTA_OK) return st;
  size_t off[3];
  const size_t need = oista_offsets(dict->d, N, T, off);
  if (ws_bytes < need) return fail(SLISTA_EINVAL, "workspace must hold %zu bytes", need);
  tape_forget(ws, need);
  if (N > 0 && !Z) return fail(SLISTA_EINVAL, "Z is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    if (loss) LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    return SLISTA_OK;
  }
  const Run r{&dict->d, make_layout(dict->d, N, T, 0, false), (char*)ws, N, T, s};
  if (T == 0) return run_forward(r, X, lambda, nullptr, Sched{prec, 0, 0}, Z, F, 0, loss, true);
  const int mp = dict->d.m_pad;
  float* R = (float*)((char*)ws + off[0]);
  float* V = (float*)((char*)ws + off[1]);
  float* step = (float*)((char*)ws + off[2]);
  if ((st = prep(r, X)) != SLISTA_OK) return st;
  LAUNCH(kKOther, s, slista::launch_fill(V, (size_t)N * mp, 0.f, s));
  // z^0 = 0: its support is empty, so layer 0 is the ISTA step from 0
  LAUNCH(kKOther, s, slista::launch_fill(r.slot(0), (size_t)N * mp, 0.f, s));
  for (int t = 0; t < T; ++t) {
    const float* zt = r.slot(t);
    LAUNCH(kKOther, s, slista::launch_support_lipschitz(dict->d.G32, dict->d.Dt, dict->d.n, dict->d.m, mp, zt, V, L,
                                                        max_power_iter, power_rtol, N, step, s));
    slista::GemmArgs g = base_args(r, nullptr, lambda);
    g.A = zt;
    g.Bt = gram_for(*r.d, prec);
    g.Zt = zt;
    g.Out = R;
    g.fpart = r.fpart();
    LAUNCH(kKFwd, s, slista::launch_gemm(prec, slista::kEpiGrad, false, g, s));
    LAUNCH(kKOther, s, slista::launch_oista_update(zt, R, r.fpart(), r.L.col_tiles, step, L, lambda, N, mp,
                                                   r.slot(t + 1), steps ? steps + (size_t)t * N : nullptr, s));
  }
  LAUNCH(kKOther, s, slista::launch_copy_out(r.slot(T), N, mp, dict->d.m, Z, s));
  if (F || loss) {
    slista::GemmArgs g = base_args(r, nullptr, lambda);
    g.A = r.slot(T);
    g.Bt = gram_for(*r.d, prec);
    g.Zt = r.slot(T);
    g.fpart = r.fpart();
    LAUNCH(kKFinal, s, slista::launch_gemm(prec, slista::kEpiFinal, false, g, s));
    LAUNCH(kKOther, s, slista::launch_reduce_f(r.xsq(), r.fpart(), r.L.col_tiles, N, F, r.Fd(), s));
    if (loss) LAUNCH(kKOther, s, slista::launch_reduce_loss(r.Fd(), N, loss, s));
  }
  return SLISTA_OK;
}

int slista_lista_workspace_size(const slista_dict* dict, int N, int T, int prec, int tape, size_t* bytes) {
  if (!bytes) return fail(SLISTA_EINVAL, "bytes is NULL");
  int st = lista_check(dict, N, T, 1.f, prec);
  if (st != SLISTA_OK) return st;
  *bytes = lista_layout(dict->d, N, T, prec, tape != 0).total;
  return SLISTA_OK;
}

int slista_lista_forward(const slista_dict* dict, const float* X, int N, float lambda, const float* W,
                         const float* alpha, const float* beta, int T, int prec, float* Z, float* F, float* loss,
                         int tape, void* ws, size_t ws_bytes, void* stream) {
  int st = lista_check(dict, N, T, lambda, prec);
  if (st != SLISTA_OK) return st;
  if (N > 0 && (!X || !Z)) return fail(SLISTA_EINVAL, "X or Z is NULL");
  if (T > 0 && (!W || !alpha || !beta)) return fail(SLISTA_EINVAL, "W, alpha or beta is NULL");
  const ListaLayout L = lista_layout(dict->d, N, T, prec, tape != 0);
  if ((st = lista_check_ws(L, ws, ws_bytes)) != SLISTA_OK) return st;
  tape_forget(ws, L.total);
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    if (loss) LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    return SLISTA_OK;
  }
  const ListaRun r{&dict->d, L, (char*)ws, N, T, prec, s};
  return lista_forward_run(r, X, lambda, W, alpha, beta, Z, F, loss);
}

int slista_lista_backward(const slista_dict* dict, int N, float lambda, const float* alpha, const float* beta, int T,
                          int prec, const float* dZ, const float* dF, float* dW, float* dalpha, float* dbeta,
                          void* ws, size_t ws_bytes, void* stream) {
  int st = lista_check(dict, N, T, lambda, prec);
  if (st != SLISTA_OK) return st;
  if (!dZ && !dF) return fail(SLISTA_EINVAL, "dZ and dF are both NULL");
  if (T > 0 && (!alpha || !beta || !dalpha || !dbeta)) return fail(SLISTA_EINVAL, "alpha, beta, dalpha or dbeta is NULL");
  const ListaLayout L = lista_layout(dict->d, N, T, prec, true);
  if ((st = lista_check_ws(L, ws, ws_bytes)) != SLISTA_OK) return st;
  tape_forget(ws, L.total);
  hipStream_t s = (hipStream_t)stream;
  if (N == 0 || T == 0) {
    if (T > 0) {
      LAUNCH(kKOther, s, slista::launch_fill(dalpha, T, 0.f, s));
      LAUNCH(kKOther, s, slista::launch_fill(dbeta, T, 0.f, s));
      if (dW) LAUNCH(kKOther, s, slista::launch_fill(dW, (size_t)T * dict->d.n * dict->d.m, 0.f, s));
    }
    return SLISTA_OK;
  }
  const ListaRun r{&dict->d, L, (char*)ws, N, T, prec, s};
  return lista_backward_run(r, lambda, alpha, dZ, dF, 0.f, dW, dalpha, dbeta);
}

int slista_lista_forward_backward(const slista_dict* dict, const float* X, int N, float lambda, const float* W,
                                  const float* alpha, const float* beta, int T, int prec, float* Z, float* F,
                                  float* loss, float* dW, float* dalpha, float* dbeta, void* ws, size_t ws_bytes,
                                  void* stream) {
  int st = lista_check(dict, N, T, lambda, prec);
  if (st != SLISTA_OK) return st;
  if (N > 0 && (!X || !Z)) return fail(SLISTA_EINVAL, "X or Z is NULL");
  if (T > 0 && (!W || !alpha || !beta || !dalpha || !dbeta))
    return fail(SLISTA_EINVAL, "W, alpha, beta, dalpha or dbeta is NULL");
  const ListaLayout L = lista_layout(dict->d, N, T, prec, true);
  if ((st = lista_check_ws(L, ws, ws_bytes)) != SLISTA_OK) return st;
  tape_forget(ws, L.total);
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    if (loss) LAUNCH(kKOther, s, slista::launch_fill(loss, 1, 0.f, s));
    if (T > 0) {
      LAUNCH(kKOther, s, slista::launch_fill(dalpha, T, 0.f, s));
      LAUNCH(kKOther, s, slista::launch_fill(dbeta, T, 0.f, s));
      if (dW) LAUNCH(kKOther, s, slista::launch_fill(dW, (size_t)T * dict->d.n * dict->d.m, 0.f, s));
    }
    return SLISTA_OK;
  }
  const ListaRun r{&dict->d, L, (char*)ws, N, T, prec, s};
  if ((st = lista_forward_run(r, X, lambda, W, alpha, beta, Z, F, loss)) != SLISTA_OK) return st;
  return lista_backward_run(r, lambda, alpha, nullptr, nullptr, (float)(1.0 / N), dW, dalpha, dbeta);
}

// ------------------------------------------------------------- training
// Workspace of slista_train: the forward/backward workspace with the full
// tape, then the gradient [T], the candidate steps [T], the FP64 loss and
// the loss weights dF = 1/N [N], each 256-byte aligned.
static size_t train_extra_offsets(const slista::Dict& d, int N, int T, size_t off[4]) {
  size_t o = align256(make_layout(d, N, T, 1).total);
  off[0] = o;
  o += align256((size_t)T * sizeof(float));
  off[1] = o;
  o += align256((size_t)T * sizeof(float));
  off[2] = o;
  o += align256(sizeof(double));
  off[3] = o;
  o += align256((size_t)N * sizeof(float));
  return o;
}

int slista_train_workspace_size(const slista_dict* dict, int N, int T, int prec, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 1 || N > kMaxN || T < 1 || T > kMaxT) return fail(SLISTA_EINVAL, "training needs 1 <= N, 1 <= T");
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  size_t off[4];
  *bytes = train_extra_offsets(dict->d, N, T, off);
  return SLISTA_OK;
}

int slista_train(const slista_dict* dict, const float* X, int N, float lambda, float* alpha, int T, int prec,
                 int iters, double lr, int max_halvings, float* Z, double* losses, int* accepted, double* lr_out,
                 void* ws, size_t ws_bytes, void* stream) {
  if (!dict || !X || !alpha || !Z || !ws) return fail(SLISTA_EINVAL, "dict, X, alpha, Z or ws is NULL");
  if (N < 1 || N > kMaxN || T < 1 || T > kMaxT) return fail(SLISTA_EINVAL, "training needs 1 <= N, 1 <= T");
  if (iters < 0 || max_halvings < 0 || max_halvings > 1000)
    return fail(SLISTA_EINVAL, "iters >= 0 and 0 <= max_halvings <= 1000 required");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(SLISTA_EINVAL, "lr must be finite and > 0");
  if (g_prof.on) return fail(SLISTA_EINVAL, "kernel timing must be off while training");
  size_t off[4];
  const size_t need = train_extra_offsets(dict->d, N, T, off);
  if (((uintptr_t)ws & 255) || ws_bytes < need)
    return fail(SLISTA_EINVAL, "workspace must be 256-byte aligned with %zu bytes", need);
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "unknown precision %d", prec);
  tape_forget(ws, need);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t main_bytes = off[0];
  float* g = (float*)(w + off[0]);
  float* cand = (float*)(w + off[1]);
  double* Jd = (double*)(w + off[2]);
  float* dF = (float*)(w + off[3]);
  const Run r{&dict->d, make_layout(dict->d, N, T, 1), w, N, T, s};
  int st;
  LAUNCH(kKOther, s, slista::launch_fill(dF, (size_t)N, (float)(1.0 / N), s));
  // loss and gradient at the starting steps
  if ((st = slista_forward_backward(dict, X, N, lambda, alpha, T, prec, Z, nullptr, (float*)Jd, g, 1, ws,
                                    main_bytes, stream)) != SLISTA_OK)
    return st;
  auto loss_now = [&](double* out) -> int {
    LAUNCH(kKOther, s, slista::launch_mean_d(r.Fd(), N, Jd, s));
    HIP_TRY(hipMemcpyAsync(out, Jd, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SLISTA_OK;
  };
  double J = 0.0;
  if ((st = loss_now(&J)) != SLISTA_OK) return st;
  if (losses) losses[0] = J;
  double eta = lr;
  int acc = 0;
  for (int it = 0; it < iters; ++it) {
    bool ok = false;
    for (int h = 0; h <= max_halvings; ++h) {
      LAUNCH(kKOther, s, slista::launch_alpha_step(alpha, g, eta, T, cand, s));
      // forward at the candidate, keeping the tape for the gradient if accepted
      // (the FP32 loss output lands in the FP64 slot, which loss_now overwrites)
      if ((st = slista_forward(dict, X, N, lambda, cand, T, prec, Z, nullptr, 0, (float*)Jd, 1, ws, main_bytes,
                               stream)) != SLISTA_OK)
        return st;
      double Jc = 0.0;
      if ((st = loss_now(&Jc)) != SLISTA_OK) return st;
      if (!(Jc < J)) {
        eta *= 0.5;
        continue;
      }
      HIP_TRY(hipMemcpyAsync(alpha, cand, (size_t)T * sizeof(float), hipMemcpyDeviceToDevice, s));
      J = Jc;
      // the gradient from the tape the candidate's forward kept (same step pointer, so the tape is used)
      if ((st = slista_backward(dict, X, N, lambda, cand, T, prec, nullptr, dF, g, 1, ws, main_bytes, stream)) !=
          SLISTA_OK)
        return st;
      eta *= 2.0;
      ok = true;
      break;
    }
    if (!ok) break;
    ++acc;
    if (losses) losses[acc] = J;
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (accepted) *accepted = acc;
  if (lr_out) *lr_out = eta;
  return SLISTA_OK;
}

int slista_autotune(const slista_dict* dict, const float* X, int N, float lambda, const float* alpha, int T, int prec,
                    int ckpt_every, float* Z, float* dalpha, void* ws, size_t ws_bytes, void* stream, int* best,
                    double* ms) {
  if (!best) return fail(SLISTA_EINVAL, "best is NULL");
  if (!dict || N < 1 || T < 1 || ckpt_every < 1) return fail(SLISTA_EINVAL, "autotune needs N, T, ckpt_every >= 1");
  if (prec != SLISTA_FP32 && prec != SLISTA_BF16) return fail(SLISTA_EINVAL, "autotune takes SLISTA_FP32 or SLISTA_BF16");
  if (g_prof.on) return fail(SLISTA_EINVAL, "kernel timing must be off while tuning");
  int nv = 0;
  for (int v = 1; v <= slista::kPersistMaxVariant; ++v) nv += slista::persist_has_variant(dict->d.m_pad, v);
  if (ms)
    for (int v = 0; v < slista::kPersistMaxVariant; ++v) ms[v] = 0.0;
  if (nv == 0) {
    *best = 0;
    return SLISTA_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  t_family_override = 2;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = SLISTA_OK, bestv = 1;
  double bestms = 1e300;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = fail(SLISTA_EHIP, "hipEventCreate failed");
  }
  for (int v = 1; v <= slista::kPersistMaxVariant && st == SLISTA_OK; ++v) {
    if (!slista::persist_has_variant(dict->d.m_pad, v)) continue;
    t_variant_override = v;
    st = slista_forward_backward(dict, X, N, lambda, alpha, T, prec, Z, nullptr, nullptr, dalpha, ckpt_every, ws,
                                 ws_bytes, stream);
    if (st != SLISTA_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(SLISTA_EHIP, "hipEventRecord failed"); break; }
    for (int rep = 0; rep < 2 && st == SLISTA_OK; ++rep)
      st = slista_forward_backward(dict, X, N, lambda, alpha, T, prec, Z, nullptr, nullptr, dalpha, ckpt_every, ws,
                                   ws_bytes, stream);
    if (st != SLISTA_OK) break;
    float t = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      st = fail(SLISTA_EHIP, "event timing failed");
      break;
    }
    const double m = t / 2.0;
    if (ms) ms[v - 1] = m;
    if (m < bestms) {
      bestms = m;
      bestv = v;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  t_family_override = -1;
  t_variant_override = -1;
  if (st != SLISTA_OK) return st;
  record_tuned(prec, slista::persist_np(dict->d.m_pad), log2_bucket(N), bestv);
  *best = bestv;
  return SLISTA_OK;
}

int slista_tune_save(const char* path) {
  if (!path) return fail(SLISTA_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SLISTA_EINVAL, "cannot open %s for writing", path);
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  for (const auto& kv : g_tuned)
    std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
  std::fclose(f);
  return SLISTA_OK;
}

int slista_tune_load(const char* path) {
  if (!path) return fail(SLISTA_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SLISTA_EINVAL, "cannot open %s", path);
  int prec, np, nb, v, n = 0;
  while (std::fscanf(f, "%d %d %d %d", &prec, &np, &nb, &v) == 4) {
    if ((prec == SLISTA_FP32 || prec == SLISTA_BF16) && (np == 1 || np == 2 || np == 4 || np == 8) && nb >= 0 &&
        nb < 31 && v >= 1 && v <= slista::kPersistMaxVariant) {
      record_tuned(prec, np, nb, v);
      ++n;
    }
  }
  std::fclose(f);
  (void)n;
  return SLISTA_OK;
}

static void batch_release_graph(slista_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Tile rows and work count of bucket `bi` in precision pr for tile variant v.
static void batch_set_variant(slista_batch* b, size_t bi, int pr, int v) {
  slista_batch::Bucket& bk = b->buckets[bi];
  bk.variant[pr] = slista::persist_resolve_variant(pr, bk.max_m_pad, v);
  bk.nwork[pr] = 0;
  for (int p : bk.problems) {
    b->rows[pr][p] = slista::persist_rows(pr, b->probs[p].dict->d.m_pad, v);
    bk.nwork[pr] += (b->probs[p].N + b->rows[pr][p] - 1) / b->rows[pr][p];
  }
}

static Run batch_run_of(const slista_batch* b, int p, hipStream_t s);

// (problem, tile) work lists of all buckets and precisions, uploaded to
// d_work, and, once a workspace is bound, the small kernels' table, uploaded
// to d_small; synchronises.
static int batch_upload_work(slista_batch* b, hipStream_t s) {
  std::vector<int2> work;
  for (auto& bk : b->buckets) {
    // longest tiles first: larger m_pad, then problem order
    std::vector<int> order = bk.problems;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return b->probs[x].dict->d.m_pad > b->probs[y].dict->d.m_pad;
    });
    for (int pr = 0; pr < 2; ++pr) {
      bk.work_off[pr] = work.size();
      if (!b->uses[pr]) continue;
      for (int p : order) {
        const int tiles = (b->probs[p].N + b->rows[pr][p] - 1) / b->rows[pr][p];
        for (int t = 0; t < tiles; ++t) work.push_back(make_int2(p, t));
      }
    }
  }
  if (work.size() > b->work_cap) {
    // capacity for the smallest tile any variant uses (16 rows), in both precisions
    size_t cap = 0;
    for (const auto& q : b->probs) cap += 2 * (size_t)((q.N + 15) / 16);
    cap = std::max(cap, work.size());
    HIP_TRY(hipStreamSynchronize(s));
    if (b->d_work) HIP_TRY(hipFree(b->d_work));
    b->d_work = nullptr;
    b->work_cap = 0;
    HIP_TRY(hipMalloc(&b->d_work, sizeof(int2) * cap));
    b->work_cap = cap;
  }
  HIP_TRY(hipMemcpyAsync(b->d_work, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, s));
  std::vector<slista::BatchSmall> small;
  std::vector<slista::GemmArgs> corr;
  std::vector<int> tstart;
  if (b->ws) {
    // the small kernels' table: buffers of the bound workspace and the
    // step-gradient partial counts of the current tile rows
    const Sched sc{b->base, b->tail, b->T};
    const int p_lo = sc.at(0), p_hi = sc.at(b->T > 0 ? b->T - 1 : 0);
    for (auto& bk : b->buckets) {
      bk.small_off = small.size();
      bk.tstart_off = tstart.size();
      bk.corr_tiles = 0;
      bk.max_N = 0;
      bk.max_group_elems = 0;
      for (int p : bk.problems) {
        const slista_problem& q = b->probs[p];
        Run r = batch_run_of(b, p, s);
        corr.push_back(corr_args(r, q.X));
        tstart.push_back(bk.corr_tiles);
        bk.corr_tiles += corr.back().row_tiles * corr.back().col_tiles;
        const int tiles_lo = (q.N + b->rows[p_lo][p] - 1) / b->rows[p_lo][p];
        const int tiles_hi = (q.N + b->rows[p_hi][p] - 1) / b->rows[p_hi][p];
        slista::BatchSmall e;
        e.X = q.X;
        e.N = q.N;
        e.n = q.dict->d.n;
        e.mp = q.dict->d.m_pad;
        e.xsq = r.xsq();
        e.C = r.C();
        e.Cg = r.L.groups ? r.Cg() : nullptr;
        e.Fd = r.Fd();
        e.loss = q.loss;
        e.dpart = r.dpart();
        e.P = r.L.P;
        e.count0 = tiles_lo;
        e.count = tiles_lo;
        e.t_split = sc.split();
        e.count_hi = tiles_hi;
        e.alpha = q.alpha;
        e.dalpha = q.dalpha;
        small.push_back(e);
        bk.max_N = std::max(bk.max_N, q.N);
        if (e.Cg) bk.max_group_elems = std::max(bk.max_group_elems, (size_t)slista::tape_rows(q.N) / 4 * e.mp);
      }
      tstart.push_back(bk.corr_tiles);
    }
    if (!b->d_small) HIP_TRY(hipMalloc(&b->d_small, sizeof(slista::BatchSmall) * std::max(b->P, 1)));
    if (!b->d_corr) HIP_TRY(hipMalloc(&b->d_corr, sizeof(slista::GemmArgs) * std::max(b->P, 1)));
    if (!b->d_tstart) HIP_TRY(hipMalloc(&b->d_tstart, sizeof(int) * (b->P + b->buckets.size())));
    HIP_TRY(hipMemcpyAsync(b->d_small, small.data(), sizeof(slista::BatchSmall) * small.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_corr, corr.data(), sizeof(slista::GemmArgs) * corr.size(), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipMemcpyAsync(b->d_tstart, tstart.data(), sizeof(int) * tstart.size(), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return SLISTA_OK;
}

int slista_batch_create(const slista_problem* problems, int P, int T, int prec, int ckpt_every, slista_batch** out) {
  if (!out) return fail(SLISTA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!problems || P < 1 || P > 1 << 20) return fail(SLISTA_EINVAL, "need 1 <= P problems");
  if (T < 1 || T > kMaxT) return fail(SLISTA_EINVAL, "T=%d outside [1, %d]", T, kMaxT);
  if (ckpt_every < 1 || ckpt_every > kMaxT) return fail(SLISTA_EINVAL, "ckpt_every=%d must be >= 1", ckpt_every);
  Sched sc;
  int st = parse_sched(prec, T, ckpt_every, &sc);
  if (st != SLISTA_OK) return st;
  for (int p = 0; p < P; ++p) {
    const slista_problem& q = problems[p];
    if (!q.dict || !q.X || !q.alpha || !q.Z || !q.dalpha)
      return fail(SLISTA_EINVAL, "problem %d: dict, X, alpha, Z or dalpha is NULL", p);
    if (q.N < 1 || q.N > kMaxN) return fail(SLISTA_EINVAL, "problem %d: N=%d outside [1, %d]", p, q.N, kMaxN);
    if (!(q.lambda > 0.f) || !std::isfinite(q.lambda)) return fail(SLISTA_EINVAL, "problem %d: bad lambda", p);
    if (slista::persist_np(q.dict->d.m_pad) == 0)
      return fail(SLISTA_ENOTSUP, "problem %d: m_pad=%d > 2048 is not batched", p, q.dict->d.m_pad);
  }
  slista_batch* b = new (std::nothrow) slista_batch;
  if (!b) return fail(SLISTA_ENOMEM, "host allocation failed");
  b->P = P;
  b->T = T;
  b->prec = prec;
  b->base = sc.base;
  b->tail = sc.tail;
  b->k = ckpt_every;
  Span sp[2];
  const int ns = spans_of(sc, sp);
  for (int i = 0; i < ns; ++i) b->uses[sp[i].prec] = true;
  b->probs.assign(problems, problems + P);
  size_t off = 0;
  for (int p = 0; p < P; ++p) {
    b->offset.push_back(off);
    off += align256(make_layout(problems[p].dict->d, problems[p].N, T, ckpt_every).total);
  }
  b->total = off;
  b->rows[0].assign(P, 0);
  b->rows[1].assign(P, 0);
  for (int np : {8, 4, 2, 1}) {
    slista_batch::Bucket bk;
    bk.np = np;
    long long rows_total = 0;
    for (int p = 0; p < P; ++p)
      if (slista::persist_np(problems[p].dict->d.m_pad) == np) {
        bk.problems.push_back(p);
        bk.max_m_pad = std::max(bk.max_m_pad, problems[p].dict->d.m_pad);
        rows_total += problems[p].N;
      }
    if (bk.problems.empty()) continue;
    bk.rows_total = (int)std::min<long long>(rows_total, kMaxN);
    b->buckets.push_back(bk);
    // one tile variant per bucket launch: forced, tuned for the bucket's rows, or default
    for (int pr = 0; pr < 2; ++pr)
      if (b->uses[pr]) batch_set_variant(b, b->buckets.size() - 1, pr, variant_for(pr, bk.max_m_pad, bk.rows_total));
  }
  *out = b;
  return SLISTA_OK;
}

int slista_batch_workspace_size(const slista_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(SLISTA_EINVAL, "batch or bytes is NULL");
  *bytes = b->total;
  return SLISTA_OK;
}

static Run batch_run_of(const slista_batch* b, int p, hipStream_t s) {
  const slista_problem& q = b->probs[p];
  return Run{&q.dict->d, make_layout(q.dict->d, q.N, b->T, b->k), b->ws + b->offset[p], q.N, b->T, s};
}

int slista_batch_bind(slista_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!b) return fail(SLISTA_EINVAL, "batch is NULL");
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < b->total)
    return fail(SLISTA_EINVAL, "workspace must be 256-byte aligned with %zu bytes", b->total);
  hipStream_t s = (hipStream_t)stream;
  tape_forget(ws, ws_bytes);
  b->ws = (char*)ws;
  b->ws_bytes = ws_bytes;
  batch_release_graph(b);
  while (b->side.size() < b->buckets.size()) {
    hipStream_t q = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    b->side.push_back(q);
  }
  while (b->ev.size() < b->buckets.size() + 1) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->ev.push_back(e);
  }
  for (int pr = 0; pr < 2; ++pr) {
    if (!b->uses[pr]) continue;
    std::vector<slista::PersistArgs> args(b->P);
    for (int p = 0; p < b->P; ++p) {
      const slista_problem& q = b->probs[p];
      Run r = batch_run_of(b, p, s);
      slista::PersistArgs a = persist_args(r, pr, q.alpha, q.lambda);
      a.F = q.F;
      a.Fd = r.Fd();
      a.Zuser = q.Z;
      a.Vout = r.vbuf(0);
      a.Vio = r.vbuf(0);
      a.dpart = r.dpart();
      a.dF_scalar = (float)(1.0 / q.N);
      a.mode_mask = slista::kModeF | slista::kModeSeed;
      args[p] = a;
    }
    if (!b->d_args[pr]) HIP_TRY(hipMalloc(&b->d_args[pr], sizeof(slista::PersistArgs) * b->P));
    HIP_TRY(hipMemcpyAsync(b->d_args[pr], args.data(), sizeof(slista::PersistArgs) * b->P, hipMemcpyHostToDevice, s));
  }
  return batch_upload_work(b, s);
}

// Every launch of bucket bi (its problems' preparation, the forward and
// backward phases, the losses and step gradients) in stream order on s.
static int batch_run_bucket(slista_batch* b, size_t bi, hipStream_t s) {
  const slista_batch::Bucket& bk = b->buckets[bi];
  const int T = b->T, k = b->k;
  const Sched sc{b->base, b->tail, T};
  int st;
  const slista::BatchSmall* small = b->d_small + bk.small_off;
  const int nprob = (int)bk.problems.size();
  // c of every problem (one grouped correlation launch), then the norms and
  // the row-group copies of every problem in one launch
  LAUNCH(kKCorr, s, slista::launch_corr_grouped(b->d_corr + bk.small_off, b->d_tstart + bk.tstart_off, nprob,
                                                bk.corr_tiles, s));
  LAUNCH(kKOther, s, slista::launch_batch_prep(small, nprob, bk.max_N, bk.max_group_elems, s));
  auto phase = [&](bool fwd, int pr, slista::PersistPhase ph) -> int {
    LAUNCH(fwd ? kKFwd : kKBwd, s,
           slista::launch_persist_batched(fwd, pr, bk.np, bk.variant[pr], b->d_args[pr], b->d_work + bk.work_off[pr],
                                          bk.nwork[pr], bk.max_m_pad, ph, s));
    return SLISTA_OK;
  };
  Span sp[2];
  const int ns = spans_of(sc, sp);
  for (int i = 0; i < ns; ++i) {
    const int mode = i == ns - 1 ? (slista::kModeF | slista::kModeSeed) : 0;
    if ((st = phase(true, sp[i].prec, slista::PersistPhase{sp[i].t0, sp[i].t1, mode, 0, 0, 0})) != SLISTA_OK)
      return st;
  }
  LAUNCH(kKOther, s, slista::launch_batch_loss(small, nprob, s));
  if (k == 1) {
    for (int i = ns - 1; i >= 0; --i)
      if ((st = phase(false, sp[i].prec, slista::PersistPhase{0, 0, 0, 0, sp[i].t1 - 1, sp[i].t0})) != SLISTA_OK)
        return st;
  } else {
    const int nseg = (T + k - 1) / k;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int a0 = sgi * k;
      const int e = (a0 + k < T) ? a0 + k : T;
      const int pr = sc.at(a0);
      if (sgi != nseg - 1 && e - 1 > a0)
        if ((st = phase(true, pr, slista::PersistPhase{a0, e - 1, 0, 1, 0, 0})) != SLISTA_OK) return st;
      if ((st = phase(false, pr, slista::PersistPhase{0, 0, 0, 0, e - 1, a0})) != SLISTA_OK) return st;
    }
  }
  LAUNCH(kKOther, s, slista::launch_batch_dalpha(small, nprob, T, s));
  return SLISTA_OK;
}

int slista_batch_run(slista_batch* b, void* stream) {
  if (!b || !b->ws) return fail(SLISTA_EINVAL, "batch is NULL or not bound to a workspace");
  hipStream_t s = (hipStream_t)stream;
  int st;
  const size_t nb = b->buckets.size();
  if (nb == 1) return batch_run_bucket(b, 0, s);
  // the buckets share nothing: fork one stream per bucket from s and join them back
  HIP_TRY(hipEventRecord(b->ev[0], s));
  for (size_t bi = 0; bi < nb; ++bi) {
    HIP_TRY(hipStreamWaitEvent(b->side[bi], b->ev[0], 0));
    if ((st = batch_run_bucket(b, bi, b->side[bi])) != SLISTA_OK) return st;
    HIP_TRY(hipEventRecord(b->ev[1 + bi], b->side[bi]));
    HIP_TRY(hipStreamWaitEvent(s, b->ev[1 + bi], 0));
  }
  return SLISTA_OK;
}

int slista_batch_autotune(slista_batch* b, void* stream, int* variants) {
  if (!b || !b->ws) return fail(SLISTA_EINVAL, "batch is NULL or not bound to a workspace");
  if (g_prof.on) return fail(SLISTA_EINVAL, "kernel timing must be off while tuning");
  hipStream_t s = (hipStream_t)stream;
  batch_release_graph(b);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(SLISTA_EHIP, "hipEventCreate failed");
  }
  int st = SLISTA_OK;
  // one (bucket, precision) pair at a time, the others at their current variant
  for (size_t bi = 0; bi < b->buckets.size() && st == SLISTA_OK; ++bi) {
    for (int pr = 0; pr < 2 && st == SLISTA_OK; ++pr) {
      if (!b->uses[pr]) continue;
      const int mp = b->buckets[bi].max_m_pad;
      int nv = 0;
      for (int v = 1; v <= slista::kPersistMaxVariant; ++v) nv += slista::persist_has_variant(mp, v);
      if (nv < 2) continue;
      int bestv = b->buckets[bi].variant[pr];
      double bestms = 1e300;
      for (int v = 1; v <= slista::kPersistMaxVariant && st == SLISTA_OK; ++v) {
        if (!slista::persist_has_variant(mp, v)) continue;
        batch_set_variant(b, bi, pr, v);
        if ((st = batch_upload_work(b, s)) != SLISTA_OK) break;
        if ((st = slista_batch_run(b, stream)) != SLISTA_OK) break;  // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(SLISTA_EHIP, "hipEventRecord failed"); break; }
        if ((st = slista_batch_run(b, stream)) != SLISTA_OK) break;
        float t = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
          st = fail(SLISTA_EHIP, "event timing failed");
          break;
        }
        if (t < bestms) {
          bestms = t;
          bestv = v;
        }
      }
      batch_set_variant(b, bi, pr, bestv);
      if (st == SLISTA_OK) {
        const auto& bk = b->buckets[bi];
        record_tuned(pr, bk.np, log2_bucket(bk.rows_total), bestv);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int st2 = batch_upload_work(b, s);
  if (st != SLISTA_OK) return st;
  if (st2 != SLISTA_OK) return st2;
  if (variants) {
    // the variants of the schedule's first precision (the only one without an FP32 tail)
    const int pr = b->uses[b->base] ? b->base : (int)slista::kF32;
    for (int i = 0; i < 4; ++i) variants[i] = 0;
    for (const auto& bk : b->buckets) variants[bk.np == 1 ? 0 : bk.np == 2 ? 1 : bk.np == 4 ? 2 : 3] = bk.variant[pr];
  }
  return SLISTA_OK;
}

int slista_batch_capture(slista_batch* b, void* stream) {
  if (!b || !b->ws) return fail(SLISTA_EINVAL, "batch is NULL or not bound to a workspace");
  if (g_prof.on) return fail(SLISTA_EINVAL, "kernel timing must be off during capture");
  hipStream_t s = (hipStream_t)stream;
  batch_release_graph(b);
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int st = slista_batch_run(b, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != SLISTA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(SLISTA_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return SLISTA_OK;
}

int slista_batch_replay(slista_batch* b, void* stream) {
  if (!b || !b->exec) return fail(SLISTA_EINVAL, "batch is NULL or has no captured graph");
  HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return SLISTA_OK;
}

int slista_batch_destroy(slista_batch* b) {
  if (!b) return SLISTA_OK;
  (void)hipDeviceSynchronize();
  batch_release_graph(b);
  (void)hipFree(b->d_args[0]);
  (void)hipFree(b->d_args[1]);
  (void)hipFree(b->d_work);
  (void)hipFree(b->d_small);
  (void)hipFree(b->d_corr);
  (void)hipFree(b->d_tstart);
  for (hipStream_t q : b->side) (void)hipStreamDestroy(q);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  delete b;
  return SLISTA_OK;
}

// ------------------------------------------------------------- checks
int slista_kkt(const slista_dict* dict, const float* X, int N, float lambda, const float* Z, double* kkt, double* F,
               void* stream) {
  if (!dict) return fail(SLISTA_EINVAL, "dict is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  if (!(lambda >= 0.f) || !std::isfinite(lambda)) return fail(SLISTA_EINVAL, "lambda must be finite and >= 0");
  if (N > 0 && (!X || !Z || !kkt)) return fail(SLISTA_EINVAL, "X, Z or kkt is NULL");
  if (dict->d.n > slista::kkt_max_n())
    return fail(SLISTA_ENOTSUP, "slista_kkt supports n <= %d (n=%d)", slista::kkt_max_n(), dict->d.n);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(kKOther, s, slista::launch_kkt(X, dict->d.Dt, N, dict->d.n, dict->d.m, (double)lambda, Z, kkt, F, s));
  return SLISTA_OK;
}

int slista_lambda_max_workspace_size(const slista_dict* dict, int N, size_t* bytes) {
  if (!dict || !bytes) return fail(SLISTA_EINVAL, "dict or bytes is NULL");
  if (N < 0 || N > kMaxN) return fail(SLISTA_EINVAL, "N=%d outside [0, %d]", N, kMaxN);
  *bytes = align256((size_t)N * dict->d.m_pad * sizeof(float)) + align256((size_t)(N > 0 ? N : 1) * sizeof(float));
  return SLISTA_OK;
}

int slista_lambda_max(const slista_dict* dict, const float* X, int N, float* lam_max, float* lam_max_rows, void* ws,
                      size_t ws_bytes, void* stream) {
  size_t need = 0;
  int st = slista_lambda_max_workspace_size(dict, N, &need);
  if (st != SLISTA_OK) return st;
  if (!lam_max) return fail(SLISTA_EINVAL, "lam_max is NULL");
  if (N > 0 && !X) return fail(SLISTA_EINVAL, "X is NULL");
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
    return fail(SLISTA_EINVAL, "workspace must be 256-byte aligned with %zu bytes", need);
  tape_forget(ws, need);
  hipStream_t s = (hipStream_t)stream;
  const slista::Dict& d = dict->d;
  float* C = (float*)ws;
  float* rows = lam_max_rows ? lam_max_rows : (float*)((char*)ws + align256((size_t)N * d.m_pad * sizeof(float)));
  if (N > 0) {
    // the correlation product of the forward pass, same kernel and launch shape
    slista::GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = X;
    g.lda = d.n;
    g.Bt = d.Dt;
    g.ldb = d.n;
    g.rows = N;
    g.ncols = d.m_pad;
    g.K = d.n;
    g.Out = C;
    g.ldz = d.m_pad;
    slista::gemm_grid(N, d.m_pad, g);
    LAUNCH(kKCorr, s, slista::launch_gemm(slista::kF32, slista::kEpiCorr, true, g, s));
    LAUNCH(kKOther, s, slista::launch_row_absmax(C, N, d.m_pad, d.m, rows, s));
  }
  LAUNCH(kKOther, s, slista::launch_absmax(rows, N, 1, 1, lam_max, s));
  return SLISTA_OK;
}

// ------------------------------------------------------------- one-call batches
// Plans (a bound slista_batch, its captured graph and a capture stream) kept
// per (problem array contents, T, prec, ckpt_every, workspace), least recently
// used first out.
namespace {
struct Plan {
  std::vector<unsigned char> key;
  slista_batch* b = nullptr;
  hipStream_t cap = nullptr;
  bool captured = false;
};
std::mutex g_plan_mu;
std::vector<Plan> g_plans;
constexpr size_t kMaxPlans = 8;

void plan_release(Plan& pl) {
  if (pl.b) slista_batch_destroy(pl.b);
  if (pl.cap) (void)hipStreamDestroy(pl.cap);
  pl.b = nullptr;
  pl.cap = nullptr;
}

void plan_key(std::vector<unsigned char>& key, const slista_problem* problems, int P, int T, int prec, int k,
              void* ws, size_t ws_bytes) {
  key.assign(sizeof(slista_problem) * (size_t)P + 3 * sizeof(int) + sizeof(void*) + sizeof(size_t), 0);
  unsigned char* q = key.data();
  std::memcpy(q, problems, sizeof(slista_problem) * (size_t)P);
  q += sizeof(slista_problem) * (size_t)P;
  const int v[3] = {T, prec, k};
  std::memcpy(q, v, sizeof v);
  q += sizeof v;
  std::memcpy(q, &ws, sizeof ws);
  q += sizeof ws;
  std::memcpy(q, &ws_bytes, sizeof ws_bytes);
}
}  // namespace

int slista_batched_workspace_size(const slista_problem* problems, int P, int T, int prec, int ckpt_every,
                                  size_t* bytes) {
  if (!bytes) return fail(SLISTA_EINVAL, "bytes is NULL");
  slista_batch* b = nullptr;
  const int st = slista_batch_create(problems, P, T, prec, ckpt_every, &b);
  if (st != SLISTA_OK) return st;
  *bytes = b->total;
  slista_batch_destroy(b);
  return SLISTA_OK;
}

int slista_batched_fwd_bwd(const slista_problem* problems, int P, int T, int prec, int ckpt_every, void* ws,
                           size_t ws_bytes, void* stream, int use_graph) {
  if (!problems || P < 1 || P > 1 << 20) return fail(SLISTA_EINVAL, "need 1 <= P problems");
  if (use_graph && g_prof.on) return fail(SLISTA_EINVAL, "kernel timing must be off with use_graph");
  hipStream_t s = (hipStream_t)stream;
  std::vector<unsigned char> key;
  plan_key(key, problems, P, T, prec, ckpt_every, ws, ws_bytes);
  std::lock_guard<std::mutex> lock(g_plan_mu);
  size_t idx = g_plans.size();
  for (size_t i = 0; i < g_plans.size(); ++i)
    if (g_plans[i].key == key) idx = i;
  if (idx == g_plans.size()) {
    Plan pl;
    pl.key = std::move(key);
    int st = slista_batch_create(problems, P, T, prec, ckpt_every, &pl.b);
    if (st == SLISTA_OK) st = slista_batch_bind(pl.b, ws, ws_bytes, stream);
    if (st != SLISTA_OK) {
      plan_release(pl);
      return st;
    }
    if (g_plans.size() >= kMaxPlans) {
      plan_release(g_plans.front());
      g_plans.erase(g_plans.begin());
    }
    g_plans.push_back(std::move(pl));
    idx = g_plans.size() - 1;
  } else if (idx + 1 != g_plans.size()) {
    // most recently used last
    Plan pl = std::move(g_plans[idx]);
    g_plans.erase(g_plans.begin() + (long)idx);
    g_plans.push_back(std::move(pl));
    idx = g_plans.size() - 1;
  }
  Plan& pl = g_plans[idx];
  if (!use_graph) return slista_batch_run(pl.b, stream);
  if (!pl.captured) {
    // capture on a stream of the plan's own (a legacy default stream cannot
    // be captured); the graph is then launched on the caller's stream
    if (!pl.cap) HIP_TRY(hipStreamCreateWithFlags(&pl.cap, hipStreamNonBlocking));
    const int st = slista_batch_capture(pl.b, pl.cap);
    if (st != SLISTA_OK) return st;
    pl.captured = true;
  }
  return slista_batch_replay(pl.b, s);
}

int slista_batched_release(void) {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  for (auto& pl : g_plans) plan_release(pl);
  g_plans.clear();
  return SLISTA_OK;
}

}  // extern "C"
