// Preparation, elementwise and reduction kernels around the fused layer
// contraction: Gram matrix, power iteration for L, ||x||^2, the first layer
// (z^(0) = 0 makes it elementwise), the copy of z^(T) to the caller's
// layout, and the fixed-order reductions of the objective and of
// d loss / d alpha.
//
// Every reduction runs in a fixed order that depends only on the sizes, so
// results are bitwise reproducible run to run; no floating-point atomics.
#include "common.hpp"

namespace slista {
namespace {

constexpr int kRedThreads = 256;

// Fixed-order block reduction of one double per thread (tree over LDS).
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// G = D^T D accumulated in FP64, rounded to FP32 and BF16; D^T stored
// K-contiguous for the correlation product. One thread per entry of G.
__global__ void k_gram(const float* __restrict__ D, int n, int m, int mp, float* __restrict__ G32,
                       uint16_t* __restrict__ Gb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= mp) return;
  double s = 0.0;
  if (i < m && j < m)
    for (int k = 0; k < n; ++k) s += (double)D[(size_t)k * m + i] * (double)D[(size_t)k * m + j];
  const float f = (float)s;
  G32[(size_t)i * mp + j] = f;
  Gb[(size_t)i * mp + j] = __builtin_bit_cast(uint16_t, (__bf16)f);
}

__global__ void k_transpose(const float* __restrict__ D, int n, int m, int mp, float* __restrict__ Dt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (k >= n) return;
  Dt[(size_t)j * n + k] = j < m ? D[(size_t)k * m + j] : 0.f;
}

// Deterministic start vector in [0.5, 1.5): an integer hash of the index.
__device__ double start_value(int j) {
  uint32_t h = (uint32_t)j * 2654435761u + 0x9e3779b9u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  return 0.5 + (double)(h & 0xffffff) / 16777216.0;
}

// Power iteration for the top eigenvalue of G (FP64 arithmetic on the FP32
// entries), one iteration = k_power_mv (all CUs: one wave per row of G) then
// k_power_norm (one workgroup: Rayleigh quotient, normalisation, stopping
// test). State in `work`: [0, mp) = v, [mp, 2mp) = w, then L, iterations,
// converged flag, previous quotient, zero-vector flag. Once a stop condition
// holds the later launches return at once, so the host can enqueue batches of
// iterations and test the flags between batches. Stops when successive
// Rayleigh quotients agree to rtol.
constexpr int kPowL = 0, kPowIt = 1, kPowConv = 2, kPowPrev = 3, kPowZero = 4;

__device__ __forceinline__ bool power_done(const double* st, int max_iter) {
  return st[kPowConv] != 0.0 || st[kPowZero] != 0.0 || st[kPowIt] >= (double)max_iter;
}

__global__ __launch_bounds__(1024) void k_power_init(int m, int mp, double* work) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  double nrm = 0.0;
  for (int j = tid; j < m; j += blockDim.x) nrm += start_value(j) * start_value(j);
  nrm = sqrt(block_sum(nrm, sh));
  for (int j = tid; j < mp; j += blockDim.x) work[j] = j < m ? start_value(j) / nrm : 0.0;
  if (tid < 8) work[2 * mp + tid] = 0.0;
}

__global__ __launch_bounds__(256) void k_power_mv(const float* __restrict__ G, int m, int mp, int max_iter,
                                                  double* __restrict__ work) {
  const double* st = work + 2 * mp;
  if (power_done(st, max_iter)) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const double* v = work;
  double s = 0.0;
  for (int j = lane; j < m; j += 64) s += (double)G[(size_t)i * mp + j] * v[j];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) work[mp + i] = s;
}

__global__ __launch_bounds__(1024) void k_power_norm(int m, int mp, int max_iter, double rtol, double* work) {
  __shared__ double sh[1024];
  double* st = work + 2 * mp;
  if (power_done(st, max_iter)) return;
  const int tid = threadIdx.x;
  double* v = work;
  const double* w = work + mp;
  double pr = 0.0, pw = 0.0;
  for (int j = tid; j < m; j += blockDim.x) {
    pr += v[j] * w[j];
    pw += w[j] * w[j];
  }
  const double rq = block_sum(pr, sh);
  const double nw = sqrt(block_sum(pw, sh));
  const double it = st[kPowIt] + 1.0;
  const double prev = st[kPowPrev];
  __syncthreads();  // every thread has read the state before thread 0 updates it
  if (nw == 0.0) {
    if (tid == 0) {
      st[kPowIt] = it;
      st[kPowL] = rq;
      st[kPowZero] = 1.0;
    }
    return;
  }
  for (int j = tid; j < m; j += blockDim.x) v[j] = w[j] / nw;
  if (tid == 0) {
    st[kPowIt] = it;
    st[kPowL] = rq;
    st[kPowPrev] = rq;
    if (it > 1.0 && fabs(rq - prev) <= rtol * fabs(rq)) st[kPowConv] = 1.0;
  }
}

// ||x_i||^2 in FP64, one wave per sample.
__device__ void xsq_rows(const float* __restrict__ X, int N, int n, double* __restrict__ xsq, int block) {
  const int lane = threadIdx.x & 63;
  const int i = block * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  double s = 0.0;
  for (int k = lane; k < n; k += 64) {
    const double x = X[(size_t)i * n + k];
    s += x * x;
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) xsq[i] = s;
}

__global__ void k_xsq(const float* __restrict__ X, int N, int n, double* __restrict__ xsq) {
  xsq_rows(X, N, n, xsq, blockIdx.x);
}

// First layer from z^(0) = 0: the product vanishes, so
// z^(1) = ST(0 - a (0 - c), lam a) with the same FP32 operation order as the
// fused layer epilogue.
__global__ void k_layer0(const float4* __restrict__ C, size_t n4, const float* __restrict__ alpha,
                         float lam, float4* __restrict__ Z1) {
  const float a = alpha[0], th = lam * a;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 c = C[i];
    float4 z;
    float u;
    u = 0.f - a * (0.f - c.x); z.x = soft_threshold(u, th);
    u = 0.f - a * (0.f - c.y); z.y = soft_threshold(u, th);
    u = 0.f - a * (0.f - c.z); z.z = soft_threshold(u, th);
    u = 0.f - a * (0.f - c.w); z.w = soft_threshold(u, th);
    Z1[i] = z;
  }
}

__global__ void k_copy_out(const float* __restrict__ Zs, int N, int ldz, int m, float* __restrict__ Z) {
  const size_t total = (size_t)N * m;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / m, j = e - i * m;
    Z[e] = Zs[i * ldz + j];
  }
}

__global__ void k_fill(float* __restrict__ p, size_t count, float v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// Row-group copy of a [N][ld] matrix: the four rows 4q..4q+3 of column j go
// to the 16 bytes at float (q ld + j) 4, rows past N as 0 (the order of the
// persistent kernels' accumulator, so a lane reads its four rows at once).
// One thread per (group, column): coalesced reads of four rows, coalesced
// 16-byte writes.
__device__ void row_groups(const float* __restrict__ A, int N, int ld, float4* __restrict__ out) {
  // every group of the tape_rows(N) rows: zeros past N
  const size_t ng = (size_t)tape_rows(N) / 4, total = ng * ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t q = e / ld;
    const int j = (int)(e - q * ld), i = (int)(4 * q);
    float4 v;
    v.x = i < N ? A[(size_t)i * ld + j] : 0.f;
    v.y = i + 1 < N ? A[(size_t)(i + 1) * ld + j] : 0.f;
    v.z = i + 2 < N ? A[(size_t)(i + 2) * ld + j] : 0.f;
    v.w = i + 3 < N ? A[(size_t)(i + 3) * ld + j] : 0.f;
    out[e] = v;
  }
}

__global__ void k_row_groups(const float* __restrict__ A, int N, int ld, float4* __restrict__ out) {
  row_groups(A, N, ld, out);
}

// F_i = 1/2 ||x_i||^2 + sum over column tiles of the fused partials
// (1/2 z.Gz - z.c + lam |z|), i.e. Eq. (1) in Gram form.
__global__ void k_reduce_f(const double* __restrict__ xsq, const double* __restrict__ fpart,
                           int col_tiles, int N, float* __restrict__ F, double* __restrict__ Fd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.5 * xsq[i];
  for (int c = 0; c < col_tiles; ++c) s += fpart[(size_t)c * N + i];
  if (F) F[i] = (float)s;
  if (Fd) Fd[i] = s;
}

// Sum of Fd[0..N) by one workgroup of kSumThreads: each thread keeps eight
// partial sums over a fixed stride pattern (eight loads in flight), then a
// tree over the workgroup; the order depends on N alone.
constexpr int kSumThreads = 1024;
__device__ double sum_fixed(const double* __restrict__ Fd, int N, double* sh) {
  double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 7 * kSumThreads < N; i += 8 * kSumThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u] += Fd[i + u * kSumThreads];
  }
  // fewer than eight strides remain
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (i + u * kSumThreads < N) p[u] += Fd[i + u * kSumThreads];
  const double v = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  return block_sum(v, sh);
}

__global__ __launch_bounds__(kSumThreads) void k_reduce_loss(const double* __restrict__ Fd, int N,
                                                             float* __restrict__ loss) {
  __shared__ double sh[kSumThreads];
  const double s = sum_fixed(Fd, N, sh);
  if (threadIdx.x == 0) *loss = N > 0 ? (float)(s / N) : 0.f;
}

// Mean of the per-sample objectives in FP64 (the training loop's loss).
__global__ __launch_bounds__(kSumThreads) void k_mean_d(const double* __restrict__ Fd, int N,
                                                        double* __restrict__ out) {
  __shared__ double sh[kSumThreads];
  const double s = sum_fixed(Fd, N, sh);
  if (threadIdx.x == 0) *out = N > 0 ? s / N : 0.0;
}

// Candidate steps of one training iteration: max(alpha - eta g, 0) (FP64
// arithmetic, rounded once to FP32).
__global__ void k_alpha_step(const float* __restrict__ alpha, const float* __restrict__ g, double eta, int T,
                             float* __restrict__ cand) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double a = (double)alpha[t] - eta * (double)g[t];
  cand[t] = (float)(a > 0.0 ? a : 0.0);
}

// FISTA momentum (Beck & Teboulle): tau_0 = 1, tau_{t+1} = (1 + sqrt(1 + 4
// tau_t^2)) / 2, beta_t = (tau_t - 1) / tau_{t+1}; a sequential recurrence.
__global__ void k_fista_beta(int T, float* __restrict__ beta) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double tau = 1.0;
  for (int t = 0; t < T; ++t) {
    const double tn = (1.0 + sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
    beta[t] = (float)((tau - 1.0) / tn);
    tau = tn;
  }
}

// L_S of one sample's support per wave (Oracle-ISTA, Section 3). The support
// S of row i of Z is compacted in index order (a ballot per 64 columns); then
// Lanczos (three-term recurrence in FP64, no stored basis) from a fixed start
// vector, a hash of the atom indices, with lanes owning coordinates
// lane + 64 c. Supports of at most kLsCache atoms apply G_SS, gathered once
// into LDS from the FP32 Gram matrix; larger ones apply D_S^T D_S in
// factored form, r = D_S q (lanes owning rows of D, one coalesced row of D^T
// per atom), then D_S^T r (lanes owning atoms), in FP64 from D's FP32 values:
// 2 n |S| per step and no gather of |S|^2 scattered Gram entries. The largest
// eigenvalue of the Lanczos tridiagonal matrix rises to L_S; it is evaluated
// every 4 steps (65-point multisection with Sturm counts) and
// the recurrence stops when two evaluations agree to tol, after min(|S|,
// max_iter, kLsMaxSteps) steps, or when the Krylov space is exhausted.
// step[i] = 1/L_S, 1/L for an empty support. One 64-lane workgroup per
// sample: reductions are fixed-order shuffles and the barriers cost one wave.
// L_S depends on the support alone (and the run is deterministic), so a
// sample whose support has not changed since the last call keeps step[i]:
// row i of V holds that support as a bitmask (one 64-bit word per 64
// columns) and, in its last word, a flag that step[i] is valid (V
// zero-filled before the first layer).
constexpr int kLsLanes = 64;
constexpr int kLsCache = 64;
constexpr int kLsMaxSteps = 128;  // Krylov dimension cap

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Two launches per call split the samples by support size, so that each
// sizes its LDS for its own path (the large-support one needs no G_SS cache
// and so keeps more workgroups per CU). LDS: q, q_prev, w [mp] doubles each,
// the tridiagonal (2 kLsMaxSteps doubles), then r = D_S q [n_pad] doubles
// (large supports) or G_SS [kLsCache][kLsCache + 1] floats (small ones), and
// the support indices [mp] ints.
__host__ __device__ size_t support_vec_bytes(int mp, int n, bool large) {
  return ((size_t)3 * mp + 2 * kLsMaxSteps + (large ? (size_t)(n + 63) / 64 * 64 : 0)) * sizeof(double);
}

__host__ __device__ size_t ls_lds_bytes(int mp, int n, bool large) {
  return support_vec_bytes(mp, n, large) + (large ? 0 : (size_t)kLsCache * (kLsCache + 1) * sizeof(float)) +
         (size_t)mp * sizeof(int);
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..k) and off-diagonal b[1..k) (Sturm sequence of the LDL^T pivots).
__device__ int sturm_below(const double* a, const double* b, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    d = (a[i] - x) - (i > 0 ? b[i] * b[i] / d : 0.0);
    if (d == 0.0) d = -1e-300;
    cnt += d < 0.0;
  }
  return cnt;
}

// Largest eigenvalue of the symmetric tridiagonal (a[0..k), b[1..k)): the
// Gershgorin interval narrowed by 65-point multisection, lane l testing
// lo + (l + 1)(hi - lo) / 65, until it is 1e-15 relative (at most 12 rounds).
// Wave-uniform; returns the upper end.
__device__ double tridiag_top(const double* a, const double* b, int k, int lane) {
  double lo = 1e300, hi = -1e300;
  for (int r = 0; r < k; ++r) {
    const double off = (r > 0 ? fabs(b[r]) : 0.0) + (r + 1 < k ? fabs(b[r + 1]) : 0.0);
    lo = fmin(lo, a[r] - off);
    hi = fmax(hi, a[r] + off);
  }
  for (int round = 0; round < 12 && hi - lo > 1e-15 * fmax(fabs(hi), 1e-300); ++round) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(kLsLanes + 1);
    const unsigned long long above = __ballot(sturm_below(a, b, k, x) == k);  // x above every eigenvalue
    if (above == 0ull) {
      lo = lo + (hi - lo) * (double)kLsLanes / (double)(kLsLanes + 1);
    } else {
      const int f = __ffsll((long long)above) - 1;  // first lane above the largest eigenvalue
      const double nlo = f > 0 ? lo + (hi - lo) * (double)f / (double)(kLsLanes + 1) : lo;
      hi = lo + (hi - lo) * (double)(f + 1) / (double)(kLsLanes + 1);
      lo = nlo;
    }
  }
  return hi;
}

// LARGE: this launch handles the samples whose support holds more than
// kLsCache atoms (factored form); otherwise those with at most kLsCache
// (G_SS cached in LDS), including empty supports.
template <bool LARGE>
__global__ __launch_bounds__(kLsLanes) void k_support_lipschitz(const float* __restrict__ G,
                                                               const float* __restrict__ Dt, int n, int m, int mp,
                                                               const float* __restrict__ Z, float* __restrict__ V,
                                                               double L, int max_iter, double tol,
                                                               float* __restrict__ step) {
  extern __shared__ __attribute__((aligned(16))) char sm[];
  double* q = (double*)sm;                  // [mp] q_j
  double* qp = q + mp;                      // [mp] q_{j-1}
  double* wv = qp + mp;                     // [mp] D_S^T D_S q_j, then the next residual
  double* la = wv + mp;                     // [kLsMaxSteps] tridiagonal: diagonal
  double* lb = la + kLsMaxSteps;            // [kLsMaxSteps] off-diagonal (lb[j] couples j-1, j)
  double* rv = lb + kLsMaxSteps;            // [n_pad] D_S q_j (LARGE)
  float* gs = (float*)(sm + support_vec_bytes(mp, n, LARGE));  // [kLsCache][kLsCache + 1] (not LARGE)
  int* idx = (int*)(sm + ls_lds_bytes(mp, n, LARGE) - (size_t)mp * sizeof(int));  // [mp]
  const int i = blockIdx.x, lane = threadIdx.x;
  const float* z = Z + (size_t)i * mp;
  unsigned long long* memo = (unsigned long long*)(V + (size_t)i * mp);  // [mp / 2] words
  const int valid_word = mp / 2 - 1;
  bool same = memo[valid_word] != 0ull;
  int ns = 0;
  for (int j0 = 0; j0 < m; j0 += kLsLanes) {
    const int j = j0 + lane;
    const bool nz = j < m && z[j] != 0.f;
    const unsigned long long ball = __ballot(nz);
    if (nz) idx[ns + __popcll(ball & ((1ull << lane) - 1ull))] = j;
    ns += __popcll(ball);
    same = same && memo[j0 / kLsLanes] == ball;
  }
  __syncthreads();
  if ((ns > kLsCache) != LARGE) return;  // the other launch's sample
  if (same) return;  // the support of the last call: step[i] holds its 1/L_S
  // record this support (every lane holds every ballot; lane 0 writes them)
  {
    int j0 = 0;
    for (int c = 0; j0 < m; ++c, j0 += kLsLanes) {
      const int j = j0 + lane;
      const unsigned long long ball = __ballot(j < m && z[j] != 0.f);
      if (lane == 0) memo[c] = ball;
    }
    if (lane == 0) memo[valid_word] = 1ull;
  }
  if (ns == 0) {
    if (lane == 0) step[i] = (float)(1.0 / L);
    return;
  }
  constexpr bool cached = !LARGE;
  if (cached)
    for (int e = lane; e < ns * ns; e += kLsLanes) {
      const int r = e / ns, c = e - r * ns;
      gs[r * (kLsCache + 1) + c] = G[(size_t)idx[r] * mp + idx[c]];
    }
  double nrm = 0.0;
  for (int c = lane; c < ns; c += kLsLanes) {
    q[c] = start_value(idx[c]);
    qp[c] = 0.0;
    nrm += q[c] * q[c];
  }
  nrm = sqrt(wave_sum(nrm));
  for (int c = lane; c < ns; c += kLsLanes) q[c] /= nrm;
  __syncthreads();
  int kmax = ns < max_iter ? ns : max_iter;
  if (kmax > kLsMaxSteps) kmax = kLsMaxSteps;
  double beta = 0.0, top = 0.0, prev = -1.0;
  for (int j = 0; j < kmax; ++j) {
    if (!cached) {
      // r = D_S q: lane i owns rows i, i + 64, ... of D; row idx[l] of D^T
      // is contiguous in i, so each step of the loop reads one coalesced row
      for (int i0 = 0; i0 < n; i0 += kLsLanes) {
        const int i = i0 + lane;
        double racc = 0.0;
        if (i < n)
          for (int l = 0; l < ns; ++l) racc += (double)Dt[(size_t)idx[l] * n + i] * q[l];
        rv[i] = racc;  // rv holds n_pad entries, so i < n_pad here
      }
      __syncthreads();  // r visible to every lane
    }
    double pa = 0.0;
    for (int c = lane; c < ns; c += kLsLanes) {
      double sacc = 0.0;
      if (cached) {
        const float* grow = gs + c * (kLsCache + 1);
        for (int l = 0; l < ns; ++l) sacc += (double)grow[l] * q[l];
      } else {
        // (D_S^T r)_c from row idx[c] of D^T
        const float* drow = Dt + (size_t)idx[c] * n;
        for (int i = 0; i < n; ++i) sacc += (double)drow[i] * rv[i];
      }
      wv[c] = sacc;
      pa += q[c] * sacc;
    }
    const double alpha = wave_sum(pa);
    double pb = 0.0;
    for (int c = lane; c < ns; c += kLsLanes) {
      const double r = wv[c] - alpha * q[c] - beta * qp[c];
      wv[c] = r;
      pb += r * r;
    }
    const double b = sqrt(wave_sum(pb));
    if (lane == 0) la[j] = alpha;
    const int k = j + 1;
    __syncthreads();  // la[j] visible
    const bool last = k == kmax || !(b > 1e-13 * (fabs(alpha) + beta));
    if (last || (k % 4) == 0) {
      top = tridiag_top(la, lb, k, lane);
      if (last || fabs(top - prev) <= tol * fabs(top)) break;
      prev = top;
    }
    if (lane == 0) lb[k] = b;
    for (int c = lane; c < ns; c += kLsLanes) {
      qp[c] = q[c];
      q[c] = wv[c] / b;
    }
    beta = b;
    __syncthreads();  // q_{j+1} and lb[k] visible
  }
  if (lane == 0) step[i] = (float)(top > 0.0 ? 1.0 / top : 1.0 / L);
}

// Oracle-ISTA update: row i takes a_i = step[i] if its support condition
// holds (no violations counted by the gradient epilogue), else 1/L.
__global__ void k_oista_update(const float* __restrict__ Z, const float* __restrict__ R,
                               const double* __restrict__ flags, int col_tiles, const float* __restrict__ step,
                               double L, float lam, int N, int mp, float* __restrict__ Zout,
                               float* __restrict__ steps_used) {
  const size_t total = (size_t)N * mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / mp);
    double viol = 0.0;
    for (int ct = 0; ct < col_tiles; ++ct) viol += flags[(size_t)ct * N + i];
    const float a = viol == 0.0 ? step[i] : (float)(1.0 / L);
    const float u = Z[e] - a * R[e], th = lam * a;
    Zout[e] = soft_threshold(u, th);
    if (steps_used && e == (size_t)i * mp) steps_used[i] = a;
  }
}

// Layer 0 of the adjoint: z^(0) = 0, so the partial is sum v^0 (0 - z^(1)).
__global__ void k_bwd0(const float* __restrict__ V0, const float* __restrict__ Z1, size_t total,
                       double* __restrict__ dpart) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    s += (double)V0[e] * (0.0 - (double)Z1[e]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) dpart[blockIdx.x] = s;
}

// dalpha_t = -(1/alpha_t) sum_p dpart[t][p]: on the active set,
// z^t - z^{t+1} = alpha_t (G z^t - c + lam sign u), so this equals
// -sum v (G z^t - c + lam sign u), the derivative of the layer output in a_t.
__device__ void reduce_dalpha_layer(const double* __restrict__ dpart, int P, int count0, int count, int t_split,
                                    int count_hi, const float* __restrict__ alpha, float* __restrict__ dalpha,
                                    int t, double* sh) {
  const int n = t == 0 ? count0 : (t >= t_split ? count_hi : count);
  double s = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) s += dpart[(size_t)t * P + p];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) dalpha[t] = (float)(-s / (double)alpha[t]);
}

__global__ void k_reduce_dalpha(const double* __restrict__ dpart, int P, int count0, int count, int t_split,
                                int count_hi, const float* __restrict__ alpha, float* __restrict__ dalpha) {
  __shared__ double sh[kRedThreads];
  reduce_dalpha_layer(dpart, P, count0, count, t_split, count_hi, alpha, dalpha, blockIdx.x, sh);
}

// Uneven batches: blockIdx.y indexes the bucket's problem table.
__global__ void k_batch_prep(const BatchSmall* __restrict__ tab) {
  const BatchSmall& b = tab[blockIdx.y];
  // the norms: the blocks of k_xsq's grid, then the rest of this grid idles
  if ((int)blockIdx.x < (b.N + 3) / 4) xsq_rows(b.X, b.N, b.n, b.xsq, blockIdx.x);
  if (b.Cg) row_groups(b.C, b.N, b.mp, (float4*)b.Cg);
}

__global__ void k_batch_reduce_dalpha(const BatchSmall* __restrict__ tab) {
  __shared__ double sh[kRedThreads];
  const BatchSmall& b = tab[blockIdx.y];
  reduce_dalpha_layer(b.dpart, b.P, b.count0, b.count, b.t_split, b.count_hi, b.alpha, b.dalpha, blockIdx.x, sh);
}

__global__ __launch_bounds__(kSumThreads) void k_batch_reduce_loss(const BatchSmall* __restrict__ tab) {
  __shared__ double sh[kSumThreads];
  const BatchSmall& b = tab[blockIdx.x];
  if (!b.loss) return;
  const double s = sum_fixed(b.Fd, b.N, sh);
  if (threadIdx.x == 0) *b.loss = b.N > 0 ? (float)(s / b.N) : 0.f;
}

// F_i = 1/2 ||x_i - D z_i||^2 + lam ||z_i||_1 (Eq. (1)), one wave per sample.
// Each lane owns coordinates j = lane, lane + 64, ... of the residual (at most
// 8 per lane: n <= 512); the loop over the coordinates k of z skips zeros
// (a wave-uniform branch) and adds z_k D[:, k] from the K-contiguous row k of D^T.
constexpr int kObjMaxPerLane = 8;
__global__ void k_objective(const float* __restrict__ X, const float* __restrict__ Dt, int N, int n, int m,
                            float lam, const float* __restrict__ Z, float* __restrict__ F) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  float r[kObjMaxPerLane];
#pragma unroll
  for (int q = 0; q < kObjMaxPerLane; ++q) {
    const int j = lane + 64 * q;
    r[q] = j < n ? X[(size_t)i * n + j] : 0.f;
  }
  double l1 = 0.0;
  const float* zi = Z + (size_t)i * m;
  for (int k = 0; k < m; ++k) {
    const float zk = zi[k];
    if (zk == 0.f) continue;
    if (lane == 0) l1 += fabs((double)zk);
    const float* dk = Dt + (size_t)k * n;
#pragma unroll
    for (int q = 0; q < kObjMaxPerLane; ++q) {
      const int j = lane + 64 * q;
      if (j < n) r[q] -= zk * dk[j];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kObjMaxPerLane; ++q) s += (double)r[q] * (double)r[q];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) F[i] = (float)(0.5 * s + (double)lam * l1);
}

int grid_for(size_t work, int per_block) {
  size_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (int)b;
}

}  // namespace

hipError_t launch_gram(const float* D, int n, int m, int mp, float* G32, uint16_t* Gb, float* Dt,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_gram, dim3((mp + 255) / 256, mp), dim3(256), 0, s, D, n, m, mp, G32, Gb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose, dim3((n + 255) / 256, mp), dim3(256), 0, s, D, n, m, mp, Dt);
  return hipGetLastError();
}

hipError_t launch_power_init(int m, int mp, double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_power_init, dim3(1), dim3(1024), 0, s, m, mp, work);
  return hipGetLastError();
}

hipError_t launch_power_step(const float* G32, int m, int mp, int max_iter, double rtol, double* work,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_power_mv, dim3((m + 3) / 4), dim3(256), 0, s, G32, m, mp, max_iter, work);
  hipLaunchKernelGGL(k_power_norm, dim3(1), dim3(1024), 0, s, m, mp, max_iter, rtol, work);
  return hipGetLastError();
}

hipError_t launch_xsq(const float* X, int N, int n, double* xsq, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xsq, dim3((N + 3) / 4), dim3(256), 0, s, X, N, n, xsq);
  return hipGetLastError();
}

hipError_t launch_layer0(const float* C, int N, int ldz, const float* alpha, float lam, float* Z1,
                         hipStream_t s) {
  const size_t n4 = (size_t)N * ldz / 4;
  if (n4 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_layer0, dim3(grid_for(n4, 256 * 4)), dim3(256), 0, s, (const float4*)C, n4,
                     alpha, lam, (float4*)Z1);
  return hipGetLastError();
}

hipError_t launch_copy_out(const float* Zs, int N, int ldz, int m, float* Z, hipStream_t s) {
  const size_t total = (size_t)N * m;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_out, dim3(grid_for(total, 256 * 8)), dim3(256), 0, s, Zs, N, ldz, m, Z);
  return hipGetLastError();
}

hipError_t launch_row_groups(const float* A, int N, int ld, float* out, hipStream_t s) {
  const size_t total = (size_t)tape_rows(N) / 4 * ld;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_groups, dim3(grid_for(total, 256 * 4)), dim3(256), 0, s, A, N, ld, (float4*)out);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(count, 256 * 8)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_reduce_f(const double* xsq, const double* fpart, int col_tiles, int N, float* F,
                           double* Fd, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_f, dim3((N + 255) / 256), dim3(256), 0, s, xsq, fpart, col_tiles, N, F, Fd);
  return hipGetLastError();
}

hipError_t launch_reduce_loss(const double* Fd, int N, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(kSumThreads), 0, s, Fd, N, loss);
  return hipGetLastError();
}

hipError_t launch_mean_d(const double* Fd, int N, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mean_d, dim3(1), dim3(kSumThreads), 0, s, Fd, N, out);
  return hipGetLastError();
}

hipError_t launch_alpha_step(const float* alpha, const float* g, double eta, int T, float* cand, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpha_step, dim3((T + 255) / 256), dim3(256), 0, s, alpha, g, eta, T, cand);
  return hipGetLastError();
}

size_t support_lipschitz_lds(int m_pad, int n) {
  const size_t a = ls_lds_bytes(m_pad, n, true), b = ls_lds_bytes(m_pad, n, false);
  return a > b ? a : b;
}

hipError_t launch_support_lipschitz(const float* G32, const float* Dt, int n, int m, int mp, const float* Z, float* V,
                                    double L, int max_iter, double tol, int N, float* step, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const size_t lds_l = ls_lds_bytes(mp, n, true), lds_s = ls_lds_bytes(mp, n, false);
  hipError_t e = hipFuncSetAttribute((const void*)k_support_lipschitz<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_l);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_support_lipschitz<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_support_lipschitz<true>, dim3(N), dim3(kLsLanes), lds_l, s, G32, Dt, n, m, mp, Z, V, L,
                     max_iter, tol, step);
  hipLaunchKernelGGL(k_support_lipschitz<false>, dim3(N), dim3(kLsLanes), lds_s, s, G32, Dt, n, m, mp, Z, V, L,
                     max_iter, tol, step);
  return hipGetLastError();
}

hipError_t launch_oista_update(const float* Z, const float* R, const double* flags, int col_tiles, const float* step,
                               double L, float lam, int N, int mp, float* Zout, float* steps_used, hipStream_t s) {
  const size_t total = (size_t)N * mp;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_oista_update, dim3(grid_for(total, 256 * 4)), dim3(256), 0, s, Z, R, flags, col_tiles, step, L,
                     lam, N, mp, Zout, steps_used);
  return hipGetLastError();
}

hipError_t launch_fista_beta(int T, float* beta, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fista_beta, dim3(1), dim3(64), 0, s, T, beta);
  return hipGetLastError();
}

hipError_t launch_objective(const float* X, const float* Dt, int N, int n, int m, float lam, const float* Z,
                            float* F, hipStream_t s) {
  if (N == 0) return hipSuccess;
  if (n > 64 * kObjMaxPerLane) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_objective, dim3((N + 3) / 4), dim3(256), 0, s, X, Dt, N, n, m, lam, Z, F);
  return hipGetLastError();
}

int bwd0_blocks(int N, int ldz) {
  const size_t total = (size_t)N * ldz;
  size_t b = (total + 256 * 16 - 1) / (256 * 16);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

hipError_t launch_bwd0(const float* V0, const float* Z1, int N, int ldz, double* dpart, int nblocks,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_bwd0, dim3(nblocks), dim3(kRedThreads), 0, s, V0, Z1, (size_t)N * ldz, dpart);
  return hipGetLastError();
}

hipError_t launch_batch_prep(const BatchSmall* tab, int nprob, int max_N, size_t max_group_elems, hipStream_t s) {
  if (nprob == 0 || max_N == 0) return hipSuccess;
  // as many blocks as k_xsq needs for the largest problem, at least as many
  // as k_row_groups' grid-stride loop would use
  const size_t bx_xsq = (size_t)(max_N + 3) / 4, bx_grp = (size_t)grid_for(max_group_elems, 256 * 4);
  const size_t bx = bx_xsq > bx_grp ? bx_xsq : bx_grp;
  hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)bx, nprob), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_loss(const BatchSmall* tab, int nprob, hipStream_t s) {
  if (nprob == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce_loss, dim3(nprob), dim3(kSumThreads), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_batch_dalpha(const BatchSmall* tab, int nprob, int T, hipStream_t s) {
  if (nprob == 0 || T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce_dalpha, dim3(T, nprob), dim3(kRedThreads), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_reduce_dalpha(const double* dpart, int T, int P, int count0, int count, const float* alpha,
                                float* dalpha, hipStream_t s, int t_split, int count_hi) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_dalpha, dim3(T), dim3(kRedThreads), 0, s, dpart, P, count0, count, t_split, count_hi,
                     alpha, dalpha);
  return hipGetLastError();
}

}  // namespace slista
