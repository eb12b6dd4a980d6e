// Persistent coupled-LISTA kernels (Section 4, Eq. (11)-(12)): one workgroup
// carries RB = 32 samples through every layer, so the two contractions of a
// layer run back to back on chip instead of as two launches with an HBM round
// trip between them.
//
// Forward, layer t (factored form of Eq. (11)):
//   phase A  r = z D^T - x          [RB x n_pad], K = m_pad   (A = z from LDS)
//   phase B  z' = ST(z - a_t r W_t, lam b_t)  [RB x m_pad], K = n_pad  (A = r from LDS)
// and one more phase A for R^T = D z^T - x (the objective and the backward seed).
// Backward, layer t = T-1 .. 0 (v^{T-1} comes from the seed contraction):
//   phase A' q = v W_t^T  (+ dalpha_t partial q . R^t)        K = m_pad
//   phase B' v' = [z^t != 0] (v - a_t q D)  (+ dbeta_t partial v sign z^{t+1})  K = n_pad
// The forward leaves per layer R^t (chunk-major, the layout the weight-gradient
// contraction reads) and one byte per element coding [z^t != 0] and sign z^{t+1},
// four rows to a 32-bit word in the MFMA accumulator order, so each lane's
// epilogue reads one word per four elements; the backward writes v' in the
// same chunk-major layout as R^t.
//
// MFMA tiling: 4 waves; wave w owns the 16-column blocks w, w+4, ... of a
// phase's output and both 16-row blocks. Per K step of 64 bytes each lane
// reads 16 bytes of its A row from LDS and 16 bytes of its B row (a row of the
// K-contiguous operand: D, D^T, W_t or W_t^T) from global memory, where the
// operands stay L2-resident across the workgroups; FP32 issues four
// v_mfma_f32_16x16x4_f32 per 16-byte pair, BF16 one v_mfma_f32_16x16x32_bf16.
// In the one-block phases even and odd K steps go to separate accumulators
// (two more independent MFMA chains), summed before the epilogue. LDS rows are padded by 16 bytes, which
// spreads the 16 rows of a fragment read over distinct banks. The B batches
// are sized to keep both kernels within 256 VGPRs: two waves per SIMD (two
// workgroups per CU) hide each other's load latency.
#include "common.hpp"
#include "lista_persist.hpp"

namespace slista {
namespace {

constexpr int RB = kListaRows;
constexpr int NW = 4;
constexpr int NT = 64 * NW;
// Column blocks per wave and pass (G) and K steps whose B fragments are
// loaded together (U): the narrow phases (n_pad output columns, K = m_pad)
// take one block and four K steps per batch, the wide phases (m_pad output
// columns, K = n_pad) four blocks and two K steps. Each batch's loads are
// issued before the MFMAs of the batch in front of it, and the first batch
// of a phase before the epilogue of the phase in front of it.
constexpr int GA = 1, UA = 4;
constexpr int GB = 4, UB = 2;

template <int P> struct LElem { static constexpr int bytes = 4; };
template <> struct LElem<kBF16> { static constexpr int bytes = 2; };

// Store one element into an operand tile in LDS (FP32, or BF16 rounded to nearest even).
template <int P>
__device__ __forceinline__ void put_op(char* tile, int rowb, int row, int col, float v) {
  if constexpr (P == kF32)
    *(float*)(tile + row * rowb + col * 4) = v;
  else
    *(uint16_t*)(tile + row * rowb + col * 2) = __builtin_bit_cast(uint16_t, (__bf16)v);
}

// The FP32 master iterate of the BF16 kernels (and the forward's copy of x) is
// read and written only by the lane whose accumulators hold the element, so it
// is kept in accumulator order: the four rows 4q .. 4q+3 of one column are one
// 16-byte word, and a lane's epilogue moves them with one LDS access instead of
// four.
__device__ __forceinline__ int master_at(int row, int col, int m_pad) { return ((row >> 2) * m_pad + col) * 4 + (row & 3); }

template <int P>
__device__ __forceinline__ f32x4 mma(const uint4& a, const uint4& b, f32x4 c) {
  if constexpr (P == kF32) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  } else {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                0, 0);
  }
  return c;
}

// B fragments of U consecutive K steps for the column blocks cb0 + 4 g.
template <int G, int U>
struct BFrags {
  uint4 f[U][G];
};

template <int G, int U>
__device__ __forceinline__ void load_b(BFrags<G, U>& b, const char* B, size_t browb, int k0, int nk, int cb0, int ncb,
                                       int lr, int lg) {
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int cb = cb0 + 4 * g;
      b.f[u][g] = (k0 + u < nk && cb < ncb)
                      ? *(const uint4*)(B + (size_t)(cb * 16 + lr) * browb + (size_t)(k0 + u) * 64 + 16 * lg)
                      : make_uint4(0, 0, 0, 0);
    }
}

// MFMAs of the K steps k0 .. k0+U-1: with a single column block (G = 1) even
// steps go into acc and odd steps into odd, two more independent MFMA chains;
// with G > 1 the blocks already give 2 G chains and everything goes into acc.
template <int P, int G, int U>
__device__ __forceinline__ void mma_batch(const char* A, int arowb, const BFrags<G, U>& b, int k0, int nk, int cb0,
                                          int ncb, f32x4 (&acc)[G][2], f32x4 (&odd)[G][2], int lr, int lg) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k0 + u >= nk) break;
    uint4 af[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) af[rb] = *(const uint4*)(A + (rb * 16 + lr) * arowb + (k0 + u) * 64 + 16 * lg);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (cb0 + 4 * g >= ncb) continue;  // wave-uniform: no MFMAs on an empty column block
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        if (G == 1 && (u & 1))
          odd[g][rb] = mma<P>(af[rb], b.f[u][g], odd[g][rb]);
        else
          acc[g][rb] = mma<P>(af[rb], b.f[u][g], acc[g][rb]);
      }
    }
  }
}

// acc[g][rb] = A[rb 16 .., 0..K) * B[cb_g 16 .., 0..K)^T for cb_g = cb0 + 4 g < ncb:
// A in LDS (row stride arowb bytes), B in global memory (row stride browb
// bytes), nk K steps of 64 bytes. b0 holds the first U K steps' B fragments,
// loaded by the caller (ahead of time where it can); each later batch is
// loaded before the MFMAs of the batch in front of it (two buffers).
template <int P, int G, int U>
__device__ __forceinline__ void contract(const char* A, int arowb, const char* B, size_t browb, int nk, int cb0,
                                         int ncb, f32x4 (&acc)[G][2], BFrags<G, U>& b0, int lr, int lg) {
  f32x4 odd[G][2];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      acc[g][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
      odd[g][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  BFrags<G, U> b1;
  for (int k0 = 0; k0 < nk;) {
    if (k0 + U < nk) load_b(b1, B, browb, k0 + U, nk, cb0, ncb, lr, lg);
    mma_batch<P>(A, arowb, b0, k0, nk, cb0, ncb, acc, odd, lr, lg);
    k0 += U;
    if (k0 >= nk) break;
    if (k0 + U < nk) load_b(b0, B, browb, k0 + U, nk, cb0, ncb, lr, lg);
    mma_batch<P>(A, arowb, b1, k0, nk, cb0, ncb, acc, odd, lr, lg);
    k0 += U;
  }
  if constexpr (G == 1) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) acc[0][rb] += odd[0][rb];
  }
}

// Sum of one double per (wave, row) over the 16 lanes of a row group, then
// over the waves in a fixed order; returns the row sums to threads 0..RB-1.
__device__ __forceinline__ double rows_sum(double (&part)[2][4], double* red, int wave, int lr, int lg, int tid) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      double v = part[rb][r4];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if (lr == 0) red[wave * RB + rb * 16 + 4 * lg + r4] = v;
    }
  __syncthreads();
  double s = 0.0;
  if (tid < RB) s = ((red[tid] + red[RB + tid]) + red[2 * RB + tid]) + red[3 * RB + tid];
  __syncthreads();
  return s;
}

template <int P>
__global__ __launch_bounds__(NT, 2) void lista_fwd_persist(ListaPersistArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int E = LElem<P>::bytes;
  const int n_pad = a.n_pad, m_pad = a.m_pad, N = a.N, T = a.T, Kc = a.Kc;
  const int zrowb = m_pad * E + 16, rrowb = n_pad * E + 16;
  char* zA = lds;                                         // z^t, operand precision
  char* rA = zA + RB * zrowb;                             // r^t, operand precision
  float* xs = (float*)(rA + RB * rrowb);                  // x, FP32 (master_at order over n_pad)
  float* zM = xs + RB * n_pad;                            // z^t FP32 master (BF16 mode, master_at order)
  double* red = (double*)(zM + (P == kF32 ? 0 : RB * m_pad));  // [NW][RB]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int row0 = blockIdx.x * RB;
  for (int e = tid; e < RB * n_pad; e += NT) {
    const int r = e / n_pad, c = e - r * n_pad;
    xs[master_at(r, c, n_pad)] = row0 + r < N ? a.Xp[(size_t)(row0 + r) * n_pad + c] : 0.f;
  }
  for (int e = tid; e < RB * m_pad; e += NT) {
    const int r = e / m_pad, c = e - r * m_pad;
    put_op<P>(zA, zrowb, r, c, 0.f);
    if constexpr (P != kF32) zM[e] = 0.f;
  }
  __syncthreads();

  const int ncbA = n_pad / 16, ncbB = m_pad / 16;
  const int nkA = m_pad * E / 64, nkB = n_pad * E / 64;
  const size_t rlayer = (size_t)a.n * a.Np, clayer = (size_t)a.nwg * (RB / 4) * m_pad;
  const char* Dr = (const char*)a.Dr;
  BFrags<GA, UA> preA;  // first B batch of the next phase A (rows of D)
  BFrags<GB, UB> preB;  // first B batch of the next phase B (columns of W_t)
  load_b(preA, Dr, (size_t)m_pad * E, 0, nkA, wave, ncbA, lr, lg);
  for (int t = 0; t <= T; ++t) {
    const bool last = t == T;
    {  // phase A: r = z D^T - x
      float* rtape = (!last && a.rtape) ? a.rtape + (size_t)t * rlayer : nullptr;
      float* rT = last ? a.rT : nullptr;
      const bool want_f = last && a.fres;
      double fr[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      for (int c0 = wave; c0 < ncbA; c0 += 4 * GA) {
        f32x4 acc[GA][2];
        if (c0 != wave) load_b(preA, Dr, (size_t)m_pad * E, 0, nkA, c0, ncbA, lr, lg);
        contract<P, GA, UA>(zA, zrowb, Dr, (size_t)m_pad * E, nkA, c0, ncbA, acc, preA, lr, lg);
        if (!last && c0 + 4 * GA >= ncbA)  // phase B's first W_t batch, in flight during this epilogue
          load_b(preB, (const char*)a.WT + (size_t)t * m_pad * n_pad * E, (size_t)n_pad * E, 0, nkB, wave, ncbB, lr, lg);
#pragma unroll
        for (int g = 0; g < GA; ++g) {
          const int cb = c0 + 4 * g;
          if (cb >= ncbA) continue;
          const int col = cb * 16 + lr;
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            float rv[4];
            const float4 xq = *(const float4*)(xs + master_at(rb * 16 + 4 * lg, col, n_pad));
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const int row = rb * 16 + 4 * lg + r4;
              const float r = acc[g][rb][r4] - (r4 == 0 ? xq.x : r4 == 1 ? xq.y : r4 == 2 ? xq.z : xq.w);
              rv[r4] = r;
              put_op<P>(rA, rrowb, row, col, r);
              if (want_f) fr[rb][r4] += 0.5 * (double)r * (double)r;
            }
            if (rT) {  // after the last layer only
#pragma unroll
              for (int r4 = 0; r4 < 4; ++r4) {
                const int i = row0 + rb * 16 + 4 * lg + r4;
                if (i < N) rT[(size_t)i * n_pad + col] = rv[r4];
              }
            }
            if (rtape && col < a.n) {  // 4 consecutive samples of one chunk (rows >= N hold 0)
              const int i = row0 + rb * 16 + 4 * lg;
              *(float4*)(rtape + (size_t)(i / Kc) * a.n * Kc + (size_t)col * Kc + i % Kc) =
                  make_float4(rv[0], rv[1], rv[2], rv[3]);
            }
          }
        }
      }
      if (want_f) {  // uniform
        const double s = rows_sum(fr, red, wave, lr, lg, tid);
        if (tid < RB && row0 + tid < N) a.fres[row0 + tid] = s;
      }
    }
    if (last) break;
    __syncthreads();  // r^t complete
    {  // phase B: z^{t+1} = ST(z^t - a_t r W_t, lam b_t)
      const float al = a.alpha[t], th = a.lam * a.beta[t];
      float* zT = t == T - 1 ? a.zT : nullptr;
      uint32_t* codes = a.codes ? a.codes + (size_t)t * clayer : nullptr;
      const bool want_l1 = t == T - 1 && a.fl1;
      double fl[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      const char* Wt = (const char*)a.WT + (size_t)t * m_pad * n_pad * E;
      for (int c0 = wave; c0 < ncbB; c0 += 4 * GB) {
        f32x4 acc[GB][2];
        if (c0 != wave) load_b(preB, Wt, (size_t)n_pad * E, 0, nkB, c0, ncbB, lr, lg);
        contract<P, GB, UB>(rA, rrowb, Wt, (size_t)n_pad * E, nkB, c0, ncbB, acc, preB, lr, lg);
        if (c0 + 4 * GB >= ncbB)  // the next phase A's first D batch
          load_b(preA, Dr, (size_t)m_pad * E, 0, nkA, wave, ncbA, lr, lg);
#pragma unroll
        for (int g = 0; g < GB; ++g) {
          const int cb = c0 + 4 * g;
          if (cb >= ncbB) continue;
          const int col = cb * 16 + lr;
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            uint32_t word = 0;
            float4* zq = (float4*)(zM + master_at(rb * 16 + 4 * lg, col, m_pad));
            float4 zm = make_float4(0.f, 0.f, 0.f, 0.f);
            float zs[4];
            if constexpr (P != kF32) zm = *zq;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const int row = rb * 16 + 4 * lg + r4;
              float z;
              if constexpr (P == kF32)
                z = *(const float*)(zA + row * zrowb + col * 4);
              else
                z = r4 == 0 ? zm.x : r4 == 1 ? zm.y : r4 == 2 ? zm.z : zm.w;
              const float zn = soft_threshold(z - al * acc[g][rb][r4], th);
              zs[r4] = zn;
              put_op<P>(zA, zrowb, row, col, zn);
              word |= (uint32_t)((z != 0.f ? 1u : 0u) | (zn > 0.f ? 2u : 0u) | (zn < 0.f ? 4u : 0u)) << (8 * r4);
              if (want_l1) fl[rb][r4] += (double)a.lam * fabs((double)zn);
            }
            if constexpr (P != kF32) *zq = make_float4(zs[0], zs[1], zs[2], zs[3]);
            if (zT) {  // last layer only: one uniform branch, not a masked store per element
#pragma unroll
              for (int r4 = 0; r4 < 4; ++r4) {
                const int i = row0 + rb * 16 + 4 * lg + r4;
                if (i < N) zT[(size_t)i * m_pad + col] = zs[r4];
              }
            }
            if (codes) codes[(size_t)((row0 + rb * 16) / 4 + lg) * m_pad + col] = word;
          }
        }
      }
      if (want_l1) {
        const double s = rows_sum(fl, red, wave, lr, lg, tid);
        if (tid < RB && row0 + tid < N) a.fl1[row0 + tid] = s;
      }
    }
    __syncthreads();  // z^{t+1} complete
  }
}

template <int P>
__global__ __launch_bounds__(NT, 2) void lista_bwd_persist(ListaPersistArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int E = LElem<P>::bytes;
  const int n_pad = a.n_pad, m_pad = a.m_pad, N = a.N, T = a.T, Kc = a.Kc;
  const int vrowb = m_pad * E + 16, qrowb = n_pad * E + 16;
  char* vA = lds;                                   // v^t, operand precision
  char* qA = vA + RB * vrowb;                       // W_t v, operand precision
  float* vM = (float*)(qA + RB * qrowb);            // v^t FP32 master (BF16 mode, master_at order)
  double* red = (double*)(vM + (P == kF32 ? 0 : RB * m_pad));  // [2][NW]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int row0 = blockIdx.x * RB;
  const size_t rlayer = (size_t)a.n * a.Np, vlayer = (size_t)a.m * a.Np;
  const size_t clayer = (size_t)a.nwg * (RB / 4) * m_pad;
  {  // v^{T-1} from the seed, into LDS and (chunk-major) onto the tape
    for (int e = tid; e < RB * m_pad; e += NT) {
      const int r = e / m_pad, c = e - r * m_pad;
      const float v = row0 + r < N ? a.vseed[(size_t)(row0 + r) * m_pad + c] : 0.f;
      put_op<P>(vA, vrowb, r, c, v);
      if constexpr (P != kF32) vM[master_at(r, c, m_pad)] = v;
    }
    float* vt = a.vtape + (size_t)(T - 1) * vlayer;
    for (int e = tid; e < RB * a.m; e += NT) {
      const int c = e / RB, r = e - c * RB, i = row0 + r;
      vt[(size_t)(i / Kc) * a.m * Kc + (size_t)c * Kc + i % Kc] =
          i < N ? a.vseed[(size_t)i * m_pad + c] : 0.f;
    }
  }
  __syncthreads();

  const int ncbA = n_pad / 16, ncbB = m_pad / 16;
  const int nkA = m_pad * E / 64, nkB = n_pad * E / 64;
  const char* DT = (const char*)a.DT;
  BFrags<GA, UA> preA;  // first B batch of the next phase A' (rows of W_t)
  BFrags<GB, UB> preB;  // first B batch of the next phase B' (columns of D)
  load_b(preA, (const char*)a.Wr + (size_t)(T - 1) * n_pad * m_pad * E, (size_t)m_pad * E, 0, nkA, wave, ncbA, lr, lg);
  for (int t = T - 1; t >= 0; --t) {
    const float al = a.alpha[t];
    double da = 0.0, db = 0.0;
    {  // phase A': q = W_t v (rows: samples), dalpha_t partial q . R^t
      const float* R = a.rtape + (size_t)t * rlayer;
      const char* W = (const char*)a.Wr + (size_t)t * n_pad * m_pad * E;
      for (int c0 = wave; c0 < ncbA; c0 += 4 * GA) {
        float4 rv[GA][2];  // R^t of 4 consecutive samples (0 for rows >= N), in flight during the contraction
#pragma unroll
        for (int g = 0; g < GA; ++g)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            const int col = (c0 + 4 * g) * 16 + lr;
            const int i = row0 + rb * 16 + 4 * lg;
            rv[g][rb] = c0 + 4 * g < ncbA && col < a.n
                            ? *(const float4*)(R + (size_t)(i / Kc) * a.n * Kc + (size_t)col * Kc + i % Kc)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        f32x4 acc[GA][2];
        if (c0 != wave) load_b(preA, W, (size_t)m_pad * E, 0, nkA, c0, ncbA, lr, lg);
        contract<P, GA, UA>(vA, vrowb, W, (size_t)m_pad * E, nkA, c0, ncbA, acc, preA, lr, lg);
        if (c0 + 4 * GA >= ncbA) load_b(preB, DT, (size_t)n_pad * E, 0, nkB, wave, ncbB, lr, lg);
#pragma unroll
        for (int g = 0; g < GA; ++g) {
          const int cb = c0 + 4 * g;
          if (cb >= ncbA) continue;
          const int col = cb * 16 + lr;
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            const float rr[4] = {rv[g][rb].x, rv[g][rb].y, rv[g][rb].z, rv[g][rb].w};
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const int row = rb * 16 + 4 * lg + r4;
              const float q = acc[g][rb][r4];
              put_op<P>(qA, qrowb, row, col, q);
              da += (double)q * (double)rr[r4];
            }
          }
        }
      }
    }
    __syncthreads();  // q complete
    {  // phase B': v^{t-1} = [z^t != 0] (v^t - a_t q D), dbeta_t partial v^t sign z^{t+1}
      const uint32_t* codes = a.codes + (size_t)t * clayer;
      float* vt = t >= 1 ? a.vtape + (size_t)(t - 1) * vlayer : nullptr;
      for (int c0 = wave; c0 < ncbB; c0 += 4 * GB) {
        uint32_t cw[GB][2];  // issued before the contraction, consumed by the epilogue
#pragma unroll
        for (int g = 0; g < GB; ++g)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            const int cb = c0 + 4 * g;
            cw[g][rb] = cb < ncbB ? codes[(size_t)((row0 + rb * 16) / 4 + lg) * m_pad + cb * 16 + lr] : 0u;
          }
        f32x4 acc[GB][2];
        if (c0 != wave) load_b(preB, DT, (size_t)n_pad * E, 0, nkB, c0, ncbB, lr, lg);
        contract<P, GB, UB>(qA, qrowb, DT, (size_t)n_pad * E, nkB, c0, ncbB, acc, preB, lr, lg);
        if (t >= 1 && c0 + 4 * GB >= ncbB)  // the next phase A''s first W_{t-1} batch
          load_b(preA, (const char*)a.Wr + (size_t)(t - 1) * n_pad * m_pad * E, (size_t)m_pad * E, 0, nkA, wave, ncbA,
                 lr, lg);
#pragma unroll
        for (int g = 0; g < GB; ++g) {
          const int cb = c0 + 4 * g;
          if (cb >= ncbB) continue;
          const int col = cb * 16 + lr;
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            float vv[4];
            float4* vq = (float4*)(vM + master_at(rb * 16 + 4 * lg, col, m_pad));
            float4 vm = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (P != kF32) vm = *vq;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const int row = rb * 16 + 4 * lg + r4;
              float v;
              if constexpr (P == kF32)
                v = *(const float*)(vA + row * vrowb + col * 4);
              else
                v = r4 == 0 ? vm.x : r4 == 1 ? vm.y : r4 == 2 ? vm.z : vm.w;
              const uint32_t code = cw[g][rb] >> (8 * r4);
              const float sg = (code & 2u) ? 1.f : ((code & 4u) ? -1.f : 0.f);
              db += (double)v * (double)sg;
              const float vn = (code & 1u) ? v - al * acc[g][rb][r4] : 0.f;
              vv[r4] = vn;
              put_op<P>(vA, vrowb, row, col, vn);
            }
            if constexpr (P != kF32) *vq = make_float4(vv[0], vv[1], vv[2], vv[3]);
            if (vt && col < a.m) {
              const int i = row0 + rb * 16 + 4 * lg;
              *(float4*)(vt + (size_t)(i / Kc) * a.m * Kc + (size_t)col * Kc + i % Kc) =
                  make_float4(vv[0], vv[1], vv[2], vv[3]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      da += __shfl_xor(da, o);
      db += __shfl_xor(db, o);
    }
    if (lane == 0) {
      red[wave] = da;
      red[NW + wave] = db;
    }
    __syncthreads();  // v^{t-1} and the partials complete
    if (tid == 0) {
      a.dpa[(size_t)t * a.nwg + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
      a.dpb[(size_t)t * a.nwg + blockIdx.x] = ((red[NW] + red[NW + 1]) + red[NW + 2]) + red[NW + 3];
    }
  }
}

// Zero rows i0 .. Np-1 of every layer and column of a chunk-major tape.
__global__ void k_zero_tape_rows(float* __restrict__ tape, int cols, int Kc, int Np, int i0, size_t total) {
  const int span = Np - i0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t lc = e / span;
    const int i = i0 + (int)(e - lc * span);
    const size_t layer = lc / cols, c = lc - layer * cols;
    tape[layer * cols * Np + (size_t)(i / Kc) * cols * Kc + c * Kc + i % Kc] = 0.f;
  }
}

template <int P>
size_t fwd_lds(int n_pad, int m_pad) {
  constexpr int E = LElem<P>::bytes;
  size_t b = (size_t)RB * (m_pad * E + 16) + (size_t)RB * (n_pad * E + 16) + (size_t)RB * n_pad * 4;
  if (P != kF32) b += (size_t)RB * m_pad * 4;
  return b + (size_t)NW * RB * sizeof(double);
}

template <int P>
size_t bwd_lds(int n_pad, int m_pad) {
  constexpr int E = LElem<P>::bytes;
  size_t b = (size_t)RB * (m_pad * E + 16) + (size_t)RB * (n_pad * E + 16);
  if (P != kF32) b += (size_t)RB * m_pad * 4;
  return b + 2 * NW * sizeof(double);
}

template <int P>
hipError_t launch_one(bool fwd, const ListaPersistArgs& a, hipStream_t s) {
  const size_t lds = fwd ? fwd_lds<P>(a.n_pad, a.m_pad) : bwd_lds<P>(a.n_pad, a.m_pad);
  const void* fn = fwd ? (const void*)lista_fwd_persist<P> : (const void*)lista_bwd_persist<P>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = (a.N + RB - 1) / RB;
  if (fwd)
    hipLaunchKernelGGL(lista_fwd_persist<P>, dim3(grid), dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL(lista_bwd_persist<P>, dim3(grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

}  // namespace

size_t lista_persist_lds(int prec, bool fwd, int n_pad, int m_pad) {
  if (prec == kF32) return fwd ? fwd_lds<kF32>(n_pad, m_pad) : bwd_lds<kF32>(n_pad, m_pad);
  return fwd ? fwd_lds<kBF16>(n_pad, m_pad) : bwd_lds<kBF16>(n_pad, m_pad);
}

hipError_t launch_lista_persist(int prec, bool fwd, const ListaPersistArgs& a, hipStream_t s) {
  if (a.N <= 0 || a.T <= 0) return hipSuccess;
  if (a.n_pad % 64 != 0 || a.m_pad % 64 != 0 || a.Kc <= 0 || a.Kc % 64 != 0 || a.Np % a.Kc != 0 ||
      a.Np < a.nwg * RB || a.nwg != (a.N + RB - 1) / RB || lista_persist_lds(prec, fwd, a.n_pad, a.m_pad) > kListaMaxLds)
    return hipErrorInvalidValue;
  if (!fwd && (!a.rtape || !a.codes || !a.vseed || !a.vtape || !a.dpa || !a.dpb)) return hipErrorInvalidValue;
  return prec == kF32 ? launch_one<kF32>(fwd, a, s) : launch_one<kBF16>(fwd, a, s);
}

hipError_t launch_zero_tape_rows(float* tape, int layers, int cols, int Kc, int Np, int i0, hipStream_t s) {
  if (layers <= 0 || cols <= 0 || i0 >= Np) return hipSuccess;
  const size_t total = (size_t)layers * cols * (Np - i0);
  size_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_tape_rows, dim3((unsigned)blocks), dim3(256), 0, s, tape, cols, Kc, Np, i0, total);
  return hipGetLastError();
}

}  // namespace slista
