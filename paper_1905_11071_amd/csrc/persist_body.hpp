// Device code of the persistent Step-LISTA kernels (Section 4, Eq. (14)),
// shared by the BF16 and FP32 translation units: one workgroup carries a tile
// of R samples through a whole range of layers, forward or back.
//
// On-chip state of a tile (WC column waves x WR row waves of 64 lanes):
//   LDS        the tile's iterate in the contraction's precision (BF16 or
//              FP32), [R][m_pad], the A operand of P = Z G for every layer;
//   registers  the FP32 master iterate (forward: z; backward: the adjoint v)
//              in the MFMA accumulator layout, so the step, the threshold and
//              the objective never re-read z from memory.
// G streams from L2 in a fragment-ordered copy built with the dictionary:
// the 16 x 32 (BF16) or 16 x 16 (FP32) fragment a wave needs for one K step
// is 1 KiB contiguous, one 16-byte load per lane, issued PF - 1 steps ahead.
// A pass covers 256 output columns: each column wave owns a slab of 256 / WC
// columns (FB = 16 / WC blocks of 16); the tile's rows are shared by all
// waves through LDS.
//
// Per sample and layer the forward reads c = D^T x (4 m bytes) and writes
// the kept iterate (4 m bytes); the backward reads the kept z^t (4 m bytes).
//
// The K order, the per-lane K assignment and every epilogue expression of
// the forward are the same as in the per-layer kernel (kernels_gemm.hip), so
// both give bitwise-identical iterates.
#pragma once
#include "common.hpp"
#include "persist.hpp"

namespace slista {
namespace {


template <int P> struct Elem;
template <> struct Elem<kF32> { static constexpr int bytes = 4; };
template <> struct Elem<kBF16> { static constexpr int bytes = 2; };

// Bytes per row of a tile's LDS copy: m_pad elements plus 32 bytes. Rows
// then start 32 mod 64 bytes apart, which keeps the 16-byte fragment reads of
// 16 rows x 4 lanes (and the 2-byte writes of the accumulator layout) free of
// bank conflicts; a 16-byte pad measured 2-way conflicts on every read.
template <int P>
__host__ __device__ constexpr int tile_rowb(int m_pad) { return m_pad * Elem<P>::bytes + 32; }

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// Raw buffer descriptors (CDNA): a uniform base and byte range in SGPRs, so
// each access needs one per-lane VGPR offset; the row part of an offset goes
// into the SGPR soffset and the column part into the instruction's immediate.
constexpr int kRsrcWord3 = 0x00020000;
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void* base, size_t bytes) {
  const int n = bytes > 0x7fffffffu ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, kRsrcWord3);
}
// The b32 builtins move raw 32-bit patterns (unsigned int): bit-cast, never
// convert. All accesses use the default (temporal) cache policy: a tile
// re-reads its rows of c every layer and the backward reads each kept
// iterate once, and those re-reads hit in the caches (non-temporal loads
// measured 1.5x slower); non-temporal stores of the tape measured the same
// speed but 1.46x the HBM write bytes (each 64-byte half line went out on
// its own), temporal stores write exactly the stored iterates.
constexpr int kCachePolicy = 0;
__device__ __forceinline__ float bload(Rsrc r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kCachePolicy));
}
__device__ __forceinline__ void bstore(float v, Rsrc r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, kCachePolicy);
}

// The kept iterates (checkpoint and segment slots) are stored in the
// accumulator's row order: rows 4q .. 4q+3 of one column are 16 contiguous
// bytes, element (i, j) at float ((i / 4) m_pad + j) 4 + i % 4, so each lane
// moves the four rows it owns of a column with one 16-byte access. A slot
// holds tape_rows(N) rows (N rounded up to whole 64-row tiles); a tile's slot
// descriptor starts at row0 (a multiple of 16), the lane's offset is
// (lg m_pad + col) 16 bytes, the row block's (16 fm + rbase) m_pad 4 bytes
// goes into soffset.
__device__ __forceinline__ float4 bload4(Rsrc r, int voff, int soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kCachePolicy));
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bstore4(float4 v, Rsrc r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, kCachePolicy);
}
// Bytes of a tile's slot range: its rows rounded up to whole 4-row groups.
__device__ __forceinline__ size_t tape_bytes(int nrows, int m_pad) { return (size_t)((nrows + 3) / 4) * m_pad * 16; }

__device__ __forceinline__ float* slot_ptr(const PersistArgs& g, int t) {
  const int k = g.k;
  if (t % k == 0 || t == g.T) return (float*)(g.ckpt + (size_t)((t + k - 1) / k - 1) * g.zbytes);
  return (float*)(g.seg + (size_t)(t % k - 1) * g.zbytes);
}

template <int P>
__device__ __forceinline__ void mfma_pair(f32x4& acc, const uint4& a, const uint4& b) {
  if constexpr (P == kF32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   acc, 0, 0, 0);
  }
}

// One K step: prefetch the G fragments of step kc + PF - 1 and the A
// fragments of step kc + 1 (both clamped to the last step, so the loads never
// need a branch), then the FM x 4 MFMAs of step kc.
template <int P, int FM, int FB, int PF, int J>
__device__ __forceinline__ void k_step(const Rsrc& rg, int lo, int KC, const char* arow, int rowb, int kc,
                                       uint4 (&bq)[PF][FB], uint4 (&av)[2][FM], f32x4 (&acc)[FM][FB]) {
  const int nk = min(kc + PF - 1, KC - 1);
#pragma unroll
  for (int f = 0; f < FB; ++f)
    bq[(J + PF - 1) % PF][f] =
        __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rg, lo, (f * KC + nk) * 1024, 0));
  constexpr int JB = J % PF;  // slot holding step kc
  const int na = min(kc + 1, KC - 1);
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) av[(J & 1) ^ 1][fm] = *(const uint4*)(arow + fm * 16 * rowb + na * 64);
  if constexpr (P == kF32) {
    // 4 MFMAs per (fm, f) pair; the K sub-step e is the outer loop so that
    // consecutive MFMAs update independent accumulators (same order per acc)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const uint4& a = av[J & 1][fm];
          const uint4& b = bq[JB][f];
          const uint32_t ae = e == 0 ? a.x : e == 1 ? a.y : e == 2 ? a.z : a.w;
          const uint32_t be = e == 0 ? b.x : e == 1 ? b.y : e == 2 ? b.z : b.w;
          acc[fm][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ae), __uint_as_float(be), acc[fm][f], 0, 0, 0);
        }
  } else {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int f = 0; f < FB; ++f) mfma_pair<P>(acc[fm][f], av[J & 1][fm], bq[JB][f]);
  }
  // keep the step boundary: the scheduler would otherwise sink the prefetches
  // of later steps next to their uses when registers run short
  __builtin_amdgcn_sched_barrier(0);
}

// Unrolled K steps J .. U-1 from step kc0 (run), or only those below KC (tail).
template <int PF> struct Unroll { static constexpr int value = PF == 3 ? 6 : 4; };
template <int P, int FM, int FB, int PF, int J, int U>
struct KSteps {
  static __device__ __forceinline__ void run(const Rsrc& rg, int lo, int KC, const char* arow, int rowb, int kc0,
                                             uint4 (&bq)[PF][FB], uint4 (&av)[2][FM], f32x4 (&acc)[FM][FB]) {
    k_step<P, FM, FB, PF, J>(rg, lo, KC, arow, rowb, kc0 + J, bq, av, acc);
    KSteps<P, FM, FB, PF, J + 1, U>::run(rg, lo, KC, arow, rowb, kc0, bq, av, acc);
  }
  static __device__ __forceinline__ void tail(const Rsrc& rg, int lo, int KC, const char* arow, int rowb, int kc0,
                                              uint4 (&bq)[PF][FB], uint4 (&av)[2][FM], f32x4 (&acc)[FM][FB]) {
    if (kc0 + J < KC) {
      k_step<P, FM, FB, PF, J>(rg, lo, KC, arow, rowb, kc0 + J, bq, av, acc);
      KSteps<P, FM, FB, PF, J + 1, U>::tail(rg, lo, KC, arow, rowb, kc0, bq, av, acc);
    }
  }
};
template <int P, int FM, int FB, int PF, int U>
struct KSteps<P, FM, FB, PF, U, U> {
  static __device__ __forceinline__ void run(const Rsrc&, int, int, const char*, int, int, uint4 (&)[PF][FB],
                                             uint4 (&)[2][FM], f32x4 (&)[FM][FB]) {}
  static __device__ __forceinline__ void tail(const Rsrc&, int, int, const char*, int, int, uint4 (&)[PF][FB],
                                              uint4 (&)[2][FM], f32x4 (&)[FM][FB]) {}
};

// acc[fm][f] = sum_k A[16 fm + row][k] G[k][16 FB slab + 16 f + col] over
// the whole K range, A from the LDS tile, G fragments from global memory
// issued PF - 1 K steps ahead (PF = 2, 3 or 4). KEEP: the sums start from
// the values acc already holds instead of 0.
template <int P, int FM, int FB, int PF, bool KEEP = false>
__device__ __forceinline__ void contract(const PersistArgs& g, const char* lds, int rowb, int slab, int lane,
                                         f32x4 (&acc)[FM][FB]) {
  const int lr = lane & 15, lg = lane >> 4;
  const int KC = g.KC;
  // the FB * KC fragments of this slab: FB KC KiB starting at fragment (FB slab, 0)
  const Rsrc rg = make_rsrc((const char*)g.Gsw + (size_t)(FB * slab) * KC * 1024, (size_t)FB * KC * 1024);
  const int lo = lane * 16;
  if constexpr (!KEEP) {
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int f = 0; f < FB; ++f) acc[fm][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  uint4 bq[PF][FB];
#pragma unroll
  for (int i = 0; i < PF - 1; ++i)
#pragma unroll
    for (int f = 0; f < FB; ++f)
      bq[i][f] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rg, lo, (f * KC + min(i, KC - 1)) * 1024, 0));
  const char* arow = lds + lr * rowb + 16 * lg;
  uint4 av[2][FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) av[0][fm] = *(const uint4*)(arow + fm * 16 * rowb);
  // steady state, U steps per iteration, U a multiple of PF and of 2, so step
  // kc uses bq[kc % PF] = bq[J % PF] and av[kc & 1] = av[J & 1]
  constexpr int U = Unroll<PF>::value;
  const int KF = KC - KC % U;
  for (int kc0 = 0; kc0 < KF; kc0 += U) KSteps<P, FM, FB, PF, 0, U>::run(rg, lo, KC, arow, rowb, kc0, bq, av, acc);
  // tail: the KC - KF < U remaining steps, same slot rule (KF is a multiple of U)
  if (KF < KC) KSteps<P, FM, FB, PF, 0, U>::tail(rg, lo, KC, arow, rowb, KF, bq, av, acc);
}

// Master registers -> LDS tile (the next contraction's A operand). BF16
// tiles take sc z rounded to BF16 (sc = -alpha_t where the step is folded
// into the operand, else 1); FP32 tiles take z itself. zm: float[4] or
// f32x4 elements, [NP][FM][FB].
template <int P, int FM, int FB, int NP, int WC, typename M>
__device__ __forceinline__ void master_to_lds(const M& zm, char* lds, int rowb, int npass, int m_pad, int wave,
                                              int lane, float sc = 1.f) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int slab = WC * p + wave;
    if (p < npass && slab * 16 * FB < m_pad) {
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const int col = 16 * FB * slab + 16 * f + lr;
          char* dst = lds + (16 * fm + 4 * lg) * rowb + col * Elem<P>::bytes;
          if constexpr (P == kF32) {
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) *(float*)(dst + r4 * rowb) = zm[p][fm][f][r4];
          } else {
            // rows r4 and r4 + 1 converted by one packed instruction
#pragma unroll
            for (int r2 = 0; r2 < 4; r2 += 2) {
              const f32x2 v = {sc * zm[p][fm][f][r2], sc * zm[p][fm][f][r2 + 1]};
              const bf16x2 b = __builtin_convertvector(v, bf16x2);
              *(__bf16*)(dst + r2 * rowb) = b[0];
              *(__bf16*)(dst + (r2 + 1) * rowb) = b[1];
            }
          }
        }
    }
  }
}

// Per-row objective of the tile from per-lane partials: reduce over the 16
// lanes of a row group, then over the WC column waves (fixed order), add
// 1/2 ||x||^2. Rows of this wave start at rbase within the R-row tile.
template <int FM, int R, int WC>
__device__ __forceinline__ void finish_rows(const float (&fs)[FM][4], float* red, int wc, int rbase, int lane,
                                            int tid, int row0, int N, const double* xsq, float* Fout, double* Fd) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      float v = fs[fm][r4];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if (lr == 0) red[wc * R + rbase + 16 * fm + 4 * lg + r4] = v;
    }
  __syncthreads();
  if (tid < R && row0 + tid < N) {
    double cs = (double)red[tid];
#pragma unroll
    for (int w = 1; w < WC; ++w) cs += red[w * R + tid];
    const double s = 0.5 * xsq[row0 + tid] + cs;
    if (Fout) Fout[row0 + tid] = (float)s;
    if (Fd) Fd[row0 + tid] = s;
  }
  __syncthreads();
}

// Loads this wave's 16 FM rows (from row0) of `src` ([N][m_pad] FP32) into
// the master registers; rows past N read as 0.
template <int FM, int FB, int NP, int WC>
__device__ __forceinline__ void load_master(float (&zm)[NP][FM][FB][4], const float* src, int row0, int N,
                                            int m_pad, int npass, int wave, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  constexpr int R = FM * 16;
  const int nrows = (N - row0) < R ? (N - row0) : R;
  const Rsrc rs = make_rsrc(src + (size_t)row0 * m_pad, (size_t)nrows * m_pad * 4);
  const int rstride = m_pad * 4;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int slab = WC * p + wave;
    const bool act = p < npass && slab * 16 * FB < m_pad;
    const int lo = (4 * lg * m_pad + 16 * FB * slab + lr) * 4;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const bool ok = act && (16 * fm + 4 * lg + r4) < nrows;
#pragma unroll
        for (int f = 0; f < FB; ++f)
          zm[p][fm][f][r4] = ok ? bload(rs, lo + 64 * f, (16 * fm + r4) * rstride) : 0.f;
      }
  }
}

// Loads this wave's FM row blocks (from row0) of a kept iterate (tape order)
// into the master registers; 4-row groups past N read as 0 (and the rows
// past N inside the last group hold 0 on the tape).
template <int FM, int FB, int NP, int WC, typename M>
__device__ __forceinline__ void load_master_tape(M& zm, const float* src, int row0, int N, int m_pad, int npass,
                                                 int wave, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  constexpr int R = FM * 16;
  const int nrows = (N - row0) < R ? (N - row0) : R;
  const Rsrc rs = make_rsrc(src + (size_t)row0 * m_pad, tape_bytes(nrows, m_pad));
  const int rstride = m_pad * 4;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int slab = WC * p + wave;
    const bool act = p < npass && slab * 16 * FB < m_pad;
    const int lt = (lg * m_pad + 16 * FB * slab + lr) * 16;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const bool ok = act && (16 * fm + 4 * lg) < nrows;
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const float4 q = ok ? bload4(rs, lt + 256 * f, 16 * fm * rstride) : make_float4(0.f, 0.f, 0.f, 0.f);
        zm[p][fm][f][0] = q.x;
        zm[p][fm][f][1] = q.y;
        zm[p][fm][f][2] = q.z;
        zm[p][fm][f][3] = q.w;
      }
    }
  }
}

// z^T of this wave's rows (from row0, in the master layout) into the caller's
// [N][m] buffer: rows below N, columns below m.
template <int FM, int FB, int NP, int WC, typename M>
__device__ __forceinline__ void store_user(const M& zm, const PersistArgs& g, int row0, int wave, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  const int m = g.m, m_pad = g.m_pad, npass = (m_pad + 255) / 256;
  const int nrows = (g.N - row0) < 16 * FM ? (g.N - row0) : 16 * FM;
  const Rsrc rZu = make_rsrc(g.Zuser + (size_t)row0 * m, (size_t)nrows * m * 4);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int slab = WC * p + wave;
    if (!(p < npass && slab * 16 * FB < m_pad)) continue;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int row = 16 * fm + 4 * lg + r4;
        if (row >= nrows) continue;
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const int col = 16 * FB * slab + 16 * f + lr;
          if (col < m) bstore(zm[p][fm][f][r4], rZu, (row * m + col) * 4, 0);
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Forward layers with the step folded into the A operand (BF16 tiles).
//
// The LDS tile holds BF16(-alpha_t z^t) and the accumulators start from the
// FP32 master z^t, so one contraction leaves z^t - alpha_t G z^t in them and
// the epilogue only adds alpha_t c before the threshold:
//   z^{t+1} = ST(acc + alpha_t c, lam alpha_t),  acc = z^t + G BF16(-alpha_t z^t).
// This is the layer of Eq. (14) with the product alpha_t (G z^t) formed
// from the BF16 operand -alpha_t z^t rather than from alpha_t times G BF16(z^t):
// the operand's rounding (2^-9 relative) dominates either way. Without the
// objective trace the accumulators are the master iterate itself, so a wave
// can hold the accumulators of all its column passes at once and run them
// in one contraction that reads each A fragment from LDS once per K step
// instead of once per pass and K step.

// Column passes of this wave (a prefix of 0 .. NP-1): pass p is active while
// p < npass and its slab starts below m_pad.
template <int FB, int NP, int WC>
__device__ __forceinline__ int wave_passes(int m_pad, int wave) {
  const int npass = (m_pad + 255) / 256;
  int na = 0;
#pragma unroll
  for (int p = 0; p < NP; ++p)
    if (p < npass && (WC * p + wave) * 16 * FB < m_pad) na = p + 1;
  return na;
}

// One K step over passes P0 .. P0 + NA - 1: prefetch the G fragments of step
// kc + PF - 1 and the A fragments of step kc + 1 (clamped to the last step),
// then NA FM FB MFMAs into the master accumulators. goff[q]: byte offset of
// pass q's first fragment (a pass past the wave's last active one reads the
// last active pass's fragments: valid memory, and its accumulators are not
// used).
template <int FM, int FB, int NP, int P0, int NA, int PF, int J>
__device__ __forceinline__ void kf_step(const Rsrc& rg, const int (&goff)[NA], int lo, int KC, const char* arow,
                                        int rowb, int kc, uint4 (&bq)[PF][NA][FB], uint4 (&av)[2][FM],
                                        f32x4 (&am)[NP][FM][FB]) {
  const int nk = min(kc + PF - 1, KC - 1);
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int f = 0; f < FB; ++f)
      bq[(J + PF - 1) % PF][q][f] = __builtin_bit_cast(
          uint4, __builtin_amdgcn_raw_buffer_load_b128(rg, lo, goff[q] + (f * KC + nk) * 1024, 0));
  const int na = min(kc + 1, KC - 1);
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) av[(J & 1) ^ 1][fm] = *(const uint4*)(arow + fm * 16 * rowb + na * 64);
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int f = 0; f < FB; ++f)
        am[P0 + q][fm][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[J & 1][fm]),
                                                                    __builtin_bit_cast(bf16x8, bq[J % PF][q][f]),
                                                                    am[P0 + q][fm][f], 0, 0, 0);
  __builtin_amdgcn_sched_barrier(0);
}

template <int FM, int FB, int NP, int P0, int NA, int PF, int J, int U>
struct KFSteps {
  static __device__ __forceinline__ void run(const Rsrc& rg, const int (&goff)[NA], int lo, int KC, const char* arow,
                                             int rowb, int kc0, uint4 (&bq)[PF][NA][FB], uint4 (&av)[2][FM],
                                             f32x4 (&am)[NP][FM][FB]) {
    kf_step<FM, FB, NP, P0, NA, PF, J>(rg, goff, lo, KC, arow, rowb, kc0 + J, bq, av, am);
    KFSteps<FM, FB, NP, P0, NA, PF, J + 1, U>::run(rg, goff, lo, KC, arow, rowb, kc0, bq, av, am);
  }
  static __device__ __forceinline__ void tail(const Rsrc& rg, const int (&goff)[NA], int lo, int KC,
                                              const char* arow, int rowb, int kc0, uint4 (&bq)[PF][NA][FB],
                                              uint4 (&av)[2][FM], f32x4 (&am)[NP][FM][FB]) {
    if (kc0 + J < KC) {
      kf_step<FM, FB, NP, P0, NA, PF, J>(rg, goff, lo, KC, arow, rowb, kc0 + J, bq, av, am);
      KFSteps<FM, FB, NP, P0, NA, PF, J + 1, U>::tail(rg, goff, lo, KC, arow, rowb, kc0, bq, av, am);
    }
  }
};
template <int FM, int FB, int NP, int P0, int NA, int PF, int U>
struct KFSteps<FM, FB, NP, P0, NA, PF, U, U> {
  static __device__ __forceinline__ void run(const Rsrc&, const int (&)[NA], int, int, const char*, int, int,
                                             uint4 (&)[PF][NA][FB], uint4 (&)[2][FM], f32x4 (&)[NP][FM][FB]) {}
  static __device__ __forceinline__ void tail(const Rsrc&, const int (&)[NA], int, int, const char*, int, int,
                                              uint4 (&)[PF][NA][FB], uint4 (&)[2][FM], f32x4 (&)[NP][FM][FB]) {}
};

// am[p] += A G_slab(p) for the passes p = P0 .. P0 + NA - 1 of this wave,
// over the whole K range; na (>= 1, wave-uniform) of them are active. The
// fragments of slab WC p + wave are (FB (WC p + wave) + f, kc), 1 KiB each
// at (FB (WC p + wave) + f) KC + kc KiB.
template <int FM, int FB, int NP, int WC, int P0, int NA, int PF>
__device__ __forceinline__ void contract_fused(const PersistArgs& g, const char* lds, int rowb, int wave, int lane,
                                               int na, f32x4 (&am)[NP][FM][FB]) {
  const int lr = lane & 15, lg = lane >> 4;
  const int KC = g.KC;
  const Rsrc rg = make_rsrc((const char*)g.Gsw + (size_t)(FB * (WC * P0 + wave)) * KC * 1024,
                            (size_t)(WC * FB * (na - 1) + FB) * KC * 1024);
  int goff[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) goff[q] = (q < na ? q : na - 1) * WC * FB * KC * 1024;
  const int lo = lane * 16;
  uint4 bq[PF][NA][FB];
#pragma unroll
  for (int i = 0; i < PF - 1; ++i)
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int f = 0; f < FB; ++f)
        bq[i][q][f] = __builtin_bit_cast(
            uint4, __builtin_amdgcn_raw_buffer_load_b128(rg, lo, goff[q] + (f * KC + min(i, KC - 1)) * 1024, 0));
  const char* arow = lds + lr * rowb + 16 * lg;
  uint4 av[2][FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) av[0][fm] = *(const uint4*)(arow + fm * 16 * rowb);
  // U steps per iteration, a multiple of PF and of 2 (step kc uses bq[kc % PF], av[kc & 1])
  constexpr int U = PF == 3 ? 6 : (PF == 4 ? 4 : 2);
  const int KF = KC - KC % U;
  for (int kc0 = 0; kc0 < KF; kc0 += U)
    KFSteps<FM, FB, NP, P0, NA, PF, 0, U>::run(rg, goff, lo, KC, arow, rowb, kc0, bq, av, am);
  if (KF < KC) KFSteps<FM, FB, NP, P0, NA, PF, 0, U>::tail(rg, goff, lo, KC, arow, rowb, KF, bq, av, am);
}

// The passes of a wave in groups of NG (the G prefetch registers of a group,
// PF NG FB uint4, bound NG): group P0, then P0 + NG, ...; a group with no
// active pass is skipped.
template <int FM, int FB, int NP, int WC, int NG, int PF, int P0>
struct GroupLoop {
  static __device__ __forceinline__ void run(const PersistArgs& g, const char* lds, int rowb, int wave, int lane,
                                             int na_w, f32x4 (&am)[NP][FM][FB]) {
    if constexpr (P0 < NP) {
      constexpr int NA = (NP - P0) < NG ? (NP - P0) : NG;
      if (na_w > P0) contract_fused<FM, FB, NP, WC, P0, NA, PF>(g, lds, rowb, wave, lane, na_w - P0, am);
      GroupLoop<FM, FB, NP, WC, NG, PF, P0 + NG>::run(g, lds, rowb, wave, lane, na_w, am);
    }
  }
};

// After the layers of a forward launch: z^(t_end) for a launch that
// continues the network, then, if asked, one more contraction G z^(t_end)
// for F(z^(t_end)) and the backward seed. The LDS tile holds z^(t_end) in
// the contraction's precision (unscaled); zm: float[4] or f32x4 elements.
template <int P, int R, int NP, int PF, int WR, int WC, typename M>
__device__ __forceinline__ void fwd_tail(const PersistArgs& g, int tile, char* lds, const M& zm) {
  constexpr int FM = R / (16 * WR);
  constexpr int FB = 16 / WC;
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wave = (int)(wid % WC);
  const int rbase = (int)(wid / WC) * 16 * FM;
  const int lr = lane & 15, lg = lane >> 4;
  const int row0 = tile * R;
  const int m_pad = g.m_pad, N = g.N, m = g.m;
  const int rowb = tile_rowb<P>(m_pad);
  const int npass = (m_pad + 255) / 256;
  const int nrows = (N - row0) < R ? (N - row0) : R;
  const int rstride = m_pad * 4;
  const int ustride = m * 4;
  float* red = (float*)(lds + R * rowb);
  const Rsrc rCg = make_rsrc(g.Cg + (size_t)row0 * m_pad, tape_bytes(nrows, m_pad));
  if (g.zsave) {
    // z^(t_end) for a launch that continues the network (tape order)
    const Rsrc rS = make_rsrc(g.zsave + (size_t)row0 * m_pad, tape_bytes(nrows, m_pad));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int slab = WC * p + wave;
      if (!(p < npass && slab * 16 * FB < m_pad)) continue;
      const int lt = (lg * m_pad + 16 * FB * slab + lr) * 16;
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
        if (rbase + 16 * fm + 4 * lg < nrows) {
#pragma unroll
          for (int f = 0; f < FB; ++f)
            bstore4(make_float4(zm[p][fm][f][0], zm[p][fm][f][1], zm[p][fm][f][2], zm[p][fm][f][3]), rS,
                    lt + 256 * f, (rbase + 16 * fm) * rstride);
        }
    }
  }
  if (!(g.mode & (kModeF | kModeSeed))) return;
  // final contraction: F(z^(t_end)) and / or the seed of the backward pass
  const bool want_f = (g.mode & kModeF) != 0;
  const bool seed = (g.mode & kModeSeed) != 0;
  const float lam = g.lam;
  const Rsrc rV = make_rsrc(g.Vout ? g.Vout + (size_t)row0 * m_pad : nullptr, g.Vout ? (size_t)nrows * rstride : 0);
  const Rsrc rdZ = make_rsrc(g.dZ ? g.dZ + (size_t)row0 * m : nullptr, g.dZ ? (size_t)nrows * ustride : 0);
  float fs[FM][4];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) fs[fm][r4] = 0.f;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int slab = WC * p + wave;
    if (!(p < npass && slab * 16 * FB < m_pad)) continue;
    f32x4 acc[FM][FB];
    contract<P, FM, FB, PF>(g, lds + rbase * rowb, rowb, slab, lane, acc);
    const int colb = 16 * FB * slab + lr;
    const int lo = (4 * lg * m_pad + colb) * 4;
    const int lou = (4 * lg * m + colb) * 4;
    const int lt = (lg * m_pad + colb) * 16;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const bool grp = rbase + 16 * fm + 4 * lg < nrows;
      float cg[FB][4];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const float4 q = grp ? bload4(rCg, lt + 256 * f, (rbase + 16 * fm) * rstride) : make_float4(0.f, 0.f, 0.f, 0.f);
        cg[f][0] = q.x;
        cg[f][1] = q.y;
        cg[f][2] = q.z;
        cg[f][3] = q.w;
      }
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int rl = rbase + 16 * fm + 4 * lg + r4;
        if (rl >= nrows) continue;
        const int so = (rbase + 16 * fm + r4) * rstride, sou = (rbase + 16 * fm + r4) * ustride;
        const float w = seed ? (g.dF ? g.dF[row0 + rl] : g.dF_scalar) : 0.f;
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float z = zm[p][fm][f][r4];
          const float c = cg[f][r4];
          const float pv = acc[fm][f][r4];
          if (want_f) fs[fm][r4] += 0.5f * z * pv - z * c + lam * fabsf(z);
          if (seed) {
            float gv = w * (pv - c + lam * sgnf(z));
            if (g.dZ && colb + 16 * f < m) gv += bload(rdZ, lou + 64 * f, sou);
            bstore((z != 0.f) ? gv : 0.f, rV, lo + 64 * f, so);
          }
        }
      }
    }
  }
  if (want_f) finish_rows<FM, R, WC>(fs, red, wave, rbase, lane, tid, row0, N, g.xsq, g.F, g.Fd);
}

// Forward layers [t_begin, t_end) of a BF16 tile without the objective
// trace: the folded layer above, all column passes of a wave in groups of
// NG per contraction (NG FB <= 8 keeps the prefetched G fragments at 32
// registers per stage), G fragments one K step ahead.
template <int P, int R, int NP, int PF, int WR, int WC>
__device__ __forceinline__ void fwd_body_fused(const PersistArgs& g, int tile, char* lds) {
  static_assert(P == kBF16, "the folded layer runs on BF16 tiles");
  constexpr int FM = R / (16 * WR);
  constexpr int FB = 16 / WC;
  constexpr int NG = (8 / FB) < NP ? (8 / FB) : NP;
  constexpr int PFF = 2;
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wave = (int)(wid % WC);
  const int rbase = (int)(wid / WC) * 16 * FM;
  const int lr = lane & 15, lg = lane >> 4;
  const int row0 = tile * R;
  const int m_pad = g.m_pad, N = g.N;
  const int rowb = tile_rowb<P>(m_pad);
  const int npass = (m_pad + 255) / 256;
  const int rstride = m_pad * 4;
  const int na_w = wave_passes<FB, NP, WC>(m_pad, wave);
  // all R rows of the tile: c is stored for tape_rows(N) rows, zeros past N
  const Rsrc rCg = make_rsrc(g.Cg + (size_t)row0 * m_pad, tape_bytes(R, m_pad));

  f32x4 am[NP][FM][FB];  // the master iterate, and the contraction's accumulators
  if (g.t_begin == 0) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f) am[p][fm][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  } else {
    load_master_tape<FM, FB, NP, WC>(am, g.zload ? g.zload : slot_ptr(g, g.t_begin), row0 + rbase, N, m_pad, npass,
                                     wave, lane);
  }
  master_to_lds<P, FM, FB, NP, WC>(am, lds + rbase * rowb, rowb, npass, m_pad, wave, lane,
                                   g.t_begin < g.t_end ? -g.alpha[g.t_begin] : 1.f);
  __syncthreads();

  for (int t = g.t_begin; t < g.t_end; ++t) {
    const float a = g.alpha[t];
    const float th = uniform_f32(g.lam * a);
    const bool store = g.k > 0 && (g.store_all || (t + 1) % g.k == 0 || t + 1 == g.T || t + 1 > g.a_last);
    const Rsrc rD = make_rsrc(store ? slot_ptr(g, t + 1) + (size_t)row0 * m_pad : nullptr,
                              store ? tape_bytes(R, m_pad) : 0);
    // z^0 = 0: layer 0 has nothing to contract
    if (t > 0) GroupLoop<FM, FB, NP, WC, NG, PFF, 0>::run(g, lds + rbase * rowb, rowb, wave, lane, na_w, am);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p >= na_w) {
        // a pass past the wave's last one: its accumulators took other fragments
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int f = 0; f < FB; ++f) am[p][fm][f] = f32x4{0.f, 0.f, 0.f, 0.f};
        continue;
      }
      const int colb = 16 * FB * (WC * p + wave) + lr;  // column of block f = 0
      const int lt = (lg * m_pad + colb) * 16;           // per-lane offset, tape order
      // c of the pass: every load issued before the first use (rows past N
      // read the zeros stored there, and G z is 0 for them, so z stays 0)
      float4 cq[FM][FB];
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f) cq[fm][f] = bload4(rCg, lt + 256 * f, (rbase + 16 * fm) * rstride);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float cv[4] = {cq[fm][f].x, cq[fm][f].y, cq[fm][f].z, cq[fm][f].w};
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) am[p][fm][f][r4] = soft_threshold(fmaf(a, cv[r4], am[p][fm][f][r4]), th);
        }
        // whole tile: the rows past N hold 0 and land in the slot's padding
        if (store) {
#pragma unroll
          for (int f = 0; f < FB; ++f)
            bstore4(make_float4(am[p][fm][f][0], am[p][fm][f][1], am[p][fm][f][2], am[p][fm][f][3]), rD,
                    lt + 256 * f, (rbase + 16 * fm) * rstride);
        }
      }
    }
    __syncthreads();
    master_to_lds<P, FM, FB, NP, WC>(am, lds + rbase * rowb, rowb, npass, m_pad, wave, lane,
                                     t + 1 < g.t_end ? -g.alpha[t + 1] : 1.f);
    __syncthreads();
  }
  if (g.Zuser && g.t_begin < g.t_end && g.t_end == g.T) store_user<FM, FB, NP, WC>(am, g, row0 + rbase, wave, lane);
  fwd_tail<P, R, NP, PF, WR, WC>(g, tile, lds, am);
}

// Forward over layers [t_begin, t_end): z^(t+1) = ST(z^t - a_t (G z^t - c), lam a_t),
// keeping the tape; with TRACE also F(z^t) for each t. Then fwd_tail. One
// contraction per column pass, the master iterate in its own registers;
// BF16 tiles without the trace run fwd_body_fused instead.
// FISTA: the tile also carries y^t (FISTA's extrapolated point) in
// registers; the contraction is G y^t, the epilogue z^{t+1} = ST(y^t -
// alpha_t (G y^t - c), lam alpha_t), y^{t+1} = z^{t+1} + beta_t (z^{t+1} - z^t)
// (the per-layer FISTA epilogue's expressions), and the LDS tile holds y;
// the final contraction for F takes z^T. No tape, no trace.
template <int P, int R, int NP, bool TRACE, int PF, int WR, int WC, bool FISTA = false>
__device__ __forceinline__ void fwd_body(const PersistArgs& g, int tile, char* lds) {
  static_assert(!(FISTA && TRACE), "FISTA runs without the objective trace");
  // the fused layer loop where its accumulators (the whole master) fit in
  // 128 registers per lane next to the operands of a K step
  if constexpr (P == kBF16 && !TRACE && !FISTA && NP * (R / (16 * WR)) * (16 / WC) * 4 <= 128) {
    fwd_body_fused<P, R, NP, PF, WR, WC>(g, tile, lds);
    return;
  } else {
  // BF16 Step-LISTA / ISTA layers use the folded form (see fwd_body_fused);
  // FP32 layers and FISTA form z - alpha_t (P - c) from P = G z.
  constexpr bool FOLD = P == kBF16 && !FISTA;
  constexpr int FM = R / (16 * WR);  // 16-row blocks per wave
  constexpr int FB = 16 / WC;        // 16-column blocks per wave and pass
  const int tid = threadIdx.x, lane = tid & 63;
  // wave-uniform, and known to be: descriptors built from it stay in SGPRs
  const unsigned wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wave = (int)(wid % WC);              // column wave: slab WC p + wave of pass p
  const int rbase = (int)(wid / WC) * 16 * FM;   // first tile row of this wave
  const int lr = lane & 15, lg = lane >> 4;
  const int row0 = tile * R;
  const int m_pad = g.m_pad, N = g.N;
  const int rowb = tile_rowb<P>(m_pad);
  const int npass = (m_pad + 255) / 256;
  const int rstride = m_pad * 4;      // bytes per row of the [N][m_pad] buffers
  float* red = (float*)(lds + R * rowb);
  // all R rows of the tile: c is stored for tape_rows(N) rows, zeros past N
  const Rsrc rCg = make_rsrc(g.Cg + (size_t)row0 * m_pad, tape_bytes(R, m_pad));

  float zm[NP][FM][FB][4];
  float ym[FISTA ? NP : 1][FM][FB][4];  // FISTA's y^t (z^0 = y^0 = 0; t_begin = 0)
  if constexpr (FISTA) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) ym[p][fm][f][r4] = 0.f;
  }
  if (g.t_begin == 0) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) zm[p][fm][f][r4] = 0.f;
  } else {
    load_master_tape<FM, FB, NP, WC>(zm, g.zload ? g.zload : slot_ptr(g, g.t_begin), row0 + rbase, N, m_pad, npass,
                                     wave, lane);
  }
  master_to_lds<P, FM, FB, NP, WC>(zm, lds + rbase * rowb, rowb, npass, m_pad, wave, lane,
                                   FOLD && g.t_begin < g.t_end ? -g.alpha[g.t_begin] : 1.f);
  __syncthreads();

  for (int t = g.t_begin; t < g.t_end; ++t) {
    const float a = g.alpha[t];
    const float lam = g.lam, th = uniform_f32(lam * a);
    const float bt = FISTA ? g.beta[t] : 0.f;
    const bool store = g.k > 0 && (g.store_all || (t + 1) % g.k == 0 || t + 1 == g.T || t + 1 > g.a_last);
    const Rsrc rD = make_rsrc(store ? slot_ptr(g, t + 1) + (size_t)row0 * m_pad : nullptr,
                              store ? tape_bytes(R, m_pad) : 0);
    float fs[FM][4];
    if constexpr (TRACE) {
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) fs[fm][r4] = 0.f;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int slab = WC * p + wave;
      if (!(p < npass && slab * 16 * FB < m_pad)) continue;
      f32x4 acc[FM][FB];
      if constexpr (FOLD) {
        // the accumulators start from z^t
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int f = 0; f < FB; ++f)
            acc[fm][f] = f32x4{zm[p][fm][f][0], zm[p][fm][f][1], zm[p][fm][f][2], zm[p][fm][f][3]};
        if (t > 0) contract<P, FM, FB, PF, true>(g, lds + rbase * rowb, rowb, slab, lane, acc);
      } else if (t > 0) {
        contract<P, FM, FB, PF>(g, lds + rbase * rowb, rowb, slab, lane, acc);
      } else {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int f = 0; f < FB; ++f) acc[fm][f] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      const int colb = 16 * FB * slab + lr;            // column of block f = 0
      const int lt = (lg * m_pad + colb) * 16;         // per-lane offset, tape order
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        // c of this lane's four rows, one 16-byte load per column block;
        // rows past N keep z = 0 (their c is stored as 0, and G z is 0)
        float cg[FB][4];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float4 q = bload4(rCg, lt + 256 * f, (rbase + 16 * fm) * rstride);
          cg[f][0] = q.x;
          cg[f][1] = q.y;
          cg[f][2] = q.z;
          cg[f][3] = q.w;
        }
        // (rows past N: every term is 0, and their objective partials are not used)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
#pragma unroll
          for (int f = 0; f < FB; ++f) {
            const float z = zm[p][fm][f][r4];
            const float c = cg[f][r4];
            float zn;
            if constexpr (FOLD) {
              // acc = z - a G z: G z = (z - acc) / a for the objective
              const float q = acc[fm][f][r4];
              if constexpr (TRACE) fs[fm][r4] += 0.5f * z * ((z - q) / a) - z * c + lam * fabsf(z);
              zn = soft_threshold(fmaf(a, c, q), th);
            } else if constexpr (FISTA) {
              const float pv = acc[fm][f][r4];
              const float y = ym[p][fm][f][r4];
              zn = soft_threshold(y - a * (pv - c), th);
              ym[p][fm][f][r4] = zn + bt * (zn - z);
            } else {
              const float pv = acc[fm][f][r4];
              if constexpr (TRACE) fs[fm][r4] += 0.5f * z * pv - z * c + lam * fabsf(z);
              zn = soft_threshold(z - a * (pv - c), th);
            }
            zm[p][fm][f][r4] = zn;
          }
        }
        // whole tile: the rows past N hold 0 and land in the slot's padding
        if (store) {
#pragma unroll
          for (int f = 0; f < FB; ++f)
            bstore4(make_float4(zm[p][fm][f][0], zm[p][fm][f][1], zm[p][fm][f][2], zm[p][fm][f][3]), rD,
                    lt + 256 * f, (rbase + 16 * fm) * rstride);
        }
      }
      // keep the next pass's loads after this pass (registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (TRACE)
      finish_rows<FM, R, WC>(fs, red, wave, rbase, lane, tid, row0, N, g.xsq, g.Ftrace + (size_t)t * N, nullptr);
    __syncthreads();
    if constexpr (FISTA)
      master_to_lds<P, FM, FB, NP, WC>(ym, lds + rbase * rowb, rowb, npass, m_pad, wave, lane);
    else
      master_to_lds<P, FM, FB, NP, WC>(zm, lds + rbase * rowb, rowb, npass, m_pad, wave, lane,
                                       FOLD && t + 1 < g.t_end ? -g.alpha[t + 1] : 1.f);
    __syncthreads();
  }
  if (g.Zuser && g.t_begin < g.t_end && g.t_end == g.T) store_user<FM, FB, NP, WC>(zm, g, row0 + rbase, wave, lane);
  if constexpr (FISTA) {
    // the LDS tile holds y^T; F takes z^T (every wave is past the last barrier)
    if (g.mode & (kModeF | kModeSeed)) {
      master_to_lds<P, FM, FB, NP, WC>(zm, lds + rbase * rowb, rowb, npass, m_pad, wave, lane);
      __syncthreads();
    }
  }
  fwd_tail<P, R, NP, PF, WR, WC>(g, tile, lds, zm);
  }
}


template <int P, int R, int NP, int PF, int WR, int WC>
__device__ __forceinline__ void bwd_body(const PersistArgs& g, int tile, char* lds) {
  constexpr int FM = R / (16 * WR);  // 16-row blocks per wave
  constexpr int FB = 16 / WC;        // 16-column blocks per wave and pass
  const int tid = threadIdx.x, lane = tid & 63;
  // wave-uniform, and known to be: descriptors built from it stay in SGPRs
  const unsigned wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wave = (int)(wid % WC);              // column wave: slab WC p + wave of pass p
  const int rbase = (int)(wid / WC) * 16 * FM;   // first tile row of this wave
  const int lr = lane & 15, lg = lane >> 4;
  const int row0 = tile * R;
  const int m_pad = g.m_pad, N = g.N;
  const int rowb = tile_rowb<P>(m_pad);
  const int npass = (m_pad + 255) / 256;
  const int nrows = (N - row0) < R ? (N - row0) : R;
  const int rstride = m_pad * 4;
  double* dred = (double*)(lds + R * rowb);

  float vm[NP][FM][FB][4];
  load_master<FM, FB, NP, WC>(vm, g.Vio, row0 + rbase, N, m_pad, npass, wave, lane);
  master_to_lds<P, FM, FB, NP, WC>(vm, lds + rbase * rowb, rowb, npass, m_pad, wave, lane);

  // The step-size partial of layer t is sum v^t (z^t - z^{t+1}). Its second
  // part, s2 = sum v^t z^{t+1}, is accumulated when v^t is formed (one layer
  // earlier, with z^{t+1} already loaded there), so each layer reads only
  // z^t. The products of two floats are exact in FP64; only the sums round.
  // For the first layer of the launch, s2 comes from one pass over z^{t_hi+1}.
  double s2 = 0.0;
  {
    const Rsrc rz1 = make_rsrc(slot_ptr(g, g.t_hi + 1) + (size_t)row0 * m_pad, tape_bytes(nrows, m_pad));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int slab = WC * p + wave;
      if (!(p < npass && slab * 16 * FB < m_pad)) continue;
      const int lt = (lg * m_pad + 16 * FB * slab + lr) * 16;
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        if (rbase + 16 * fm + 4 * lg >= nrows) continue;  // rows past N inside a group hold 0
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float4 z1 = bload4(rz1, lt + 256 * f, (rbase + 16 * fm) * rstride);
          s2 += (double)vm[p][fm][f][0] * (double)z1.x;
          s2 += (double)vm[p][fm][f][1] * (double)z1.y;
          s2 += (double)vm[p][fm][f][2] * (double)z1.z;
          s2 += (double)vm[p][fm][f][3] * (double)z1.w;
        }
      }
    }
  }
  __syncthreads();

  for (int t = g.t_hi; t >= g.t_lo; --t) {
    const float a = g.alpha[t];
    // all R rows of the tile (a slot holds tape_rows(N) rows; groups past N
    // are not written, so their loads are discarded below)
    const Rsrc rz0 = make_rsrc(t >= 1 ? slot_ptr(g, t) + (size_t)row0 * m_pad : nullptr,
                               t >= 1 ? tape_bytes(R, m_pad) : 0);
    double dsum = -s2;
    s2 = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int slab = WC * p + wave;
      if (!(p < npass && slab * 16 * FB < m_pad)) continue;
      f32x4 acc[FM][FB];
      if (t >= 1) contract<P, FM, FB, PF>(g, lds + rbase * rowb, rowb, slab, lane, acc);
      const int lt = (lg * m_pad + 16 * FB * slab + lr) * 16;
      if (t >= 1) {
        // z^t of the pass, every load issued before the first is used; row
        // groups past N are taken as 0 (v is 0 there too, so they add nothing)
        float4 zq[FM][FB];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int f = 0; f < FB; ++f) zq[fm][f] = bload4(rz0, lt + 256 * f, (rbase + 16 * fm) * rstride);
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
          if (rbase + 16 * fm + 4 * lg >= nrows) {
#pragma unroll
            for (int f = 0; f < FB; ++f) zq[fm][f] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
          for (int f = 0; f < FB; ++f) {
            const float4 z4 = zq[fm][f];
            const float zz[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const float v = vm[p][fm][f][r4];
              const float z0 = zz[r4];
              dsum += (double)v * (double)z0;
              const float vn = (z0 != 0.f) ? v - a * acc[fm][f][r4] : 0.f;
              vm[p][fm][f][r4] = vn;
              s2 += (double)vn * (double)z0;
            }
          }
        }
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dsum += __shfl_xor(dsum, o);
    if (lane == 0) dred[wid] = dsum;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < WC * WR; ++w) tot += dred[w];
      g.dpart[(size_t)t * g.P_stride + tile] = tot;
    }
    if (t >= 1 && t > g.t_lo) master_to_lds<P, FM, FB, NP, WC>(vm, lds + rbase * rowb, rowb, npass, m_pad, wave, lane);
    __syncthreads();
  }
  if (g.t_lo >= 1) {
    const Rsrc rv = make_rsrc(g.Vio + (size_t)row0 * m_pad, (size_t)nrows * rstride);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int slab = WC * p + wave;
      if (!(p < npass && slab * 16 * FB < m_pad)) continue;
      const int lo = (4 * lg * m_pad + 16 * FB * slab + lr) * 4;
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          if (rbase + 16 * fm + 4 * lg + r4 >= nrows) continue;
#pragma unroll
          for (int f = 0; f < FB; ++f) bstore(vm[p][fm][f][r4], rv, lo + 64 * f, (rbase + 16 * fm + r4) * rstride);
        }
    }
  }
}

// Single problem: workgroup b carries tile b.
template <int P, int R, int NP, bool TRACE, int PF, int OCC, int WR, int WC>
__global__ __launch_bounds__(64 * WC * WR, OCC) void fwd_persist(PersistArgs g) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  fwd_body<P, R, NP, TRACE, PF, WR, WC>(g, blockIdx.x, lds);
}

template <int P, int R, int NP, int PF, int OCC, int WR, int WC>
__global__ __launch_bounds__(64 * WC * WR, OCC) void fista_persist(PersistArgs g) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  fwd_body<P, R, NP, false, PF, WR, WC, true>(g, blockIdx.x, lds);
}

template <int P, int R, int NP, int PF, int OCC, int WR, int WC>
__global__ __launch_bounds__(64 * WC * WR, OCC) void bwd_persist(PersistArgs g) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  bwd_body<P, R, NP, PF, WR, WC>(g, blockIdx.x, lds);
}

// Several problems in one launch: workgroup b carries tile work[b].y of
// problem work[b].x, whose arguments are tab[work[b].x] with the layer range
// and mode of this launch (ph) filled in. The work list is ordered longest
// tile first.
__device__ __forceinline__ PersistArgs batched_args(const PersistArgs* tab, const int2* work, const PersistPhase& ph,
                                                    int& tile) {
  const int2 w = work[blockIdx.x];
  PersistArgs g = tab[w.x];
  g.t_begin = ph.t_begin;
  g.t_end = ph.t_end;
  g.mode = ph.mode & g.mode_mask;
  g.store_all = ph.store_all;
  g.t_hi = ph.t_hi;
  g.t_lo = ph.t_lo;
  tile = w.y;
  return g;
}

template <int P, int R, int NP, int PF, int OCC, int WR, int WC>
__global__ __launch_bounds__(64 * WC * WR, OCC) void fwd_persist_batched(const PersistArgs* tab, const int2* work,
                                                                          PersistPhase ph) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  int tile;
  const PersistArgs g = batched_args(tab, work, ph, tile);
  fwd_body<P, R, NP, false, PF, WR, WC>(g, tile, lds);
}

template <int P, int R, int NP, int PF, int OCC, int WR, int WC>
__global__ __launch_bounds__(64 * WC * WR, OCC) void bwd_persist_batched(const PersistArgs* tab, const int2* work,
                                                                          PersistPhase ph) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  int tile;
  const PersistArgs g = batched_args(tab, work, ph, tile);
  bwd_body<P, R, NP, PF, WR, WC>(g, tile, lds);
}

// LDS of a tile: the A operand rows plus the per-wave row partials.
template <int P, int R, int WC>
size_t tile_lds(int m_pad) {
  return (size_t)R * tile_rowb<P>(m_pad) + (size_t)WC * R * sizeof(float) + 64;
}

template <int P, int R, int NP, int PF, int OCC, int WR = 1, int WC = 4>
hipError_t launch_pair(bool fwd, const PersistArgs& a, hipStream_t s) {
  const int tiles = (a.N + R - 1) / R;
  if (tiles == 0) return hipSuccess;
  const size_t lds = tile_lds<P, R, WC>(a.m_pad);
  const bool trace = fwd && (a.mode & kModeTrace);
  const void* fn = !fwd ? (const void*)bwd_persist<P, R, NP, PF, OCC, WR, WC>
                        : trace ? (const void*)fwd_persist<P, R, NP, true, PF, OCC, WR, WC>
                                : (const void*)fwd_persist<P, R, NP, false, PF, OCC, WR, WC>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 block(64 * WC * WR);
  if (!fwd)
    hipLaunchKernelGGL((bwd_persist<P, R, NP, PF, OCC, WR, WC>), dim3(tiles), block, lds, s, a);
  else if (trace)
    hipLaunchKernelGGL((fwd_persist<P, R, NP, true, PF, OCC, WR, WC>), dim3(tiles), block, lds, s, a);
  else
    hipLaunchKernelGGL((fwd_persist<P, R, NP, false, PF, OCC, WR, WC>), dim3(tiles), block, lds, s, a);
  return hipGetLastError();
}

template <int P, int R, int NP, int PF, int OCC, int WR = 1, int WC = 4>
hipError_t launch_fista(const PersistArgs& a, hipStream_t s) {
  const int tiles = (a.N + R - 1) / R;
  if (tiles == 0) return hipSuccess;
  const size_t lds = tile_lds<P, R, WC>(a.m_pad);
  hipError_t e = hipFuncSetAttribute((const void*)fista_persist<P, R, NP, PF, OCC, WR, WC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fista_persist<P, R, NP, PF, OCC, WR, WC>), dim3(tiles), dim3(64 * WC * WR), lds, s, a);
  return hipGetLastError();
}

template <int P, int R, int NP, int PF, int OCC, int WR = 1, int WC = 4>
hipError_t launch_pair_batched(bool fwd, const PersistArgs* tab, const int2* work, int nwork, int max_m_pad,
                               const PersistPhase& ph, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  const size_t lds = tile_lds<P, R, WC>(max_m_pad);
  const void* fn = fwd ? (const void*)fwd_persist_batched<P, R, NP, PF, OCC, WR, WC>
                       : (const void*)bwd_persist_batched<P, R, NP, PF, OCC, WR, WC>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 block(64 * WC * WR);
  if (fwd)
    hipLaunchKernelGGL((fwd_persist_batched<P, R, NP, PF, OCC, WR, WC>), dim3(nwork), block, lds, s, tab, work, ph);
  else
    hipLaunchKernelGGL((bwd_persist_batched<P, R, NP, PF, OCC, WR, WC>), dim3(nwork), block, lds, s, tab, work, ph);
  return hipGetLastError();
}

}  // namespace
}  // namespace slista
