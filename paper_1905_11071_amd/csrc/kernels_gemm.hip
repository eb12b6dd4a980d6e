// Fused MFMA contraction for one unfolded-ISTA layer (forward or adjoint).
//
// Every layer of Step-LISTA (Eq. (14)) computes, for all samples of the
// batch at once, the Gram-form gradient G z - c, i.e. one dense product
// P = Z G with Z [N, m_pad] (sample-major) and G = D^T D [m_pad, m_pad]
// (symmetric, so G itself is the K-contiguous "B^T"). The product runs on the
// gfx950 matrix cores, and the elementwise rest of the layer is applied to
// the accumulators before anything is written back:
//   forward  u = z - a (P - c), z' = ST(u, lam a), objective partials (Eq. (1));
//   backward v' = [z^t != 0] (v - a P) and the partial of d loss / d a_t.
//
// Tiling (one workgroup = 4 wave64s, 2 x 2):
//   workgroup tile 128 samples x 128 coordinates, wave tile 64 x 64 made of
//   4 x 4 blocks of 16 x 16 accumulators; K is staged through LDS in steps of
//   128 bytes per row (32 FP32 or 64 BF16 values), double buffered, with the
//   next step's global loads issued before the current step's MFMAs.
//   FP32: v_mfma_f32_16x16x4_f32, 4 per 16-byte operand read.
//   BF16: v_mfma_f32_16x16x32_bf16, 1 per 16-byte operand read; z is rounded
//         to BF16 (RNE, v_cvt_pk_bf16_f32) while it is staged into LDS, so no
//         separate BF16 copy of the iterates is ever stored.
//   Each lane reads 16 contiguous bytes of one LDS row; rows are 144 bytes
//   apart, which spreads the 8 lanes of each ds_read_b128 phase over
//   distinct banks.
//   Tiles are handed out XCD-contiguously: workgroup b runs on XCD b % 8, so
//   tile (b % 8) * tiles_per_xcd + b / 8 keeps the column tiles of one row
//   block, which read the same rows of Z, c and z, inside one XCD's L2.
#include "common.hpp"

namespace slista {
namespace {

constexpr int BM = 128, BN = 128, NTHREADS = 256;
constexpr int S = 2;                 // 64-byte chunks per LDS row per stage
constexpr int ROWB = S * 64 + 16;    // LDS row stride in bytes
constexpr int A_BYTES = BM * ROWB;
constexpr int B_BYTES = BN * ROWB;
constexpr int STAGE_BYTES = A_BYTES + B_BYTES;

template <int P> struct KStep;
template <> struct KStep<kF32> { static constexpr int KS = S * 16; };
template <> struct KStep<kBF16> { static constexpr int KS = S * 32; };

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  uint16_t a = __builtin_bit_cast(uint16_t, (__bf16)lo);
  uint16_t b = __builtin_bit_cast(uint16_t, (__bf16)hi);
  return (uint32_t)a | ((uint32_t)b << 16);
}

template <int P> struct StageRegs;
template <> struct StageRegs<kF32> { float4 a[4]; uint4 b[4]; };
template <> struct StageRegs<kBF16> { float4 a[8]; uint4 b[4]; };

// Global -> registers for one K step. Thread (r = tid / 8, q = tid % 8)
// covers rows r, r+32, r+64, r+96 of both tiles and 16-byte quad q of the
// 128-byte LDS row segment.
template <int P, bool SAFE>
__device__ __forceinline__ void load_stage(StageRegs<P>& st, const GemmArgs& g, int row0, int col0,
                                           int k0, int tid) {
  const int q = tid & 7, r = tid >> 3;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int row = row0 + r + 32 * p;
    const int col = col0 + r + 32 * p;
    if constexpr (P == kF32) {
      if constexpr (SAFE) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + 4 * q + e;
          v[e] = (row < g.rows && k < g.K) ? g.A[(size_t)row * g.lda + k] : 0.f;
        }
        st.a[p] = make_float4(v[0], v[1], v[2], v[3]);
        const float* B = (const float*)g.Bt;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + 4 * q + e;
          v[e] = (col < g.ncols && k < g.K) ? B[(size_t)col * g.ldb + k] : 0.f;
        }
        st.b[p] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                             __float_as_uint(v[3]));
      } else {
        st.a[p] = row < g.rows ? *(const float4*)(g.A + (size_t)row * g.lda + k0 + 4 * q)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
        st.b[p] = col < g.ncols
                      ? *(const uint4*)((const float*)g.Bt + (size_t)col * g.ldb + k0 + 4 * q)
                      : make_uint4(0, 0, 0, 0);
      }
    } else {
      if (row < g.rows) {
        const float* src = g.A + (size_t)row * g.lda + k0 + 8 * q;
        st.a[2 * p] = *(const float4*)src;
        st.a[2 * p + 1] = *(const float4*)(src + 4);
      } else {
        st.a[2 * p] = make_float4(0.f, 0.f, 0.f, 0.f);
        st.a[2 * p + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      st.b[p] = col < g.ncols
                    ? *(const uint4*)((const uint16_t*)g.Bt + (size_t)col * g.ldb + k0 + 8 * q)
                    : make_uint4(0, 0, 0, 0);
    }
  }
}

// SCALE: the BF16 A operand is sc z (the folded forward layer, sc = -alpha_t).
template <int P, bool SCALE = false>
__device__ __forceinline__ void store_stage(const StageRegs<P>& st, char* buf, int tid, float sc = 1.f) {
  const int q = tid & 7, r = tid >> 3;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int off = (r + 32 * p) * ROWB + 16 * q;
    if constexpr (P == kF32) {
      *(float4*)(buf + off) = st.a[p];
    } else {
      float4 lo = st.a[2 * p], hi = st.a[2 * p + 1];
      if constexpr (SCALE) {
        lo = make_float4(sc * lo.x, sc * lo.y, sc * lo.z, sc * lo.w);
        hi = make_float4(sc * hi.x, sc * hi.y, sc * hi.z, sc * hi.w);
      }
      *(uint4*)(buf + off) = make_uint4(pack_bf16x2(lo.x, lo.y), pack_bf16x2(lo.z, lo.w),
                                        pack_bf16x2(hi.x, hi.y), pack_bf16x2(hi.z, hi.w));
    }
    *(uint4*)(buf + A_BYTES + off) = st.b[p];
  }
}

template <int P>
__device__ __forceinline__ void compute_stage(const char* buf, f32x4 (&acc)[4][4], int wm, int wn,
                                              int lr, int lg) {
#pragma unroll
  for (int c = 0; c < S; ++c) {
    uint4 av[4], bv[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      av[f] = *(const uint4*)(buf + (wm * 64 + f * 16 + lr) * ROWB + 64 * c + 16 * lg);
      bv[f] = *(const uint4*)(buf + A_BYTES + (wn * 64 + f * 16 + lr) * ROWB + 64 * c + 16 * lg);
    }
    if constexpr (P == kF32) {
      // K sub-step e outermost: consecutive MFMAs update independent accumulators
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int fm = 0; fm < 4; ++fm)
#pragma unroll
          for (int fn = 0; fn < 4; ++fn) {
            const uint32_t ae = e == 0 ? av[fm].x : e == 1 ? av[fm].y : e == 2 ? av[fm].z : av[fm].w;
            const uint32_t be = e == 0 ? bv[fn].x : e == 1 ? bv[fn].y : e == 2 ? bv[fn].z : bv[fn].w;
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(ae), __uint_as_float(be),
                                                                acc[fm][fn], 0, 0, 0);
          }
    } else {
#pragma unroll
      for (int fm = 0; fm < 4; ++fm)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[fm]),
                                                                 __builtin_bit_cast(bf16x8, bv[fn]),
                                                                 acc[fm][fn], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// One output tile of a fused contraction (the tile index already mapped).
template <int P, int EPI, bool SAFE>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int tile, char* smem) {
  const int rt = tile / g.col_tiles, ct = tile - rt * g.col_tiles;
  const int row0 = rt * BM, col0 = ct * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  const float a = (EPI == kEpiCorr) ? 0.f : g.alpha ? g.alpha[g.t] : 0.f;
  // The BF16 forward layer folds the step into the operand, as the
  // persistent kernels do: A = BF16(-a z^t), the accumulators start from z^t
  // (so they end as z^t - a G z^t), and the epilogue adds a c.
  constexpr bool FOLD = EPI == kEpiFwd && P == kBF16;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (FOLD) {
        const int col = col0 + wn * 64 + j * 16 + lr;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int row = row0 + wm * 64 + i * 16 + 4 * lg + r4;
          if (row < g.rows && col < g.ncols) acc[i][j][r4] = g.Zt[(size_t)row * g.ldz + col];
        }
      }
    }

  constexpr int KS = KStep<P>::KS;
  const int nk = (g.K + KS - 1) / KS;
  StageRegs<P> st;
  load_stage<P, SAFE>(st, g, row0, col0, 0, tid);
  store_stage<P, FOLD>(st, smem, tid, -a);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const bool more = kt + 1 < nk;
    if (more) load_stage<P, SAFE>(st, g, row0, col0, (kt + 1) * KS, tid);
    compute_stage<P>(smem + (kt & 1) * STAGE_BYTES, acc, wm, wn, lr, lg);
    if (more) store_stage<P, FOLD>(st, smem + ((kt + 1) & 1) * STAGE_BYTES, tid, -a);
    __syncthreads();
  }

  // ------------------------------------------------------------ epilogue
  const float lam = g.lam;
  const float th = uniform_f32(lam * a);
  const float bt = (EPI == kEpiFista) ? g.beta[g.t] : 0.f;
  const float lth = (EPI == kEpiLista) ? lam * g.beta[g.t] : 0.f;  // LISTA threshold lam beta_t
  double fs[4][4];
  double dsum = 0.0;
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) fs[fm][r4] = 0.0;

#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int row = row0 + wm * 64 + fm * 16 + 4 * lg + r4;
      if (row >= g.rows) continue;
      float w = 0.f;
      if constexpr (EPI == kEpiSeed) w = g.dF ? g.dF[row] : g.dF_scalar;
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        const int col = col0 + wn * 64 + fn * 16 + lr;
        if (col >= g.ncols) continue;
        const size_t idx = (size_t)row * g.ldz + col;
        const float p = acc[fm][fn][r4];
        if constexpr (EPI == kEpiCorr || EPI == kEpiSplit) {
          g.Out[idx] = p;
        } else if constexpr (EPI == kEpiResid) {
          const float r = p - g.C[idx];  // D z - x
          g.Out[idx] = r;
          if (g.fpart) fs[fm][r4] += 0.5 * (double)r * (double)r;
        } else if constexpr (EPI == kEpiLista) {
          const float zn = soft_threshold(g.Zt[idx] - a * p, lth);
          g.Out[idx] = zn;
          if (g.fpart) fs[fm][r4] += (double)lam * fabs((double)zn);
        } else if constexpr (EPI == kEpiListaQ) {
          g.Out[idx] = p;  // W_t v
          dsum += (double)p * (double)g.C[idx];  // (W_t v) . (D z^t - x)
        } else if constexpr (EPI == kEpiListaBwd) {
          const float v = g.Vin[idx], zt = g.Zt[idx];
          dsum += (double)v * (double)sgnf(g.Zt1[idx]);
          g.Out[idx] = (zt != 0.f) ? v - a * p : 0.f;
        } else if constexpr (EPI == kEpiFwd) {
          const float z = g.Zt[idx], c = g.C[idx];
          if constexpr (FOLD) {
            // p = z - a G z
            g.Out[idx] = soft_threshold(fmaf(a, c, p), th);
            if (g.fpart) fs[fm][r4] += (double)(0.5f * z * ((z - p) / a) - z * c + lam * fabsf(z));
          } else {
            g.Out[idx] = soft_threshold(z - a * (p - c), th);
            if (g.fpart) fs[fm][r4] += (double)(0.5f * z * p - z * c + lam * fabsf(z));
          }
        } else if constexpr (EPI == kEpiFinal) {
          const float z = g.Zt[idx], c = g.C[idx];
          fs[fm][r4] += (double)(0.5f * z * p - z * c + lam * fabsf(z));
        } else if constexpr (EPI == kEpiSeed) {
          const float z = g.Zt[idx], c = g.C ? g.C[idx] : 0.f;  // LISTA seeds pass P = D^T (D z - x), no c
          float gv = w * (p - c + lam * sgnf(z));
          if (g.dZ && col < g.m) gv += g.dZ[(size_t)row * g.m + col];
          g.Out[idx] = (z != 0.f) ? gv : 0.f;
          if (g.fpart) fs[fm][r4] += (double)(0.5f * z * p - z * c + lam * fabsf(z));
        } else if constexpr (EPI == kEpiGrad) {
          const float z = g.Zt[idx], r = p - g.C[idx];
          g.Out[idx] = r;
          if (z == 0.f && fabsf(r) > lam) fs[fm][r4] += 1.0;
        } else if constexpr (EPI == kEpiFista) {
          // A = y^t (Zt: its FP32 copy), Zt1 = z^t
          const float y = g.Zt[idx], zo = g.Zt1[idx], c = g.C[idx];
          const float zn = soft_threshold(y - a * (p - c), th);
          g.Out[idx] = zn;
          g.Out2[idx] = zn + bt * (zn - zo);
        } else {  // kEpiBwd
          const float v = g.Vin[idx], zt = g.Zt[idx], zt1 = g.Zt1[idx];
          dsum += (double)v * ((double)zt - (double)zt1);
          const float gv = v - a * p;
          g.Out[idx] = (zt != 0.f) ? gv : 0.f;
        }
      }
    }
  }

  if constexpr (EPI == kEpiFwd || EPI == kEpiFinal || EPI == kEpiSeed || EPI == kEpiGrad || EPI == kEpiResid ||
                EPI == kEpiLista) {
    if (g.fpart) {  // uniform across the workgroup
      double* red = (double*)smem;  // [2][BM]
#pragma unroll
      for (int fm = 0; fm < 4; ++fm)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          double v = fs[fm][r4];
          v += __shfl_xor(v, 1);
          v += __shfl_xor(v, 2);
          v += __shfl_xor(v, 4);
          v += __shfl_xor(v, 8);
          if (lr == 0) red[wn * BM + wm * 64 + fm * 16 + 4 * lg + r4] = v;
        }
      __syncthreads();
      if (tid < BM) {
        const int row = row0 + tid;
        if (row < g.rows) g.fpart[(size_t)ct * g.rows + row] = red[tid] + red[BM + tid];
      }
    }
  }
  if constexpr (EPI == kEpiBwd || EPI == kEpiListaQ || EPI == kEpiListaBwd) {
    double* red = (double*)smem;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dsum += __shfl_xor(dsum, o);
    if (lane == 0) red[wave] = dsum;
    __syncthreads();
    if (tid == 0) g.dpart[tile] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

template <int P, int EPI, bool SAFE>
__global__ __launch_bounds__(NTHREADS) void gemm_fused(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) char smem[2 * STAGE_BYTES];
  if constexpr (EPI == kEpiSplit) {  // K chunk of one batch entry of a split contraction
    const size_t y = blockIdx.y, bi = y / g.ksplit, sp = y - bi * g.ksplit;
    g.A += bi * g.a_batch + sp * g.a_split;
    g.Bt = (const float*)g.Bt + bi * g.b_batch + sp * g.b_split;
    g.Out += y * g.out_split;
  }
  const int b = blockIdx.x;
  // split contractions launch exactly their tiles in x, so that the (tile,
  // chunk) workgroups spread over all XCDs; the others order tiles XCD-contiguously
  const int tile = EPI == kEpiSplit ? b : (b & 7) * g.tiles_per_xcd + (b >> 3);
  if (tile >= g.row_tiles * g.col_tiles) return;
  gemm_tile<P, EPI, SAFE>(g, tile, smem);
}

// Correlation products c = X D of several problems in one launch: workgroup
// b takes tile b - tile_start[p] of problem p, where tile_start (nprob + 1
// prefix sums of the problems' tile counts) brackets b. Each tile runs
// gemm_tile exactly as a single-problem launch would.
__global__ __launch_bounds__(NTHREADS) void gemm_corr_grouped(const GemmArgs* __restrict__ tab,
                                                              const int* __restrict__ tile_start, int nprob) {
  __shared__ __attribute__((aligned(16))) char smem[2 * STAGE_BYTES];
  const int b = blockIdx.x;
  int lo = 0, hi = nprob;  // largest p with tile_start[p] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_start[mid] <= b) lo = mid; else hi = mid;
  }
  const GemmArgs g = tab[lo];
  const int tile = b - tile_start[lo];
  if (tile >= g.row_tiles * g.col_tiles) return;
  gemm_tile<kF32, kEpiCorr, true>(g, tile, smem);
}

template <int P, int EPI, bool SAFE>
hipError_t launch_one(const GemmArgs& a, hipStream_t s) {
  const int grid = EPI == kEpiSplit ? a.row_tiles * a.col_tiles : 8 * a.tiles_per_xcd;
  const int splits = EPI == kEpiSplit ? a.ksplit * (a.nbatch > 0 ? a.nbatch : 1) : 1;
  if (grid == 0 || splits < 1) return grid == 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_fused<P, EPI, SAFE>), dim3(grid, splits), dim3(NTHREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace

void gemm_grid(int rows, int ncols, GemmArgs& a) {
  a.row_tiles = (rows + BM - 1) / BM;
  a.col_tiles = (ncols + BN - 1) / BN;
  const int total = a.row_tiles * a.col_tiles;
  a.tiles_per_xcd = (total + 7) / 8;
}

hipError_t launch_corr_grouped(const GemmArgs* tab, const int* tile_start, int nprob, int total_tiles,
                               hipStream_t s) {
  if (nprob == 0 || total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_corr_grouped, dim3(total_tiles), dim3(NTHREADS), 0, s, tab, tile_start, nprob);
  return hipGetLastError();
}

hipError_t launch_gemm(int prec, int epi, bool safe, const GemmArgs& a, hipStream_t s) {
  if (safe) {
    if (prec == kF32 && epi == kEpiCorr) return launch_one<kF32, kEpiCorr, true>(a, s);
    return hipErrorInvalidValue;
  }
  if (prec == kF32) {
    switch (epi) {
      case kEpiFwd: return launch_one<kF32, kEpiFwd, false>(a, s);
      case kEpiFinal: return launch_one<kF32, kEpiFinal, false>(a, s);
      case kEpiSeed: return launch_one<kF32, kEpiSeed, false>(a, s);
      case kEpiBwd: return launch_one<kF32, kEpiBwd, false>(a, s);
      case kEpiFista: return launch_one<kF32, kEpiFista, false>(a, s);
      case kEpiGrad: return launch_one<kF32, kEpiGrad, false>(a, s);
      case kEpiResid: return launch_one<kF32, kEpiResid, false>(a, s);
      case kEpiLista: return launch_one<kF32, kEpiLista, false>(a, s);
      case kEpiListaQ: return launch_one<kF32, kEpiListaQ, false>(a, s);
      case kEpiListaBwd: return launch_one<kF32, kEpiListaBwd, false>(a, s);
      case kEpiSplit: return launch_one<kF32, kEpiSplit, false>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (epi) {
    case kEpiFwd: return launch_one<kBF16, kEpiFwd, false>(a, s);
    case kEpiFinal: return launch_one<kBF16, kEpiFinal, false>(a, s);
    case kEpiSeed: return launch_one<kBF16, kEpiSeed, false>(a, s);
    case kEpiBwd: return launch_one<kBF16, kEpiBwd, false>(a, s);
    case kEpiFista: return launch_one<kBF16, kEpiFista, false>(a, s);
    case kEpiGrad: return launch_one<kBF16, kEpiGrad, false>(a, s);
    case kEpiResid: return launch_one<kBF16, kEpiResid, false>(a, s);
    case kEpiLista: return launch_one<kBF16, kEpiLista, false>(a, s);
    case kEpiListaQ: return launch_one<kBF16, kEpiListaQ, false>(a, s);
    case kEpiListaBwd: return launch_one<kBF16, kEpiListaBwd, false>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace slista
