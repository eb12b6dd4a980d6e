// Persistent Step-LISTA kernels: tile policy, dispatch and the
// fragment-ordered copies of G. The kernels themselves are in
// persist_body.hpp, instantiated per precision in kernels_persist_bf16.hip
// and kernels_persist_f32.hip.
#include "common.hpp"
#include "persist.hpp"

namespace slista {
namespace {

// Fragment-ordered copies of G for the persistent kernels.
// BF16: fragment (cb, kc) = G[16 cb + l % 16][32 kc + 8 (l / 16) + e], e < 8.
// FP32: fragment (cb, kc) = G[16 cb + l % 16][16 kc + 4 (l / 16) + e], e < 4.
__global__ void k_swizzle(const float* __restrict__ G, int mp, uint16_t* __restrict__ Gsb, float* __restrict__ Gsf) {
  const size_t total = (size_t)mp * mp;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    {
      const int e = i & 7, l = (i >> 3) & 63;
      const size_t frag = i >> 9;
      const int KC = mp / 32;
      const int kc = frag % KC, cb = frag / KC;
      const float v = G[(size_t)(16 * cb + (l & 15)) * mp + 32 * kc + 8 * (l >> 4) + e];
      Gsb[i] = __builtin_bit_cast(uint16_t, (__bf16)v);
    }
    {
      const int e = i & 3, l = (i >> 2) & 63;
      const size_t frag = i >> 8;
      const int KC = mp / 16;
      const int kc = frag % KC, cb = frag / KC;
      Gsf[i] = G[(size_t)(16 * cb + (l & 15)) * mp + 16 * kc + 4 * (l >> 4) + e];
    }
  }
}

// Number of 256-column passes for m_pad (0: not handled by these kernels).
int np_of(int m_pad) { return m_pad <= 256 ? 1 : m_pad <= 512 ? 2 : m_pad <= 1024 ? 4 : m_pad <= 2048 ? 8 : 0; }

}  // namespace

// Tile configurations of the persistent kernels, per precision and number of
// 256-column passes:
//   variant 1: R rows per tile, one 4-wave workgroup per CU (one wave per
//              SIMD), G fragments 3 K steps ahead;
//   variant 2: half the rows, two workgroups per CU (two waves per SIMD, so
//              one tile's FP32 epilogue runs under the other tile's MFMAs),
//              G fragments 1 K step ahead, at most 256 registers per lane;
//   variant 3: the rows of variant 1 in one 8-wave workgroup per CU: two row
//              halves x four column slabs, two waves per SIMD; the two waves
//              of a column slab read the same G fragments (one L2 fetch,
//              one L1 hit), G fragments 1 K step ahead;
//   variant 4: the rows of variant 1 in one 8-wave workgroup per CU with
//              eight 32-column slabs per pass: each G fragment is read once
//              per tile, a K step needs half the G registers of variants
//              1-3, and G fragments are issued 3 K steps ahead with two
//              waves per SIMD.
// m_pad in (1024, 2048] has variants 1 and 4.
bool persist_has_variant(int m_pad, int v) {
  const int np = np_of(m_pad);
  if (np == 0) return false;
  return np == 8 ? (v == 1 || v == 4) : (v >= 1 && v <= 4);
}

// Measured on the 256 x 1024, N = 65 536, T = 50 workload (fwd + bwd per
// launch, BF16 / FP32 ms): variant 1 19.1+15.0 / 65.9+58.9, variant 2
// 15.2+16.2 / 56.7+56.1, variant 3 15.9+16.2 / 56.5+57.6, variant 4
// 12.0+15.4 / 54.3+54.5. The autotuner can still pick per problem class.
int default_variant(int prec, int m_pad) {
  (void)prec;
  (void)m_pad;
  return 4;
}

int persist_resolve_variant(int prec, int m_pad, int variant) {
  if (np_of(m_pad) == 0) return 0;
  return persist_has_variant(m_pad, variant) ? variant : default_variant(prec, m_pad);
}

int persist_rows(int prec, int m_pad, int variant) {
  const int np = np_of(m_pad);
  if (np == 0) return 0;
  variant = persist_resolve_variant(prec, m_pad, variant);
  const bool v2 = variant == 2;
  if (prec == kBF16) return np == 8 ? 32 : (v2 ? 32 : 64);
  if (np == 8) return 16;
  if (np == 4) return v2 ? 16 : 32;
  return v2 ? 32 : 64;  // variants 3 and 4 keep the rows of variant 1
}

// Template arguments per (precision, passes, variant): rows, passes, G
// prefetch depth, waves per SIMD bound, row waves, column waves.

hipError_t launch_persist(bool fwd, int prec, const PersistArgs& a, hipStream_t s, int variant) {
  if (fwd && a.N > 0 && !a.Cg) return hipErrorInvalidValue;  // the forward reads c in row-group order
  const int np = np_of(a.m_pad);
  variant = persist_resolve_variant(prec, a.m_pad, variant);
  return prec == kBF16 ? launch_persist_bf16(fwd, np, variant, a, s) : launch_persist_f32(fwd, np, variant, a, s);
}

int persist_np(int m_pad) { return np_of(m_pad); }

hipError_t launch_persist_batched(bool fwd, int prec, int np, int variant, const PersistArgs* tab, const int2* work,
                                  int nwork, int max_m_pad, const PersistPhase& ph, hipStream_t s) {
  const int probe_m_pad = np == 8 ? 2048 : np * 256;
  variant = persist_resolve_variant(prec, probe_m_pad, variant);
  return prec == kBF16 ? launch_persist_batched_bf16(fwd, np, variant, tab, work, nwork, max_m_pad, ph, s)
                       : launch_persist_batched_f32(fwd, np, variant, tab, work, nwork, max_m_pad, ph, s);
}

bool fista_persist_applies(int m_pad) { const int np = np_of(m_pad); return np == 1 || np == 2; }

static int fista_variant(int variant) { return variant == 2 ? 2 : 4; }

int fista_persist_rows(int prec, int m_pad, int variant) {
  return fista_persist_applies(m_pad) ? persist_rows(prec, m_pad, fista_variant(variant)) : 0;
}

hipError_t launch_fista_persist(int prec, const PersistArgs& a, hipStream_t s, int variant) {
  if (!fista_persist_applies(a.m_pad) || a.t_begin != 0 || a.k != 0 || (a.N > 0 && (!a.Cg || !a.beta)))
    return hipErrorInvalidValue;
  const int np = np_of(a.m_pad), v = fista_variant(variant);
  return prec == kBF16 ? launch_fista_persist_bf16(np, v, a, s) : launch_fista_persist_f32(np, v, a, s);
}

hipError_t launch_swizzle(const float* G32, int mp, uint16_t* Gsb, float* Gsf, hipStream_t s) {
  const size_t total = (size_t)mp * mp;
  size_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_swizzle, dim3((unsigned)blocks), dim3(256), 0, s, G32, mp, Gsb, Gsf);
  return hipGetLastError();
}

}  // namespace slista
