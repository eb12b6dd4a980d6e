// Arguments of the persistent Step-LISTA kernels (kernels_persist.hip).
#pragma once

#include "common.hpp"

namespace slista {

enum PersistMode : int {
  kModeF = 1,      // objective F(z^{t_end}) per sample (into F, Fd)
  kModeSeed = 2,   // backward seed v^{T-1} from G z^T (into Vout)
  kModeTrace = 4   // objective F(z^t) for every t in [t_begin, t_end) (into Ftrace)
};

struct PersistArgs {
  const void* Gsw;    // fragment-ordered G (BF16 or FP32)
  int m_pad, KC;      // KC = number of 64-byte K steps per row
  int N, m;
  const float* Cg;    // c = D^T x in row-group order (as the tape), read every layer
  const float* alpha;
  const float* beta;  // FISTA momentum weights beta_t (FISTA launches only)
  float lam;
  // where z^t lives (see the workspace layout in api.cpp)
  char* ckpt;
  char* seg;
  size_t zbytes;
  int k, T, a_last;
  int store_all;
  // a launch that ends (starts) inside the network without a tape slot for
  // that iterate writes (reads) it here instead, in tape order; else NULL
  float* zsave;
  const float* zload;
  // forward range and outputs
  int t_begin, t_end, mode;
  float* F;
  double* Fd;
  float* Ftrace;
  const double* xsq;
  float* Zuser;
  float* Vout;
  const float* dF;
  float dF_scalar;
  const float* dZ;
  // backward range and outputs
  float* Vio;
  double* dpart;
  int P_stride, t_hi, t_lo;
  int mode_mask;      // batched launches: modes this problem takes part in
};

// Layer range and mode of one launch over several problems.
struct PersistPhase {
  int t_begin, t_end, mode, store_all, t_hi, t_lo;
};

// Highest tile variant number; persist_has_variant tells which exist for m_pad
// (none when m_pad is not handled by the persistent kernels).
constexpr int kPersistMaxVariant = 4;
bool persist_has_variant(int m_pad, int v);
// Rows per tile for (prec, m_pad, variant); variant 0 = the default one.
int persist_rows(int prec, int m_pad, int variant);
// The variant a launch with this request runs (0 or out of range -> default).
int persist_resolve_variant(int prec, int m_pad, int variant);
hipError_t launch_persist(bool fwd, int prec, const PersistArgs& a, hipStream_t s, int variant);
// Per-precision tile tables (variant already resolved).
hipError_t launch_persist_bf16(bool fwd, int np, int variant, const PersistArgs& a, hipStream_t s);
hipError_t launch_persist_f32(bool fwd, int np, int variant, const PersistArgs& a, hipStream_t s);
hipError_t launch_persist_batched_bf16(bool fwd, int np, int variant, const PersistArgs* tab, const int2* work,
                                       int nwork, int max_m_pad, const PersistPhase& ph, hipStream_t s);
hipError_t launch_persist_batched_f32(bool fwd, int np, int variant, const PersistArgs* tab, const int2* work,
                                      int nwork, int max_m_pad, const PersistPhase& ph, hipStream_t s);
hipError_t launch_swizzle(const float* G32, int m_pad, uint16_t* Gsb, float* Gsf, hipStream_t s);
// FISTA forward through the persistent kernels (variants 2 and 4, m_pad <=
// 512: the tile carries z and y in registers). a.t_begin = 0, a.k = 0;
// a.beta holds the momentum weights. Variant 0 or one that does not exist
// runs variant 4.
bool fista_persist_applies(int m_pad);
int fista_persist_rows(int prec, int m_pad, int variant);
hipError_t launch_fista_persist(int prec, const PersistArgs& a, hipStream_t s, int variant);
hipError_t launch_fista_persist_bf16(int np, int variant, const PersistArgs& a, hipStream_t s);
hipError_t launch_fista_persist_f32(int np, int variant, const PersistArgs& a, hipStream_t s);
// Column-pass bucket of m_pad (1, 2, 4, 8; 0 = not handled).
int persist_np(int m_pad);
// One launch over the work list (problem, tile) of problems in bucket np; the
// LDS is sized for max_m_pad.
hipError_t launch_persist_batched(bool fwd, int prec, int np, int variant, const PersistArgs* tab, const int2* work,
                                  int nwork, int max_m_pad, const PersistPhase& ph, hipStream_t s);

}  // namespace slista
