// BF16 instantiations of the persistent kernels: the tile table of
// this precision (see the variant descriptions in kernels_persist.hip).
#include "persist_body.hpp"

namespace slista {

// Template arguments per (passes, variant): rows, passes, G prefetch depth,
// waves-per-SIMD bound, row waves, column waves.
#define SLISTA_TILES(X) \
  X(1, 1, 64, 1, 4, 1, 1, 4) X(1, 2, 32, 1, 2, 2, 1, 4) \
  X(1, 3, 64, 1, 2, 1, 2, 4) X(1, 4, 64, 1, 4, 2, 1, 8) \
  X(2, 1, 64, 2, 4, 1, 1, 4) X(2, 2, 32, 2, 2, 2, 1, 4) \
  X(2, 3, 64, 2, 2, 1, 2, 4) X(2, 4, 64, 2, 4, 2, 1, 8) \
  X(4, 1, 64, 4, 4, 1, 1, 4) X(4, 2, 32, 4, 2, 2, 1, 4) \
  X(4, 3, 64, 4, 2, 1, 2, 4) X(4, 4, 64, 4, 4, 2, 1, 8) \
  X(8, 1, 32, 8, 4, 1, 1, 4) X(8, 4, 32, 8, 4, 2, 1, 8)
// the FISTA subset: variants 2 and 4 of the one- and two-pass buckets (the
// tile then holds both z and y in registers)
#define SLISTA_FISTA_TILES(X) \
  X(1, 2, 32, 1, 2, 2, 1, 4) X(1, 4, 64, 1, 4, 2, 1, 8) \
  X(2, 2, 32, 2, 2, 2, 1, 4) X(2, 4, 64, 2, 4, 2, 1, 8)

hipError_t launch_persist_bf16(bool fwd, int np, int variant, const PersistArgs& a, hipStream_t s) {
  switch (np * 8 + variant) {
#define SLISTA_CASE(NPV, V, R, NPT, PF, OCC, WR, WC) \
  case NPV * 8 + V:                                \
    return launch_pair<kBF16, R, NPT, PF, OCC, WR, WC>(fwd, a, s);
    SLISTA_TILES(SLISTA_CASE)
#undef SLISTA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_persist_batched_bf16(bool fwd, int np, int variant, const PersistArgs* tab, const int2* work,
                                     int nwork, int max_m_pad, const PersistPhase& ph, hipStream_t s) {
  switch (np * 8 + variant) {
#define SLISTA_CASE(NPV, V, R, NPT, PF, OCC, WR, WC) \
  case NPV * 8 + V:                                \
    return launch_pair_batched<kBF16, R, NPT, PF, OCC, WR, WC>(fwd, tab, work, nwork, max_m_pad, ph, s);
    SLISTA_TILES(SLISTA_CASE)
#undef SLISTA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// FISTA: variants 2 and 4 of the one- and two-pass buckets.
hipError_t launch_fista_persist_bf16(int np, int variant, const PersistArgs& a, hipStream_t s) {
  switch (np * 8 + variant) {
#define SLISTA_CASE(NPV, V, R, NPT, PF, OCC, WR, WC) \
  case NPV * 8 + V:                                \
    return launch_fista<kBF16, R, NPT, PF, OCC, WR, WC>(a, s);
    SLISTA_FISTA_TILES(SLISTA_CASE)
#undef SLISTA_CASE
    default:
      return hipErrorInvalidValue;
  }
}
#undef SLISTA_TILES
#undef SLISTA_FISTA_TILES

}  // namespace slista
