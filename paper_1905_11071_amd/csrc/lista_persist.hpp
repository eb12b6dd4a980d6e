// Persistent coupled-LISTA kernels (kernels_lista_persist.hip): arguments and
// launchers shared with the host code.
#pragma once

#include "common.hpp"

namespace slista {

constexpr int kListaRows = 32;                 // samples per workgroup
constexpr size_t kListaMaxLds = 160 * 1024;    // LDS per workgroup (one CU's)

// Tapes of the persistent path (what the backward and the weight gradient read):
//   rtape  R^t = D z^t - x for t < T, chunk-major: [T][Np / Kc][n][Kc]
//   codes  per layer t < T and element (i, j): bit 0 = [z^t_ij != 0], bit 1 =
//          [z^{t+1}_ij > 0], bit 2 = [z^{t+1}_ij < 0]; byte i % 4 of word
//          (i / 4) m_pad + j of layer t's [nwg * 8][m_pad] words
//   vtape  v^t for t < T (the gradient reaching the output of layer t, masked),
//          chunk-major: [T][Np / Kc][m][Kc]
// Rows N .. Np-1 of the chunk-major tapes must hold zeros (rows below nwg * 32
// are written as zeros by the kernels; the host clears the rest).
struct ListaPersistArgs {
  int N, n, m, n_pad, m_pad, T;
  int Kc, Np;           // sample chunks of the chunk-major tapes (Kc: a multiple of 64)
  const float* Xp;      // [N][n_pad] samples, zero padded
  const void* Dr;       // [n_pad][m_pad] rows of D (operand precision)
  const void* DT;       // [m_pad][n_pad] columns of D
  const void* Wr;       // [T][n_pad][m_pad] rows of W_t
  const void* WT;       // [T][m_pad][n_pad] columns of W_t
  const float* alpha;   // [T]
  const float* beta;    // [T]
  float lam;
  float* zT;            // forward out: [N][m_pad] z^T
  float* rT;            // forward out: [N][n_pad] R^T, or null
  float* rtape;         // forward out / backward in, or null (forward without tape)
  uint32_t* codes;      // forward out / backward in, or null
  double* fres;         // forward out: [N] 1/2 |R^T|^2 per sample, or null
  double* fl1;          // forward out: [N] lam |z^T|_1 per sample, or null
  const float* vseed;   // backward in: [N][m_pad] v^{T-1} from the seed contraction
  float* vtape;         // backward out
  double* dpa;          // backward out: [T][nwg] dalpha partials
  double* dpb;          // backward out: [T][nwg] dbeta partials
  int nwg;              // workgroups of the launch: ceil(N / kListaRows)
};

// Dynamic LDS bytes of the forward (fwd) or backward kernel.
size_t lista_persist_lds(int prec, bool fwd, int n_pad, int m_pad);
// One launch over ceil(N / kListaRows) workgroups; hipErrorInvalidValue when
// n_pad or m_pad is not a multiple of 64, Kc not a multiple of 64, or the
// tile does not fit in LDS.
hipError_t launch_lista_persist(int prec, bool fwd, const ListaPersistArgs& a, hipStream_t s);
// Zero rows i0 .. Np-1 of a chunk-major tape [layers][Np / Kc][cols][Kc].
hipError_t launch_zero_tape_rows(float* tape, int layers, int cols, int Kc, int Np, int i0, hipStream_t s);

}  // namespace slista
