// Persistent coupled-LISTA kernels (kernels_lista_persist.hip): arguments and
// launchers shared with the host code.
#pragma once

#include "common.hpp"

namespace slista {

constexpr int kListaRows = 32;                 // samples per workgroup
constexpr size_t kListaMaxLds = 160 * 1024;    // LDS per workgroup (one CU's)

struct ListaPersistArgs {
  int N, n_pad, m_pad, T;
  const float* Xp;      // [N][n_pad] samples, zero padded
  const void* Dr;       // [n_pad][m_pad] rows of D (operand precision)
  const void* DT;       // [m_pad][n_pad] columns of D
  const void* Wr;       // [T][n_pad][m_pad] rows of W_t
  const void* WT;       // [T][m_pad][n_pad] columns of W_t
  const float* alpha;   // [T]
  const float* beta;    // [T]
  float lam;
  float* zs;            // z^t at zs + slot(t) N m_pad: slot t (tape) or t & 1
  float* rs;            // R^t = D z^t - x at rs + t N n_pad (tape), or R^T at rs
  int tape;             // forward: store every z^{t+1} and R^t
  double* fres;         // [N] 1/2 |R^T|^2 per sample, or null
  double* fl1;          // [N] lam |z^T|_1 per sample, or null
  float* vs;            // backward: v^t at vs + t N m_pad (v^{T-1} from the seed)
  double* dpa;          // backward: [T][nwg] dalpha partials
  double* dpb;          // backward: [T][nwg] dbeta partials
  int nwg;              // workgroups of the launch: ceil(N / kListaRows)
};

// Dynamic LDS bytes of the forward (fwd) or backward kernel.
size_t lista_persist_lds(int prec, bool fwd, int n_pad, int m_pad);
// One launch over ceil(N / kListaRows) workgroups; hipErrorInvalidValue when
// n_pad or m_pad is not a multiple of 64 or the tile does not fit in LDS.
hipError_t launch_lista_persist(int prec, bool fwd, const ListaPersistArgs& a, hipStream_t s);

}  // namespace slista
