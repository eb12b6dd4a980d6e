// FP64 forward of ISTA / Step-LISTA (Eq. (2) with alpha_t = 1/L, Eq. (14)
// with learned steps) for the small double-precision workload: every
// quantity in FP64, the gradient in the factored form D^T (D z - x) of the
// paper's layer, with D's FP32 values widened exactly. One wave carries one
// sample through all layers: z and the residual live in the wave's LDS
// slice, and the loops over atoms skip zero coordinates of z (a wave-uniform
// branch), so a sparse iterate costs a fraction of the dense product.
#include "common.hpp"

namespace slista {
namespace {

constexpr int kF64Waves = 4;        // waves (samples in flight) per workgroup
constexpr int kF64MaxN = 512;       // n <= 512: eight residual entries per lane

__device__ double wave_sum_f64(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// F_x(z) = 1/2 ||x - D z||^2 + lam ||z||_1 (Eq. (1)) from the wave's residual
// r = D z - x and z, both in LDS.
__device__ double objective_f64(const double* r, const double* z, int n, int m, double lam, int lane) {
  double rr = 0.0, l1 = 0.0;
  for (int i = lane; i < n; i += 64) rr += r[i] * r[i];
  for (int j = lane; j < m; j += 64) l1 += fabs(z[j]);
  return 0.5 * wave_sum_f64(rr) + lam * wave_sum_f64(l1);
}

// r = D z - x: lane i owns residual entries i, i + 64, ...; the loop runs
// over the atoms j with z_j != 0 and reads row j of D^T (contiguous in i).
__device__ void residual_f64(const float* __restrict__ Dt, const double* __restrict__ x, int n, int m,
                             const double* z, double* r, int lane) {
  double acc[kF64MaxN / 64];
#pragma unroll
  for (int q = 0; q < kF64MaxN / 64; ++q) acc[q] = 0.0;
  for (int j = 0; j < m; ++j) {
    const double zj = z[j];
    if (zj == 0.0) continue;
    const float* drow = Dt + (size_t)j * n;
#pragma unroll
    for (int q = 0; q < kF64MaxN / 64; ++q) {
      const int i = lane + 64 * q;
      if (i < n) acc[q] += (double)drow[i] * zj;
    }
  }
#pragma unroll
  for (int q = 0; q < kF64MaxN / 64; ++q) {
    const int i = lane + 64 * q;
    if (i < n) r[i] = acc[q] - x[i];
  }
}

__global__ __launch_bounds__(64 * kF64Waves) void k_ista_f64(const float* __restrict__ Dt, int n, int m, int mp,
                                                            const double* __restrict__ X, int N, double lam,
                                                            const double* __restrict__ alpha, int T,
                                                            double* __restrict__ Z, double* __restrict__ F,
                                                            int f_trace, double* __restrict__ Fd) {
  extern __shared__ __attribute__((aligned(16))) double sm64[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int npad = (n + 63) / 64 * 64;
  double* z = sm64 + (size_t)w * (mp + npad);
  double* r = z + mp;
  for (int s = blockIdx.x * kF64Waves + w; s < N; s += gridDim.x * kF64Waves) {
    const double* x = X + (size_t)s * n;
    for (int j = lane; j < mp; j += 64) z[j] = 0.0;
    double f = 0.0;
    for (int t = 0;; ++t) {
      residual_f64(Dt, x, n, m, z, r, lane);
      if (f_trace || t == T) {
        f = objective_f64(r, z, n, m, lam, lane);
        if (f_trace && lane == 0) F[(size_t)t * N + s] = f;
      }
      if (t == T) break;
      // z <- ST(z - a D^T r, lam a): lane j owns atoms j, j + 64, ...
      const double a = alpha[t], th = lam * a;
      for (int j = lane; j < m; j += 64) {
        const float* drow = Dt + (size_t)j * n;
        double g = 0.0;
        for (int i = 0; i < n; ++i) g += (double)drow[i] * r[i];
        const double u = z[j] - a * g;
        const double au = fabs(u) - th;
        z[j] = au > 0.0 ? copysign(au, u) : 0.0;
      }
    }
    for (int j = lane; j < m; j += 64) Z[(size_t)s * m + j] = z[j];
    if (lane == 0) {
      if (F && !f_trace) F[s] = f;
      if (Fd) Fd[s] = f;
    }
  }
}

}  // namespace

int f64_max_n() { return kF64MaxN; }

size_t ista_f64_lds(int n, int m_pad) { return (size_t)kF64Waves * (m_pad + (n + 63) / 64 * 64) * sizeof(double); }

hipError_t launch_ista_f64(const float* Dt, int n, int m, int m_pad, const double* X, int N, double lam,
                           const double* alpha, int T, double* Z, double* F, int f_trace, double* Fd, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const size_t lds = ista_f64_lds(n, m_pad);
  hipError_t e = hipFuncSetAttribute((const void*)k_ista_f64, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int blocks = (N + kF64Waves - 1) / kF64Waves;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_ista_f64, dim3(blocks), dim3(64 * kF64Waves), lds, s, Dt, n, m, m_pad, X, N, lam, alpha, T,
                     Z, F, f_trace, Fd);
  return hipGetLastError();
}

}  // namespace slista
