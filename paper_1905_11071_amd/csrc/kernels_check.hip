// Checks on the device: the optimality conditions of the Lasso in FP64
// (Lemma 2.1, Eq. (3)) together with the cost of Eq. (1), the largest
// correlation |D_j^T x_i| over a batch (lambda_max, Section 2), and a count of
// non-finite values in a buffer.
//
// No floating-point atomics: the maximum of non-negative floats is taken on
// their bit patterns with an integer atomicMax, which is exact and does not
// depend on the order of the updates.
#include "common.hpp"

namespace slista {
namespace {

constexpr int kKktThreads = 256;

// One workgroup per sample i:
//   r = x_i - D z_i                  (FP64; products of two floats are exact)
//   g_j = D_j^T r                    (FP64)
//   viol_j = |g_j - lam sign z_j|    if z_j != 0
//          = max(|g_j| - lam, 0)     if z_j == 0
//   kkt[i] = max_j viol_j,  F[i] = 1/2 ||r||^2 + lam ||z_i||_1.
// Thread t owns residual coordinates k = t + 256 q (q < kKktMaxPerThread) and
// gradient coordinates j = t + 256 q'; the residual is shared through LDS.
// Every sum runs in an order fixed by the sizes alone.
constexpr int kKktMaxPerThread = 32;  // n <= 8192
__global__ __launch_bounds__(kKktThreads) void k_kkt(const float* __restrict__ X, const float* __restrict__ Dt, int N,
                                                     int n, int m, double lam, const float* __restrict__ Z,
                                                     double* __restrict__ kkt, double* __restrict__ F) {
  extern __shared__ double sh[];  // r [n], kKktThreads reduction slots, then z_i [m] (floats)
  double* red = sh + n;
  float* zs = (float*)(red + kKktThreads);
  const int tid = threadIdx.x;
  const int i = blockIdx.x;
  if (i >= N) return;
  const float* zi = Z + (size_t)i * m;
  for (int j = tid; j < m; j += kKktThreads) zs[j] = zi[j];
  double r[kKktMaxPerThread];
#pragma unroll
  for (int q = 0; q < kKktMaxPerThread; ++q) {
    const int k = tid + kKktThreads * q;
    r[q] = k < n ? (double)X[(size_t)i * n + k] : 0.0;
  }
  __syncthreads();
  double l1 = 0.0;
  for (int j = 0; j < m; ++j) {
    const float zj = zs[j];  // the same value in every thread: a uniform branch
    if (zj == 0.f) continue;
    l1 += fabs((double)zj);
    const float* dj = Dt + (size_t)j * n;
#pragma unroll
    for (int q = 0; q < kKktMaxPerThread; ++q) {
      const int k = tid + kKktThreads * q;
      if (k < n) r[q] -= (double)zj * (double)dj[k];
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int q = 0; q < kKktMaxPerThread; ++q) {
    const int k = tid + kKktThreads * q;
    if (k < n) {
      sh[k] = r[q];
      ss += r[q] * r[q];
    }
  }
  __syncthreads();
  double worst = 0.0;
  for (int j = tid; j < m; j += kKktThreads) {
    const float* dj = Dt + (size_t)j * n;
    // four partial sums over k mod 4, added in a fixed order
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
    int k = 0;
    for (; k + 3 < n; k += 4) {
      g0 += (double)dj[k] * sh[k];
      g1 += (double)dj[k + 1] * sh[k + 1];
      g2 += (double)dj[k + 2] * sh[k + 2];
      g3 += (double)dj[k + 3] * sh[k + 3];
    }
    for (; k < n; ++k) g0 += (double)dj[k] * sh[k];
    const double g = (g0 + g1) + (g2 + g3);
    const float zj = zs[j];
    const double v = zj != 0.f ? fabs(g - (zj > 0.f ? lam : -lam)) : fmax(fabs(g) - lam, 0.0);
    worst = fmax(worst, v);
  }
  // fixed-order tree reductions: the maximum, then the sum of squares
  red[tid] = worst;
  __syncthreads();
  for (int s = kKktThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  if (tid == 0) kkt[i] = red[0];
  __syncthreads();
  red[tid] = ss;
  __syncthreads();
  for (int s = kKktThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0 && F) F[i] = 0.5 * red[0] + lam * l1;
}

// max over i < N, j < m of |C[i][j]| (C is [N][ld]), as a float bit pattern.
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ C, int N, int ld, int m,
                                                unsigned int* __restrict__ out) {
  __shared__ unsigned int sh[256];
  unsigned int best = 0u;
  const size_t total = (size_t)N * m;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / m;
    const int j = (int)(e - i * m);
    // |c| as a bit pattern: for non-negative floats the integer order is the float order
    const unsigned int b = __float_as_uint(C[i * ld + j]) & 0x7fffffffu;
    best = b > best ? b : best;
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, sh[0]);
}

// Per-row maximum |C[i][j]| over j < m, one wave per row.
__global__ __launch_bounds__(256) void k_row_absmax(const float* __restrict__ C, int N, int ld, int m,
                                                    float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  unsigned int b = 0u;
  for (int j = lane; j < m; j += 64) {
    const unsigned int v = __float_as_uint(C[(size_t)i * ld + j]) & 0x7fffffffu;
    b = v > b ? v : b;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned int v = (unsigned int)__shfl_xor((int)b, o);
    b = v > b ? v : b;
  }
  if (lane == 0) out[i] = __uint_as_float(b);
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// Number of entries of p[0..count) that are NaN or +-Inf, added to *out.
__global__ __launch_bounds__(256) void k_count_nonfinite(const float* __restrict__ p, size_t count,
                                                         unsigned int* __restrict__ out) {
  __shared__ unsigned int sh[256];
  unsigned int c = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    c += ((__float_as_uint(p[e]) & 0x7f800000u) == 0x7f800000u) ? 1u : 0u;
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0] != 0u) atomicAdd(out, sh[0]);
}

int blocks_for(size_t work) {
  size_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

}  // namespace

int kkt_max_n() { return kKktThreads * kKktMaxPerThread; }

hipError_t launch_kkt(const float* X, const float* Dt, int N, int n, int m, double lam, const float* Z, double* kkt,
                      double* F, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const size_t lds = ((size_t)n + kKktThreads) * sizeof(double) + (size_t)m * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)k_kkt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kkt, dim3(N), dim3(kKktThreads), lds, s, X, Dt, N, n, m, lam, Z, kkt, F);
  return hipGetLastError();
}

hipError_t launch_absmax(const float* C, int N, int ld, int m, float* out, hipStream_t s) {
  unsigned int* o = reinterpret_cast<unsigned int*>(out);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, o);
  if (N > 0) hipLaunchKernelGGL(k_absmax, dim3(blocks_for((size_t)N * m)), dim3(256), 0, s, C, N, ld, m, o);
  return hipGetLastError();
}

hipError_t launch_row_absmax(const float* C, int N, int ld, int m, float* out, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_absmax, dim3((N + 3) / 4), dim3(256), 0, s, C, N, ld, m, out);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* p, size_t count, unsigned int* out, hipStream_t s) {
  if (count == 0 || p == nullptr) return hipSuccess;
  hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks_for(count)), dim3(256), 0, s, p, count, out);
  return hipGetLastError();
}

}  // namespace slista
