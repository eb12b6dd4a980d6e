// Helpers of the coupled LISTA network (Section 4, Eq. (11)-(12)) around the
// fused contraction: operand copies of the per-layer matrices W_t and of D,
// zero-padded copies of the samples, the sample-to-column transposes that
// feed the weight-gradient contraction (a sum over samples), and the
// fixed-order reductions of the objective and of the parameter gradients.
//
// Every reduction runs in an order fixed by the sizes alone, so results are
// bitwise reproducible; no floating-point atomics.
#include "common.hpp"

namespace slista {
namespace {

constexpr int kThreads = 256;

__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint16_t to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// One thread per entry of the padded [T][n_pad][m_pad] stack. Entry (t, k, j)
// of M is M[t * mstride + k * ld + j], or M[t * mstride + j * ld + k] when the
// source holds the transpose. Mr gets it at (t, k, j), Mt at (t, j, k); both
// are zero outside k < n, j < m.
__global__ void k_lista_pack(const float* __restrict__ M, int T, int n, int m, int ld, size_t mstride, int trans,
                             int n_pad, int m_pad, int bf16, void* __restrict__ Mr, void* __restrict__ Mt) {
  const size_t per = (size_t)n_pad * m_pad, total = per * T;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t t = e / per, rem = e - t * per;
    const int k = (int)(rem / m_pad), j = (int)(rem - (size_t)k * m_pad);
    float v = 0.f;
    if (k < n && j < m) v = trans ? M[t * mstride + (size_t)j * ld + k] : M[t * mstride + (size_t)k * ld + j];
    const size_t et = t * per + (size_t)j * n_pad + k;
    if (bf16) {
      ((uint16_t*)Mr)[e] = to_bf16(v);
      ((uint16_t*)Mt)[et] = to_bf16(v);
    } else {
      ((float*)Mr)[e] = v;
      ((float*)Mt)[et] = v;
    }
  }
}

__global__ void k_pad_rows(const float* __restrict__ X, int N, int n, int n_pad, float* __restrict__ Xp) {
  const size_t total = (size_t)N * n_pad;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n_pad;
    const int k = (int)(e - i * n_pad);
    Xp[e] = k < n ? X[i * n + k] : 0.f;
  }
}

// 64 x 64 tile through LDS: coalesced row reads of the sample-major source and
// coalesced row writes of the chunk-major destination (chunk = Kc samples, a
// multiple of 64: dst[i / Kc][c][i % Kc]); the 65-float row stride keeps the
// transposed LDS reads on distinct banks.
__global__ __launch_bounds__(kThreads) void k_transpose_pad(const float* __restrict__ src, int N, int ld, int cols,
                                                            int Np, int Kc, float* __restrict__ dst, size_t src_stride,
                                                            size_t dst_stride) {
  __shared__ float tile[64][65];
  const int i0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  src += blockIdx.z * src_stride;
  dst += blockIdx.z * dst_stride;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += kThreads / 64) {
    const int i = i0 + r, c = c0 + tx;
    tile[r][tx] = (i < N && c < cols) ? src[(size_t)i * ld + c] : 0.f;
  }
  __syncthreads();
  const size_t chunk = (size_t)(i0 / Kc) * cols * Kc;  // the 64 samples share one chunk
  const int ic = i0 % Kc + tx;
  for (int r = ty; r < 64; r += kThreads / 64) {
    const int c = c0 + r;
    if (c < cols && i0 + tx < Np) dst[chunk + (size_t)c * Kc + ic] = tile[tx][r];
  }
}

// F_i = sum_c fres[c][i] (1/2 |D z - x|^2 by column tile) + sum_c fl1[c][i]
// (lam |z|_1 by column tile): Eq. (1) from the factored residual.
__global__ void k_lista_reduce_f(const double* __restrict__ fres, int ctn, const double* __restrict__ fl1, int ctm,
                                 int N, float* __restrict__ F, double* __restrict__ Fd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int c = 0; c < ctn; ++c) s += fres[(size_t)c * N + i];
  for (int c = 0; c < ctm; ++c) s += fl1[(size_t)c * N + i];
  if (F) F[i] = (float)s;
  if (Fd) Fd[i] = s;
}

// One workgroup per layer t: dalpha_t = -sum (W_t v) . (D z^t - x),
// dbeta_t = -lam sum v sign(z^{t+1}) from the per-tile partials.
__global__ __launch_bounds__(kThreads) void k_lista_reduce_ab(const double* __restrict__ dpa, int Pa,
                                                              const double* __restrict__ dpb, int Pb, float lam,
                                                              float* __restrict__ dalpha, float* __restrict__ dbeta) {
  __shared__ double sh[kThreads];
  const int t = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int p = threadIdx.x; p < Pa; p += blockDim.x) a += dpa[(size_t)t * Pa + p];
  for (int p = threadIdx.x; p < Pb; p += blockDim.x) b += dpb[(size_t)t * Pb + p];
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    dalpha[t] = (float)(-a);
    dbeta[t] = (float)(-(double)lam * b);
  }
}

// dW_t[e] = -alpha_t sum_s part[t][s][e] over the K chunks of the sample sum,
// for every layer t (one thread per entry of the [T][count] output).
__global__ void k_lista_reduce_w(const float* __restrict__ part, int S, size_t count, const float* __restrict__ alpha,
                                 size_t total, float* __restrict__ dW) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t t = e / count, j = e - t * count;
    const float* p = part + t * (size_t)S * count + j;
    double s = 0.0;
    for (int c = 0; c < S; ++c) s += (double)p[(size_t)c * count];
    dW[e] = (float)(-(double)alpha[t] * s);
  }
}

int blocks_for(size_t work) {
  size_t b = (work + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

}  // namespace

hipError_t launch_lista_pack(const float* M, int T, int n, int m, int ld, size_t mstride, int trans, int n_pad,
                             int m_pad, int prec, void* Mr, void* Mt, hipStream_t s) {
  const size_t total = (size_t)T * n_pad * m_pad;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lista_pack, dim3(blocks_for(total)), dim3(kThreads), 0, s, M, T, n, m, ld, mstride, trans,
                     n_pad, m_pad, prec == kBF16 ? 1 : 0, Mr, Mt);
  return hipGetLastError();
}

hipError_t launch_pad_rows(const float* X, int N, int n, int n_pad, float* Xp, hipStream_t s) {
  const size_t total = (size_t)N * n_pad;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pad_rows, dim3(blocks_for(total)), dim3(kThreads), 0, s, X, N, n, n_pad, Xp);
  return hipGetLastError();
}

hipError_t launch_transpose_pad(const float* src, int N, int ld, int cols, int Np, int Kc, float* dst, int batch,
                                size_t src_stride, size_t dst_stride, hipStream_t s) {
  if (Np == 0 || cols == 0 || batch == 0) return hipSuccess;
  if (batch < 0 || batch > 65535 || Kc <= 0 || Kc % 64 != 0 || Np % Kc != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose_pad, dim3((Np + 63) / 64, (cols + 63) / 64, batch), dim3(kThreads), 0, s, src, N, ld,
                     cols, Np, Kc, dst, src_stride, dst_stride);
  return hipGetLastError();
}

hipError_t launch_lista_reduce_f(const double* fres, int ctn, const double* fl1, int ctm, int N, float* F, double* Fd,
                                 hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lista_reduce_f, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, s, fres, ctn, fl1, ctm,
                     N, F, Fd);
  return hipGetLastError();
}

hipError_t launch_lista_reduce_ab(const double* dpa, int Pa, const double* dpb, int Pb, int T, float lam,
                                  float* dalpha, float* dbeta, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lista_reduce_ab, dim3(T), dim3(kThreads), 0, s, dpa, Pa, dpb, Pb, lam, dalpha, dbeta);
  return hipGetLastError();
}

hipError_t launch_lista_reduce_w(const float* part, int S, size_t count, const float* alpha, int T, float* dW,
                                 hipStream_t s) {
  const size_t total = count * (size_t)T;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lista_reduce_w, dim3(blocks_for(total)), dim3(kThreads), 0, s, part, S, count, alpha, total,
                     dW);
  return hipGetLastError();
}

}  // namespace slista
