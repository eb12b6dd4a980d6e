// Internal definitions shared by the HIP translation units of libslista.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace slista {

// m is zero-padded to a multiple of kPadM inside the library (Gram matrices,
// correlations, iterates); padded coordinates stay exactly 0 in every layer
// because their rows and columns of G and their correlations are 0.
constexpr int kPadM = 64;

// The tape slots and the row-group copy of c hold N rounded up to whole
// 64-row tiles (the largest persistent tile), so every tile's loads stay
// inside them; the rows past N hold 0 in c and are never read as data from
// the tape.
constexpr int kTapeRowAlign = 64;
__host__ __device__ inline int tape_rows(int N) { return (N + kTapeRowAlign - 1) / kTapeRowAlign * kTapeRowAlign; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// ST(u, th) = sign(u) max(|u| - th, 0) (Section 1, after Eq. (2)), written
// as u - clamp(u, -th, th): one median-of-three and one subtraction. For
// every finite u and th > 0 this is the same FP32 value as the sign / max
// form (both round only |u| - th, and rounding to nearest is symmetric); a
// NaN u gives NaN.
__device__ __forceinline__ float soft_threshold(float u, float th) {
  return u - __builtin_amdgcn_fmed3f(u, -th, th);
}

// A wave-uniform float, materialised in a scalar register: a product such as
// the threshold lam alpha_t is rounded once there and cannot be contracted
// into a later subtraction (a fused |u| - lam alpha_t would round
// differently, element by element, from kernel to kernel).
__device__ __forceinline__ float uniform_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

enum Prec : int { kF32 = 0, kBF16 = 1 };

// Epilogues fused behind the contraction P = A * B^T (B^T stored K-contiguous).
enum Epi : int {
  kEpiCorr = 0,   // C = X D: store P                                   (prep)
  kEpiFwd = 1,    // z^{t+1} = ST(z^t - a (P - c), lam a); F(z^t) partial  (one layer)
  kEpiFinal = 2,  // F(z^T) partial only                                 (objective)
  kEpiSeed = 3,   // v^{T-1} = [z^T != 0] (dF (P - c + lam sign z^T) + dZ)  (backward seed)
  kEpiBwd = 4,    // dalpha_t partial; v^{t-1} = [z^t != 0] (v^t - a P)  (one layer back)
  kEpiFista = 5,  // z^{t+1} = ST(y^t - a (P - c), lam a), y^{t+1} = z^{t+1} + b (z^{t+1} - z^t)  (FISTA)
  kEpiGrad = 6,   // R = P - c; per-row count of z_j = 0 with |R_j| > lam  (Oracle-ISTA)
  // coupled LISTA (factored form, per-layer W_t)
  kEpiResid = 7,    // R = P - x (P = Z D^T); objective partial 1/2 |R|^2
  kEpiLista = 8,    // z^{t+1} = ST(z^t - a P, lam b) (P = R W_t); objective partial lam |z^{t+1}|
  kEpiListaQ = 9,   // Q = P (P = V W_t^T); dalpha partial sum Q . R^t
  kEpiListaBwd = 10,  // v^{t-1} = [z^t != 0] (v^t - a P) (P = Q D); dbeta partial sum v^t sign z^{t+1}
  kEpiSplit = 11    // P over one K chunk of a split, batched contraction (FP32 only)
};

struct Dict {
  int n, m, m_pad;
  int device;
  float* G32;      // [m_pad][m_pad] FP32 Gram matrix, zero padded
  uint16_t* Gb;    // [m_pad][m_pad] BF16 copy (bit pattern), zero padded
  float* Dt;       // [m_pad][n]     D^T, zero rows for j >= m
  double* pwork;   // power iteration scratch: [2 * m_pad + 4]
  unsigned int* flag;  // non-finite counter of the finite-value checks
  uint16_t* Gsb;   // BF16 G in MFMA fragment order (persistent kernels)
  float* Gsf;      // FP32 G in MFMA fragment order (persistent kernels)
};

// Arguments of one fused contraction launch. All matrices row-major.
struct GemmArgs {
  const float* A;     // [rows][lda] FP32 (rounded to BF16 while staging in BF16 mode)
  const void* Bt;     // [ncols][ldb] FP32 or BF16: row j holds B[:, j]
  int lda, ldb;
  int rows;           // valid rows of A / output (N)
  int ncols;          // valid output columns (rows of Bt)
  int K;              // contraction length
  int row_tiles, col_tiles, tiles_per_xcd;
  // epilogue
  const float* alpha; // device step sizes; alpha[t]
  int t;
  float lam;
  const float* C;     // [rows][ldz] correlations c = D^T x
  const float* Zt;    // [rows][ldz] z^t   (kEpiFwd, kEpiFinal, kEpiSeed, kEpiBwd)
  const float* Zt1;   // [rows][ldz] z^{t+1} (kEpiBwd)
  const float* Vin;   // [rows][ldz] v^t (kEpiBwd; FP32 copy of the A operand)
  float* Out;         // [rows][ldz] output
  int ldz;
  double* fpart;      // [col_tiles][rows] objective partial sums, or null
  double* dpart;      // [row_tiles * col_tiles] dalpha partial sums (kEpiBwd)
  const float* dF;    // [rows] seed weights, or null -> dF_scalar
  float dF_scalar;
  const float* dZ;    // [rows][m] upstream gradient of z^T, or null
  int m;
  const float* beta;  // [T] momentum weights (kEpiFista), thresholds (kEpiLista)
  float* Out2;        // [rows][ldz] second output: y^{t+1} (kEpiFista)
  // kEpiSplit: grid.y = nbatch * ksplit (nbatch 0 counts as 1); y = b * ksplit + s is K chunk s of
  // batch entry b: it reads A + b a_batch + s a_split, Bt + b b_batch +
  // s b_split and writes Out + y out_split (element offsets)
  int ksplit, nbatch;
  size_t a_split, b_split, out_split, a_batch, b_batch;
};

// Launchers (kernels_gemm.hip)
hipError_t launch_gemm(int prec, int epi, bool safe, const GemmArgs& a, hipStream_t s);
// c = X D for several problems in one launch (FP32, bounds-checked like the
// single-problem correlation product): tab[p] as prep fills it for problem p,
// tile_start[0 .. nprob] the prefix sums of their tile counts (device).
hipError_t launch_corr_grouped(const GemmArgs* tab, const int* tile_start, int nprob, int total_tiles,
                               hipStream_t s);
void gemm_grid(int rows, int ncols, GemmArgs& a);  // fills the tile counts

// Launchers (kernels_misc.hip)
hipError_t launch_gram(const float* D, int n, int m, int m_pad, float* G32, uint16_t* Gb, float* Dt,
                       hipStream_t s);
// FP64 power iteration for L: state in work (2 m_pad + 8 doubles); one step
// = one matrix-vector product over all CUs and one normalisation.
hipError_t launch_power_init(int m, int mp, double* work, hipStream_t s);
hipError_t launch_power_step(const float* G32, int m, int mp, int max_iter, double rtol, double* work,
                             hipStream_t s);
hipError_t launch_xsq(const float* X, int N, int n, double* xsq, hipStream_t s);
hipError_t launch_layer0(const float* C, int N, int ldz, const float* alpha, float lam, float* Z1,
                         hipStream_t s);
hipError_t launch_copy_out(const float* Zs, int N, int ldz, int m, float* Z, hipStream_t s);
hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s);
// out[((i/4) ld + j) 4 + i%4] = A[i ld + j] for i < 4 ceil(N/4) (0 past N);
// out holds ceil(N/4) 4 ld floats, 16-byte aligned.
hipError_t launch_row_groups(const float* A, int N, int ld, float* out, hipStream_t s);
hipError_t launch_reduce_f(const double* xsq, const double* fpart, int col_tiles, int N, float* F,
                           double* Fd, hipStream_t s);
hipError_t launch_reduce_loss(const double* Fd, int N, float* loss, hipStream_t s);
// Training loop helpers: FP64 mean of Fd; candidate steps max(alpha - eta g, 0).
hipError_t launch_mean_d(const double* Fd, int N, double* out, hipStream_t s);
hipError_t launch_alpha_step(const float* alpha, const float* g, double eta, int T, float* cand, hipStream_t s);
// FISTA momentum weights beta[0..T) (FP64 recurrence, one thread).
hipError_t launch_fista_beta(int T, float* beta, hipStream_t s);
// Oracle-ISTA: per sample, L_S of the support of z (FP64 Lanczos on G_SS,
// or on D_S^T D_S in factored form for large supports; kept while the support
// is the one recorded in row i of V) -> step[i] = 1/L_S (1/L if S is empty);
// then z' = ST(z - a_i R, lam a_i) with a_i = step[i], or 1/L where the row's
// violation count (sum over col tiles of flags) is nonzero.
size_t support_lipschitz_lds(int m_pad, int n);
hipError_t launch_support_lipschitz(const float* G32, const float* Dt, int n, int m, int mp, const float* Z, float* V,
                                    double L, int max_iter, double tol, int N, float* step, hipStream_t s);
hipError_t launch_oista_update(const float* Z, const float* R, const double* flags, int col_tiles, const float* step,
                               double L, float lam, int N, int mp, float* Zout, float* steps_used, hipStream_t s);
// Coupled LISTA helpers (kernels_lista.hip).
// Operand copies of a stack of T matrices M_t [n][m] (entry (t, k, j) at
// M[t mstride + k ld + j], or at M[t mstride + j ld + k] when trans != 0):
// Mr [T][n_pad][m_pad] (rows of M_t) and Mt [T][m_pad][n_pad] (columns of
// M_t), zero padded, as FP32 or BF16 bit patterns.
hipError_t launch_lista_pack(const float* M, int T, int n, int m, int ld, size_t mstride, int trans, int n_pad,
                             int m_pad, int prec, void* Mr, void* Mt, hipStream_t s);
// Xp [N][n_pad] = X [N][n] zero padded.
hipError_t launch_pad_rows(const float* X, int N, int n, int n_pad, float* Xp, hipStream_t s);
// For each of `batch` matrices b: src_b [N][ld] (columns 0..cols) transposed
// into chunks of Kc samples, dst_b [Np / Kc][cols][Kc] (Kc a multiple of 64
// dividing Np), 0 for samples >= N; src_b = src + b src_stride, dst_b = dst +
// b dst_stride (elements).
hipError_t launch_transpose_pad(const float* src, int N, int ld, int cols, int Np, int Kc, float* dst, int batch,
                                size_t src_stride, size_t dst_stride, hipStream_t s);
// F_i = sum of the residual partials + sum of the l1 partials (FP64).
hipError_t launch_lista_reduce_f(const double* fres, int ctn, const double* fl1, int ctm, int N, float* F,
                                 double* Fd, hipStream_t s);
// dalpha_t = -sum_p dpa[t][p]; dbeta_t = -lam sum_p dpb[t][p].
hipError_t launch_lista_reduce_ab(const double* dpa, int Pa, const double* dpb, int Pb, int T, float lam,
                                  float* dalpha, float* dbeta, hipStream_t s);
// For every layer t < T: dW_t = -alpha_t sum_s part[t][s] (part [T][S][count],
// dW [T][count]; FP64 sums in a fixed order).
hipError_t launch_lista_reduce_w(const float* part, int S, size_t count, const float* alpha, int T, float* dW,
                                 hipStream_t s);
hipError_t launch_bwd0(const float* V0, const float* Z1, int N, int ldz, double* dpart, int nblocks,
                       hipStream_t s);
// dalpha_t = -(1/alpha_t) sum of the first n_t partials of row t of dpart
// [T][P]: n_0 = count0, n_t = count for 0 < t < t_split, count_hi for
// t >= t_split (layers run with different tile sizes).
hipError_t launch_reduce_dalpha(const double* dpart, int T, int P, int count0, int count, const float* alpha,
                                float* dalpha, hipStream_t s, int t_split = 1 << 30, int count_hi = 0);
int bwd0_blocks(int N, int ldz);
hipError_t launch_objective(const float* X, const float* Dt, int N, int n, int m, float lam, const float* Z,
                            float* F, hipStream_t s);
// The small per-problem steps of an uneven batch in one launch each over a
// table of problems (device memory): the norms ||x_i||^2 and the row-group
// copy of c before the forward; the mean loss and the step gradients after
// the backward. Per problem the arithmetic and its order are those of
// launch_xsq / launch_row_groups / launch_reduce_loss / launch_reduce_dalpha.
struct BatchSmall {
  const float* X;            // [N, n]
  int N, n, mp;
  double* xsq;               // [N]
  const float* C;            // [N, mp] row-major c
  float* Cg;                 // its row-group copy, or NULL
  const double* Fd;          // [N] per-sample objectives
  float* loss;               // mean objective, or NULL
  const double* dpart;       // [T][P] step-gradient partials
  int P, count0, count, t_split, count_hi;
  const float* alpha;        // [T]
  float* dalpha;             // [T]
};
hipError_t launch_batch_prep(const BatchSmall* tab, int nprob, int max_N, size_t max_group_elems, hipStream_t s);
hipError_t launch_batch_loss(const BatchSmall* tab, int nprob, hipStream_t s);
hipError_t launch_batch_dalpha(const BatchSmall* tab, int nprob, int T, hipStream_t s);
// FP64 forward (kernels_f64.hip): ISTA / Step-LISTA in double precision, one
// wave per sample, factored gradient D^T (D z - x); n <= f64_max_n().
// F: [T + 1][N] trace if f_trace, else F(z^T) [N] (either may be NULL);
// Fd: F(z^T) [N] (may be NULL).
int f64_max_n();
size_t ista_f64_lds(int n, int m_pad);
hipError_t launch_ista_f64(const float* Dt, int n, int m, int m_pad, const double* X, int N, double lam,
                           const double* alpha, int T, double* Z, double* F, int f_trace, double* Fd, hipStream_t s);
// Checks (kernels_check.hip).
// Per sample, in FP64: the largest violation of the Lasso optimality
// conditions (Lemma 2.1) by z_i, and F(z_i) (Eq. (1)); n <= kkt_max_n().
int kkt_max_n();
hipError_t launch_kkt(const float* X, const float* Dt, int N, int n, int m, double lam, const float* Z, double* kkt,
                      double* F, hipStream_t s);
// *out = max over i < N, j < m of |C[i][ld * i + j]| (out zeroed first).
hipError_t launch_absmax(const float* C, int N, int ld, int m, float* out, hipStream_t s);
// out[i] = max over j < m of |C[i ld + j]| for i < N.
hipError_t launch_row_absmax(const float* C, int N, int ld, int m, float* out, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, hipStream_t s);
// *out += number of NaN / Inf entries of p[0..count).
hipError_t launch_count_nonfinite(const float* p, size_t count, unsigned int* out, hipStream_t s);

}  // namespace slista
