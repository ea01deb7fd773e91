// Complex128 GEMMs on FP64 MFMA (v_mfma_f64_16x16x4f64, gfx950).
//
// Two shapes cover the path:
//   CN  C[M x N] = A^H B, A: K x M, B: K x N, K = npw large.  The paper's
//       scalar products p_ij = <beta_j|psi_i> and O_ij = <psi_i|O|psi_j>
//       (section on new parallelization levels), done as one matrix-matrix
//       product per block, as the paper does before its reduce over the
//       plane-wave group.  K is split over workgroups; the partial tiles
//       are summed in a fixed order, so results are bitwise reproducible.
//   NN  C[M x N] = alpha A B + beta C, A: M x K, M = npw large.  The
//       nonlocal update sum_j beta_j(G) (D p)_jn and the Ritz/basis updates.
// All matrices are column-major complex128 (band-major blocks).
//
// A 256-thread workgroup owns a 64 x 64 complex tile; its four waves each
// own 32 x 32 = 2 x 2 MFMA blocks.  A complex product takes four real MFMAs
// (re*re, im*im, re*im, im*re) into four accumulators, combined at the end
// (with the sign pattern of conj(A) for CN).  K advances 16 complex per
// LDS stage; the next stage's global loads are issued before the current
// stage's MFMAs.  The MFMA operands are fed "transposed" (the N-side tile
// as the first operand) so that each lane's output column runs along M,
// the contiguous direction of C.
#include "common.h"

namespace pw {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64;
constexpr int GB_N = 64;
constexpr int GB_K = 16;
constexpr int G_THR = 256;

__device__ __forceinline__ d4_t mfma64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Load a 16(k) x 64(mn) tile of a K-contiguous column-major matrix
// (element (k, c) at P[c * ld + k]) into registers: thread t covers column
// t/4 and k = 4*(t%4) .. +3.
__device__ __forceinline__ void load_kcontig(const double2 *__restrict__ P, int64_t ld, int64_t k0,
                                             int64_t c0, int64_t K, int64_t C, double2 r[4]) {
  const int t = threadIdx.x;
  const int64_t c = c0 + (t >> 2);
  const int64_t k = k0 + ((t & 3) << 2);
  if (c < C) {
    const double2 *p = P + c * ld + k;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = (k + u < K) ? p[u] : double2{0.0, 0.0};
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = double2{0.0, 0.0};
  }
}
__device__ __forceinline__ void store_kcontig(double2 (*S)[GB_M + 1], const double2 r[4]) {
  const int t = threadIdx.x;
  const int c = t >> 2;
  const int k = (t & 3) << 2;
#pragma unroll
  for (int u = 0; u < 4; ++u) S[k + u][c] = r[u];
}

// Load a 64(m) x 16(k) tile of an M-contiguous column-major matrix
// (element (m, k) at P[k * ld + m]): thread t covers k = t/16 and
// m = 4*(t%16) .. +3.
__device__ __forceinline__ void load_mcontig(const double2 *__restrict__ P, int64_t ld, int64_t m0,
                                             int64_t k0, int64_t M, int64_t K, double2 r[4]) {
  const int t = threadIdx.x;
  const int64_t k = k0 + (t >> 4);
  const int64_t m = m0 + ((t & 15) << 2);
  if (k < K) {
    const double2 *p = P + k * ld + m;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = (m + u < M) ? p[u] : double2{0.0, 0.0};
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = double2{0.0, 0.0};
  }
}
__device__ __forceinline__ void store_mcontig(double2 (*S)[GB_M + 1], const double2 r[4]) {
  const int t = threadIdx.x;
  const int k = t >> 4;
  const int m = (t & 15) << 2;
#pragma unroll
  for (int u = 0; u < 4; ++u) S[k][m + u] = r[u];
}

struct Acc {
  d4_t rr[2][2], ii[2][2], ri[2][2], ir[2][2];
};

// One LDS stage: As[k][m], Bs[k][n], 16 complex k.
__device__ __forceinline__ void mma_stage(const double2 (*As)[GB_M + 1],
                                          const double2 (*Bs)[GB_M + 1], Acc &acc, int wm, int wn) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15;
  const int lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < GB_K; kk += 4) {
    double2 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm * 32 + i * 16 + lr];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lk][wn * 32 + j * 16 + lr];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // first operand: N side (rows of the accumulator), second: M side
        acc.rr[i][j] = mfma64(b[j].x, a[i].x, acc.rr[i][j]);
        acc.ii[i][j] = mfma64(b[j].y, a[i].y, acc.ii[i][j]);
        acc.ri[i][j] = mfma64(b[j].y, a[i].x, acc.ri[i][j]);  // re(A) im(B)
        acc.ir[i][j] = mfma64(b[j].x, a[i].y, acc.ir[i][j]);  // im(A) re(B)
      }
    }
  }
}

// Accumulator element r of a lane: row n = lane/16 + 4*r of the block's
// N side, column m = lane%16 of its M side (v_mfma_f64_16x16x4f64 layout).
template <bool CONJ_A, typename F>
__device__ __forceinline__ void for_each_out(const Acc &acc, int wm, int wn, F &&f) {
  const int lane = threadIdx.x & 63;
  const int lm = lane & 15;
  const int ln = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double re = CONJ_A ? acc.rr[i][j][r] + acc.ii[i][j][r] : acc.rr[i][j][r] - acc.ii[i][j][r];
        const double im = CONJ_A ? acc.ri[i][j][r] - acc.ir[i][j][r] : acc.ri[i][j][r] + acc.ir[i][j][r];
        f(wm * 32 + i * 16 + lm, wn * 32 + j * 16 + ln + 4 * r, re, im);
      }
}

__device__ __forceinline__ void zero_acc(Acc &acc) {
  const d4_t z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc.rr[i][j] = acc.ii[i][j] = acc.ri[i][j] = acc.ir[i][j] = z;
}

// CN: grid (tilesM, tilesN, splits).  out = C (splits == 1) or part[split] (M x N, ld M).
__global__ __launch_bounds__(G_THR, 2) void k_zgemm_cn(int64_t M, int64_t N, int64_t K,
                                                    const double2 *__restrict__ A, int64_t lda,
                                                    const double2 *__restrict__ B, int64_t ldb,
                                                    double2 *__restrict__ C, int64_t ldc,
                                                    int64_t kchunk, int direct) {
  __shared__ double2 As[GB_K][GB_M + 1];
  __shared__ double2 Bs[GB_K][GB_M + 1];
  const int64_t m0 = (int64_t)blockIdx.x * GB_M;
  const int64_t n0 = (int64_t)blockIdx.y * GB_N;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  Acc acc;
  zero_acc(acc);
  double2 ra[4], rb[4];
  if (kb < ke) {
    load_kcontig(A, lda, kb, m0, ke, M, ra);
    load_kcontig(B, ldb, kb, n0, ke, N, rb);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += GB_K) {
    store_kcontig(As, ra);
    store_kcontig(Bs, rb);
    __syncthreads();
    if (k0 + GB_K < ke) {
      load_kcontig(A, lda, k0 + GB_K, m0, ke, M, ra);
      load_kcontig(B, ldb, k0 + GB_K, n0, ke, N, rb);
    }
    mma_stage(As, Bs, acc, wm, wn);
    __syncthreads();
  }
  double2 *out = direct ? C : C + (int64_t)blockIdx.z * M * N;
  const int64_t ldo = direct ? ldc : M;
  for_each_out<true>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
    const int64_t m = m0 + mi, n = n0 + ni;
    if (m < M && n < N) out[n * ldo + m] = double2{re, im};
  });
}

__global__ void k_splitk_reduce(int64_t M, int64_t N, int splits, const double2 *__restrict__ part,
                                double2 *__restrict__ C, int64_t ldc) {
  const int64_t tot = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < splits; ++s) {
      const double2 v = part[(int64_t)s * tot + e];
      re += v.x;
      im += v.y;
    }
    const int64_t n = e / M, m = e - n * M;
    C[n * ldc + m] = double2{re, im};
  }
}

// NN: grid (tilesM, tilesN).  C = alpha A B + beta C.
__global__ __launch_bounds__(G_THR, 2) void k_zgemm_nn(int64_t M, int64_t N, int64_t K, double alpha,
                                                    const double2 *__restrict__ A, int64_t lda,
                                                    const double2 *__restrict__ B, int64_t ldb,
                                                    double beta, double2 *__restrict__ C,
                                                    int64_t ldc) {
  __shared__ double2 As[GB_K][GB_M + 1];
  __shared__ double2 Bs[GB_K][GB_M + 1];
  const int64_t m0 = (int64_t)blockIdx.x * GB_M;
  const int64_t n0 = (int64_t)blockIdx.y * GB_N;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  Acc acc;
  zero_acc(acc);
  double2 ra[4], rb[4];
  if (K > 0) {
    load_mcontig(A, lda, m0, 0, M, K, ra);
    load_kcontig(B, ldb, 0, n0, K, N, rb);
  }
  for (int64_t k0 = 0; k0 < K; k0 += GB_K) {
    store_mcontig(As, ra);
    store_kcontig(Bs, rb);
    __syncthreads();
    if (k0 + GB_K < K) {
      load_mcontig(A, lda, m0, k0 + GB_K, M, K, ra);
      load_kcontig(B, ldb, k0 + GB_K, n0, K, N, rb);
    }
    mma_stage(As, Bs, acc, wm, wn);
    __syncthreads();
  }
  for_each_out<false>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
    const int64_t m = m0 + mi, n = n0 + ni;
    if (m < M && n < N) {
      double2 o = double2{alpha * re, alpha * im};
      if (beta != 0.0) {
        const double2 c = C[n * ldc + m];
        o.x += beta * c.x;
        o.y += beta * c.y;
      }
      C[n * ldc + m] = o;
    }
  });
}

int choose_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N);
  // aim for >= 2 workgroups per CU on 256 CUs, each with >= 32 K stages
  int64_t s = (512 + tiles - 1) / tiles;
  const int64_t maxs = (K + 32 * GB_K - 1) / (32 * GB_K);
  if (s > maxs) s = maxs;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

int zgemm_cn(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
             int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  if (splits < 1) splits = 1;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + GB_K - 1) / GB_K * GB_K;
  if (kchunk <= 0) kchunk = GB_K;
  const int direct = (splits == 1) ? 1 : 0;
  dim3 grid((unsigned)((M + GB_M - 1) / GB_M), (unsigned)((N + GB_N - 1) / GB_N), (unsigned)splits);
  hipLaunchKernelGGL(k_zgemm_cn, grid, dim3(G_THR), 0, s, M, N, K, static_cast<const double2 *>(A),
                     lda, static_cast<const double2 *>(B), ldb,
                     static_cast<double2 *>(direct ? C : part), ldc, kchunk, direct);
  if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  if (!direct) {
    int64_t blocks = (M * N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, M, N, splits,
                       static_cast<const double2 *>(part), static_cast<double2 *>(C), ldc);
    if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  }
  return PW_OK;
}

int zgemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
             const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  dim3 grid((unsigned)((M + GB_M - 1) / GB_M), (unsigned)((N + GB_N - 1) / GB_N));
  hipLaunchKernelGGL(k_zgemm_nn, grid, dim3(G_THR), 0, s, M, N, K, alpha,
                     static_cast<const double2 *>(A), lda, static_cast<const double2 *>(B), ldb,
                     beta, static_cast<double2 *>(C), ldc);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

}  // namespace pw
