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
// own 32 x 32 = 2 x 2 MFMA blocks.  In FP64 a complex product takes three
// real MFMAs (the three-multiplication form of a complex product, known as
// 3M): re*re, im*im and (re(A) +- im(A)) (re(B) + im(B)), the sign minus for
// conj(A), combined at the end into re = rr -+ ii, im = s - rr -+ ii.  That
// is a quarter fewer MFMAs for two VALU adds per operand pair; the error of
// the imaginary part is bounded by (|re A| + |im A|)(|re B| + |im B|) terms
// instead of |re A||im B| + |im A||re B|.  The FP32 flavour keeps four
// products (re*re, im*im, re*im, im*re): with three, its H psi is 16 %
// faster but its rounding floor reaches the 1e-6 Ry target on the 512-band,
// 38k-plane-wave cell, where a learned-preconditioner solve then stalls
// with two bands at 1.003x the tolerance.  K advances 16 complex per
// LDS stage; the next stage's global loads are issued before the current
// stage's MFMAs.  The MFMA operands are fed "transposed" (the N-side tile
// as the first operand) so that each lane's output column runs along M,
// the contiguous direction of C.
#include "common.h"

namespace pw {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64;
constexpr int GB_N = 64;
constexpr int GB_K = 16;
constexpr int G_THR = 256;

// Workgroups are dealt to the 8 XCDs round-robin, each XCD with its own L2.
// A 1-D grid of 8 * ceil(T / 8) blocks is mapped so that XCD x takes tiles
// x * P .. x * P + P - 1 (P = ceil(T / 8)) in order: tiles next to each other
// in the tile order (the N tiles of one M tile, the tiles of one K chunk)
// then run together under one L2, which fetches their shared operand panels
// from HBM once.  Returns false for the padding blocks.
__device__ __forceinline__ bool xcd_tile(int64_t ntiles, int64_t *t) {
  const int64_t per = (ntiles + 7) / 8;
  const int64_t b = blockIdx.x;
  *t = (b & 7) * per + (b >> 3);
  return *t < ntiles;
}
static inline dim3 xcd_grid(int64_t ntiles) { return dim3((unsigned)(8 * ((ntiles + 7) / 8))); }
// tile t -> (M tile, N tile, K chunk) with N fastest, then M, then K
__device__ __forceinline__ void tile_mnz(int64_t t, int64_t M, int64_t N, int64_t *m0, int64_t *n0, int64_t *z) {
  const int64_t tn = (N + GB_N - 1) / GB_N, tm = (M + GB_M - 1) / GB_M;
  const int64_t r = t % (tm * tn);
  *z = t / (tm * tn);
  *m0 = (r / tn) * GB_M;
  *n0 = (r % tn) * GB_N;
}

// MFMA flavours with K = 4 per instruction: operand lanes hold A[i = l%16][k = l/16]
// and B[k = l/16][j = l%16].  The accumulator's row for register r of lane l
// differs: l/16 + 4r for the f64 instruction, 4(l/16) + r for the f32 one.
struct MF64 {
  using S = double;
  using S2 = double2;
  using acc_t = d4_t;
  static constexpr bool three = false;  // four real products per complex one
  static __device__ __forceinline__ acc_t mfma(S a, S b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
struct MF64x3 : MF64 {
  static constexpr bool three = true;  // three real products per complex one
};
struct MF32 {
  using S = float;
  using S2 = float2;
  using acc_t = f4_t;
  static constexpr bool three = false;
  static __device__ __forceinline__ acc_t mfma(S a, S b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename S2> __device__ __forceinline__ S2 cvt2(double2 v);
template <> __device__ __forceinline__ double2 cvt2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 cvt2<float2>(double2 v) { return float2{(float)v.x, (float)v.y}; }
template <typename S2> __device__ __forceinline__ S2 cvt2(float2 v);
template <> __device__ __forceinline__ float2 cvt2<float2>(float2 v) { return v; }
template <> __device__ __forceinline__ double2 cvt2<double2>(float2 v) { return double2{v.x, v.y}; }

// LDS tiles are [k][mn] with a padded row: with 16-byte elements a stride
// of 2 (mod 8) elements, with 8-byte elements 4 (mod 16), spreads the rows a
// group of lanes touches at once over distinct banks, for the stores below
// (consecutive lanes: consecutive k of one column, then the next column)
// and for the MFMA operand reads (consecutive lanes: consecutive mn).
template <typename S2> struct Lds {
  static constexpr int stride = GB_M + (sizeof(S2) == 16 ? 2 : 4);
};
template <typename S2> using LdsTile = S2[GB_K][Lds<S2>::stride];

// Load a 16(k) x 64(mn) tile of a K-contiguous column-major matrix
// (element (k, c) at P[c * ld + k]) into registers: thread t covers column
// t/4 and k = t%4 + 4u, u = 0..3 (the four lanes of a column read 16
// consecutive k together).  Values stay in the source type until the LDS
// store, so a conversion does not wait for the loads of the next stage.
template <typename T>
__device__ __forceinline__ void load_kcontig(const T *__restrict__ P, int64_t ld, int64_t k0,
                                             int64_t c0, int64_t K, int64_t C, T r[4]) {
  const int t = threadIdx.x;
  const int64_t c = c0 + (t >> 2);
  const int64_t k = k0 + (t & 3);
  if (c < C) {
    const T *p = P + c * ld + k;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = (k + 4 * u < K) ? p[4 * u] : T{0, 0};
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = T{0, 0};
  }
}
template <typename S2, typename T>
__device__ __forceinline__ void store_kcontig(LdsTile<S2> &S, const T r[4]) {
  const int t = threadIdx.x;
  const int c = t >> 2;
  const int k = t & 3;
#pragma unroll
  for (int u = 0; u < 4; ++u) S[k + 4 * u][c] = cvt2<S2>(r[u]);
}

// Load a 64(m) x 16(k) tile of an M-contiguous column-major matrix
// (element (m, k) at P[k * ld + m]): thread t covers k = t/16 and
// m = t%16 + 16u, u = 0..3.
template <typename T>
__device__ __forceinline__ void load_mcontig(const T *__restrict__ P, int64_t ld, int64_t m0,
                                             int64_t k0, int64_t M, int64_t K, T r[4]) {
  const int t = threadIdx.x;
  const int64_t k = k0 + (t >> 4);
  const int64_t m = m0 + (t & 15);
  if (k < K) {
    const T *p = P + k * ld + m;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = (m + 16 * u < M) ? p[16 * u] : T{0, 0};
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = T{0, 0};
  }
}
template <typename S2, typename T>
__device__ __forceinline__ void store_mcontig(LdsTile<S2> &S, const T r[4]) {
  const int t = threadIdx.x;
  const int k = t >> 4;
  const int m = t & 15;
#pragma unroll
  for (int u = 0; u < 4; ++u) S[k][m + 16 * u] = cvt2<S2>(r[u]);
}

// Sums of real products: rr = re A re B, ii = im A im B; with three
// products ri holds (re A +- im A)(re B + im B) and ir is unused, else
// ri = re A im B and ir = im A re B.
template <typename MF> struct Acc {
  typename MF::acc_t rr[2][2], ii[2][2], ri[2][2], ir[2][2];
};

// One LDS stage: As[k][m], Bs[k][n], 16 complex k.
template <typename MF, bool CONJ_A>
__device__ __forceinline__ void mma_stage(const LdsTile<typename MF::S2> &As,
                                          const LdsTile<typename MF::S2> &Bs, Acc<MF> &acc, int wm,
                                          int wn) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15;
  const int lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < GB_K; kk += 4) {
    typename MF::S2 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm * 32 + i * 16 + lr];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lk][wn * 32 + j * 16 + lr];
    if constexpr (MF::three) {
      typename MF::S sa[2], sb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) sa[i] = CONJ_A ? a[i].x - a[i].y : a[i].x + a[i].y;
#pragma unroll
      for (int j = 0; j < 2; ++j) sb[j] = b[j].x + b[j].y;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // first operand: N side (rows of the accumulator), second: M side
          acc.rr[i][j] = MF::mfma(b[j].x, a[i].x, acc.rr[i][j]);
          acc.ii[i][j] = MF::mfma(b[j].y, a[i].y, acc.ii[i][j]);
          acc.ri[i][j] = MF::mfma(sb[j], sa[i], acc.ri[i][j]);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc.rr[i][j] = MF::mfma(b[j].x, a[i].x, acc.rr[i][j]);
          acc.ii[i][j] = MF::mfma(b[j].y, a[i].y, acc.ii[i][j]);
          acc.ri[i][j] = MF::mfma(b[j].y, a[i].x, acc.ri[i][j]);  // re(A) im(B)
          acc.ir[i][j] = MF::mfma(b[j].x, a[i].y, acc.ir[i][j]);  // im(A) re(B)
        }
      }
    }
  }
}

// Accumulator element r of a lane: row n = MF::row(lane, r) of the block's
// N side, column m = lane%16 of its M side.
template <typename MF, bool CONJ_A, typename F>
__device__ __forceinline__ void for_each_out(const Acc<MF> &acc, int wm, int wn, F &&f) {
  const int lane = threadIdx.x & 63;
  const int lm = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double rr = acc.rr[i][j][r], ii = acc.ii[i][j][r];
        const double re = CONJ_A ? rr + ii : rr - ii;
        double im;
        if constexpr (MF::three) {
          const double sp = acc.ri[i][j][r];
          im = CONJ_A ? sp - rr + ii : sp - rr - ii;
        } else {
          const double ri = acc.ri[i][j][r], ir = acc.ir[i][j][r];
          im = CONJ_A ? ri - ir : ri + ir;
        }
        f(wm * 32 + i * 16 + lm, wn * 32 + j * 16 + MF::row(lane, r), re, im);
      }
}

template <typename MF> __device__ __forceinline__ void zero_acc(Acc<MF> &acc) {
  const typename MF::acc_t z = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc.rr[i][j] = acc.ii[i][j] = acc.ri[i][j] = z;
      if constexpr (!MF::three) acc.ir[i][j] = z;
    }
}

// CN: tiles (M, N, K chunk) over an XCD-mapped 1-D grid.  out = C (one chunk) or
// part[chunk] (M x N, ld M).
// A in storage type TA (double2 or float2), B complex128 rounded to MF::S on load.
template <typename MF, typename TA>
__global__ __launch_bounds__(G_THR, 2) void k_zgemm_cn(int64_t M, int64_t N, int64_t K,
                                                       const TA *__restrict__ A, int64_t lda,
                                                       const double2 *__restrict__ B, int64_t ldb,
                                                       double2 *__restrict__ C, int64_t ldc,
                                                       int64_t kchunk, int direct, int64_t nsplit) {
  using S2 = typename MF::S2;
  __shared__ LdsTile<S2> As;
  __shared__ LdsTile<S2> Bs;
  int64_t t, m0, n0, kz;
  if (!xcd_tile(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N) * nsplit, &t)) return;
  tile_mnz(t, M, N, &m0, &n0, &kz);
  const int64_t kb = kz * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  Acc<MF> acc;
  zero_acc(acc);
  TA ra[4];
  double2 rb[4];
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
    mma_stage<MF, true>(As, Bs, acc, wm, wn);
    __syncthreads();
  }
  double2 *out = direct ? C : C + kz * M * N;
  const int64_t ldo = direct ? ldc : M;
  for_each_out<MF, true>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
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

// NN: tiles (M, N) over an XCD-mapped 1-D grid.  C = alpha A B + beta C (C complex128,
// combined in FP64).  Three workgroups per CU: the FP64 form then fits 168
// VGPRs (a 12-byte spill in the epilogue) and its K loop of 576 (the
// projector count) hides more of its load latency, 8 % faster than at two.
template <typename MF, typename TA>
__global__ __launch_bounds__(G_THR, 3) void k_zgemm_nn(int64_t M, int64_t N, int64_t K, double alpha,
                                                       const TA *__restrict__ A, int64_t lda,
                                                       const double2 *__restrict__ B, int64_t ldb,
                                                       double beta, double2 *__restrict__ C,
                                                       int64_t ldc) {
  using S2 = typename MF::S2;
  __shared__ LdsTile<S2> As;
  __shared__ LdsTile<S2> Bs;
  int64_t t, m0, n0, kz;
  if (!xcd_tile(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N), &t)) return;
  tile_mnz(t, M, N, &m0, &n0, &kz);
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  Acc<MF> acc;
  zero_acc(acc);
  TA ra[4];
  double2 rb[4];
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
    mma_stage<MF, false>(As, Bs, acc, wm, wn);
    __syncthreads();
  }
  for_each_out<MF, false>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
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

// ---------------------------------------------------------------- BF16 inputs, FP32 accumulation
// v_mfma_f32_16x16x32_bf16 (gfx950): operand lanes hold 8 consecutive k,
// A[i = l%16][k = 8(l/16) + v], B[k = 8(l/16) + v][j = l%16]; the
// accumulator's row for register r of lane l is 4(l/16) + r.  LDS tiles are
// [mn][k] (k contiguous) so each lane fetches its 8 values in one 16-byte
// read.  Complex storage of a bf16 matrix: (re, im) pairs, 4 bytes per
// element.  Both operands arrive in bf16: beta is converted once at create,
// psi and D P once per call (bf16_round), so the tiles of every M (or N)
// block read a quarter of the complex128 bytes and convert nothing.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
constexpr int BB_K = 32;

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// Rows of 40 bf16 (80 bytes): each group of 8 k starts 16-byte aligned, so
// a thread stores its 8 values of a row in one write, and the 16 rows a
// fragment read touches fall on distinct banks.
constexpr int BB_KP = BB_K + 8;
struct BfTile {
  unsigned short re[GB_M][BB_KP];
  unsigned short im[GB_M][BB_KP];
};
__device__ __forceinline__ uint4 bf_pack8(const unsigned short v[8]) {
  return uint4{v[0] | ((unsigned)v[1] << 16), v[2] | ((unsigned)v[3] << 16), v[4] | ((unsigned)v[5] << 16),
               v[6] | ((unsigned)v[7] << 16)};
}

// A thread's 8 values of a stage, kept as loaded between the global loads
// and the LDS store (so the loads of the next stage overlap the MFMAs of
// this one): bf16 (re, im) pairs packed re-low.
struct BfRawH {
  unsigned w[8];
};
__device__ __forceinline__ void bf_split(const BfRawH &r, unsigned short re[8], unsigned short im[8]) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    re[u] = (unsigned short)(r.w[u] & 0xFFFFu);
    im[u] = (unsigned short)(r.w[u] >> 16);
  }
}

// K-contiguous source, 64 columns x 32 k: thread t: column t/4, k = 8*(t%4) .. +7.
__device__ __forceinline__ void bf_load_kc(const ushort2 *__restrict__ P, int64_t ld, int64_t k0,
                                           int64_t c0, int64_t K, int64_t C, BfRawH &r) {
  const int t = threadIdx.x;
  const int64_t c = c0 + (t >> 2);
  const int64_t k = k0 + ((t & 3) << 3);
  const ushort2 *q = P + c * ld + k;
  if (c < C && k + 7 < K && (reinterpret_cast<uintptr_t>(q) & 15) == 0) {
    // 8 (re, im) pairs, 32 bytes: two 16-byte loads
    const uint4 v0 = reinterpret_cast<const uint4 *>(q)[0], v1 = reinterpret_cast<const uint4 *>(q)[1];
    const unsigned w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int u = 0; u < 8; ++u) r.w[u] = w[u];
    return;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    ushort2 v = ushort2{0, 0};
    if (c < C && k + u < K) v = P[c * ld + k + u];
    r.w[u] = (unsigned)v.x | ((unsigned)v.y << 16);
  }
}
template <typename R> __device__ __forceinline__ void bf_store_kc(BfTile &T, const R &r) {
  const int t = threadIdx.x;
  const int c = t >> 2;
  const int k = (t & 3) << 3;
  unsigned short re[8], im[8];
  bf_split(r, re, im);
  *reinterpret_cast<uint4 *>(&T.re[c][k]) = bf_pack8(re);
  *reinterpret_cast<uint4 *>(&T.im[c][k]) = bf_pack8(im);
}
// M-contiguous bf16 source, 64 m x 32 k: thread t: m = t%64, k = 8*(t/64) .. +7
// (each load instruction reads 64 consecutive m of one k across the wave).
__device__ __forceinline__ void bf_load_mc(const ushort2 *__restrict__ P, int64_t ld, int64_t m0,
                                           int64_t k0, int64_t M, int64_t K, BfRawH &r) {
  const int t = threadIdx.x;
  const int64_t m = m0 + (t & 63);
  const int64_t k = k0 + ((t >> 6) << 3);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    ushort2 v = ushort2{0, 0};
    if (m < M && k + u < K) v = P[(k + u) * ld + m];
    r.w[u] = (unsigned)v.x | ((unsigned)v.y << 16);
  }
}
__device__ __forceinline__ void bf_store_mc(BfTile &T, const BfRawH &r) {
  const int t = threadIdx.x;
  const int m = t & 63;
  const int k = (t >> 6) << 3;
  unsigned short re[8], im[8];
  bf_split(r, re, im);
  *reinterpret_cast<uint4 *>(&T.re[m][k]) = bf_pack8(re);
  *reinterpret_cast<uint4 *>(&T.im[m][k]) = bf_pack8(im);
}

struct AccF {
  f4_t rr[2][2], ii[2][2], ri[2][2], ir[2][2];
};

// 8 consecutive k of one row (16-byte aligned: rows are 80 bytes, k % 8 == 0)
__device__ __forceinline__ bf8_t bf_frag(const unsigned short (*S)[BB_KP], int row, int k) {
  return __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(&S[row][k]));
}

__device__ __forceinline__ void bf_stage(const BfTile &At, const BfTile &Bt, AccF &acc, int wm, int wn) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15;
  const int lk = (lane >> 4) << 3;
  bf8_t ar[2], ai[2], br[2], bi[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    ar[i] = bf_frag(At.re, wm * 32 + i * 16 + lr, lk);
    ai[i] = bf_frag(At.im, wm * 32 + i * 16 + lr, lk);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    br[j] = bf_frag(Bt.re, wn * 32 + j * 16 + lr, lk);
    bi[j] = bf_frag(Bt.im, wn * 32 + j * 16 + lr, lk);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc.rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br[j], ar[i], acc.rr[i][j], 0, 0, 0);
      acc.ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi[j], ai[i], acc.ii[i][j], 0, 0, 0);
      acc.ri[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi[j], ar[i], acc.ri[i][j], 0, 0, 0);
      acc.ir[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br[j], ai[i], acc.ir[i][j], 0, 0, 0);
    }
}

template <bool CONJ_A, typename F>
__device__ __forceinline__ void bf_out(const AccF &acc, int wm, int wn, F &&f) {
  const int lane = threadIdx.x & 63;
  const int lm = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double rr = acc.rr[i][j][r], ii = acc.ii[i][j][r];
        const double ri = acc.ri[i][j][r], ir = acc.ir[i][j][r];
        const double re = CONJ_A ? rr + ii : rr - ii;
        const double im = CONJ_A ? ri - ir : ri + ir;
        f(wm * 32 + i * 16 + lm, wn * 32 + j * 16 + 4 * (lane >> 4) + r, re, im);
      }
}

__global__ __launch_bounds__(G_THR, 2) void k_zgemm_cn_bf16(int64_t M, int64_t N, int64_t K,
                                                            const ushort2 *__restrict__ A, int64_t lda,
                                                            const ushort2 *__restrict__ B, int64_t ldb,
                                                            double2 *__restrict__ C, int64_t ldc,
                                                            int64_t kchunk, int direct, int64_t nsplit) {
  __shared__ __align__(16) BfTile At, Bt;
  int64_t t, m0, n0, kz;
  if (!xcd_tile(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N) * nsplit, &t)) return;
  tile_mnz(t, M, N, &m0, &n0, &kz);
  const int64_t kb = kz * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  AccF acc;
  const f4_t z = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc.rr[i][j] = acc.ii[i][j] = acc.ri[i][j] = acc.ir[i][j] = z;
  BfRawH ra, rb;
  if (kb < ke) {
    bf_load_kc(A, lda, kb, m0, ke, M, ra);
    bf_load_kc(B, ldb, kb, n0, ke, N, rb);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += BB_K) {
    bf_store_kc(At, ra);
    bf_store_kc(Bt, rb);
    __syncthreads();
    if (k0 + BB_K < ke) {
      bf_load_kc(A, lda, k0 + BB_K, m0, ke, M, ra);
      bf_load_kc(B, ldb, k0 + BB_K, n0, ke, N, rb);
    }
    bf_stage(At, Bt, acc, wm, wn);
    __syncthreads();
  }
  double2 *out = direct ? C : C + kz * M * N;
  const int64_t ldo = direct ? ldc : M;
  bf_out<true>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
    const int64_t m = m0 + mi, n = n0 + ni;
    if (m < M && n < N) out[n * ldo + m] = double2{re, im};
  });
}

__global__ __launch_bounds__(G_THR, 2) void k_zgemm_nn_bf16(int64_t M, int64_t N, int64_t K,
                                                            double alpha, const ushort2 *__restrict__ A,
                                                            int64_t lda, const ushort2 *__restrict__ B,
                                                            int64_t ldb, double beta,
                                                            double2 *__restrict__ C, int64_t ldc) {
  __shared__ __align__(16) BfTile At, Bt;
  int64_t t, m0, n0, kz;
  if (!xcd_tile(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N), &t)) return;
  tile_mnz(t, M, N, &m0, &n0, &kz);
  const int wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  AccF acc;
  const f4_t z = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc.rr[i][j] = acc.ii[i][j] = acc.ri[i][j] = acc.ir[i][j] = z;
  BfRawH ra, rb;
  if (K > 0) {
    bf_load_mc(A, lda, m0, 0, M, K, ra);
    bf_load_kc(B, ldb, 0, n0, K, N, rb);
  }
  for (int64_t k0 = 0; k0 < K; k0 += BB_K) {
    bf_store_mc(At, ra);
    bf_store_kc(Bt, rb);
    __syncthreads();
    if (k0 + BB_K < K) {
      bf_load_mc(A, lda, m0, k0 + BB_K, M, K, ra);
      bf_load_kc(B, ldb, k0 + BB_K, n0, K, N, rb);
    }
    bf_stage(At, Bt, acc, wm, wn);
    __syncthreads();
  }
  bf_out<false>(acc, wm, wn, [&](int mi, int ni, double re, double im) {
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

// complex128 -> float2 / bf16 pairs (round to nearest even), [rows][ld] layout kept
__global__ void k_cvt_c64(const double2 *__restrict__ src, float2 *__restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = float2{(float)src[e].x, (float)src[e].y};
}
__global__ void k_cvt_bf16(const double2 *__restrict__ src, ushort2 *__restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = ushort2{bf16_rne((float)src[e].x), bf16_rne((float)src[e].y)};
}

// [cols][lds] complex128 -> [cols][ldd] bf16 pairs, rows 0..rows-1 of each column
__global__ void k_cvt_bf16_2d(const double2 *__restrict__ src, int64_t lds, ushort2 *__restrict__ dst,
                              int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t tot = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    const double2 v = src[c * lds + r];
    dst[c * ldd + r] = ushort2{bf16_rne((float)v.x), bf16_rne((float)v.y)};
  }
}

int bf16_round(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return PW_OK;
  int64_t blocks = (rows * cols + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_cvt_bf16_2d, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const double2 *>(src),
                     lds, static_cast<ushort2 *>(dst), ldd, rows, cols);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int convert_beta(const void *src, void *dst, int64_t n, int prec, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (prec == PW_MIXED_FP32)
    hipLaunchKernelGGL(k_cvt_c64, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const double2 *>(src),
                       static_cast<float2 *>(dst), n);
  else
    hipLaunchKernelGGL(k_cvt_bf16, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const double2 *>(src),
                       static_cast<ushort2 *>(dst), n);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// FP64 products in the three-multiplication form unless PW_GEMM_3M=0
static bool gemm_3m() {
  static const int v = env_switch("PW_GEMM_3M", 1);
  return v != 0;
}

int choose_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N);
  // fill the 2 x 256 workgroup slots once, without a nearly empty second
  // round (rounding down), each workgroup with >= 32 K stages
  int64_t s = 512 / tiles;
  const int64_t maxs = (K + 32 * GB_K - 1) / (32 * GB_K);
  if (s > maxs) s = maxs;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

static int launch_reduce(int64_t M, int64_t N, int splits, void *part, void *C, int64_t ldc, hipStream_t s) {
  int64_t blocks = (M * N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, M, N, splits,
                     static_cast<const double2 *>(part), static_cast<double2 *>(C), ldc);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int zgemm_cn_p(int prec, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
               int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  if (splits < 1) splits = 1;
  const int kq = prec == PW_MIXED_BF16 ? BB_K : GB_K;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kq - 1) / kq * kq;
  if (kchunk <= 0) kchunk = kq;
  const int direct = (splits == 1) ? 1 : 0;
  void *out = direct ? C : part;
  const int64_t ns = splits;
  const dim3 grid = xcd_grid(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N) * ns);
  const double2 *Bd = static_cast<const double2 *>(B);
  double2 *O = static_cast<double2 *>(out);
  if (prec == PW_FP64 && gemm_3m())
    hipLaunchKernelGGL((k_zgemm_cn<MF64x3, double2>), grid, dim3(G_THR), 0, s, M, N, K,
                       static_cast<const double2 *>(A), lda, Bd, ldb, O, ldc, kchunk, direct, ns);
  else if (prec == PW_FP64)
    hipLaunchKernelGGL((k_zgemm_cn<MF64, double2>), grid, dim3(G_THR), 0, s, M, N, K,
                       static_cast<const double2 *>(A), lda, Bd, ldb, O, ldc, kchunk, direct, ns);
  else if (prec == PW_MIXED_FP32)
    hipLaunchKernelGGL((k_zgemm_cn<MF32, float2>), grid, dim3(G_THR), 0, s, M, N, K,
                       static_cast<const float2 *>(A), lda, Bd, ldb, O, ldc, kchunk, direct, ns);
  else
    hipLaunchKernelGGL(k_zgemm_cn_bf16, grid, dim3(G_THR), 0, s, M, N, K,
                       static_cast<const ushort2 *>(A), lda, static_cast<const ushort2 *>(B), ldb, O, ldc,
                       kchunk, direct, ns);
  if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  return direct ? PW_OK : launch_reduce(M, N, splits, part, C, ldc, s);
}

int zgemm_nn_p(int prec, int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
               const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  const dim3 grid = xcd_grid(((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N));
  const double2 *Bd = static_cast<const double2 *>(B);
  double2 *Cd = static_cast<double2 *>(C);
  if (prec == PW_FP64 && gemm_3m())
    hipLaunchKernelGGL((k_zgemm_nn<MF64x3, double2>), grid, dim3(G_THR), 0, s, M, N, K, alpha,
                       static_cast<const double2 *>(A), lda, Bd, ldb, beta, Cd, ldc);
  else if (prec == PW_FP64)
    hipLaunchKernelGGL((k_zgemm_nn<MF64, double2>), grid, dim3(G_THR), 0, s, M, N, K, alpha,
                       static_cast<const double2 *>(A), lda, Bd, ldb, beta, Cd, ldc);
  else if (prec == PW_MIXED_FP32)
    hipLaunchKernelGGL((k_zgemm_nn<MF32, float2>), grid, dim3(G_THR), 0, s, M, N, K, alpha,
                       static_cast<const float2 *>(A), lda, Bd, ldb, beta, Cd, ldc);
  else
    hipLaunchKernelGGL(k_zgemm_nn_bf16, grid, dim3(G_THR), 0, s, M, N, K, alpha,
                       static_cast<const ushort2 *>(A), lda, static_cast<const ushort2 *>(B), ldb, beta, Cd,
                       ldc);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int zgemm_cn(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
             int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s) {
  return zgemm_cn_p(PW_FP64, M, N, K, A, lda, B, ldb, C, ldc, splits, part, s);
}

int zgemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
             const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s) {
  return zgemm_nn_p(PW_FP64, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

}  // namespace pw
