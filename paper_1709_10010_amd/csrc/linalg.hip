// Dense FP64 linear algebra of the Davidson subspace (gfx950).
//
// The paper names subspace diagonalisation as the most expensive dense
// linear-algebra step of PWscf's iterative diagonalisation, done there with
// ScaLAPACK / ELPA on the linear-algebra group (section on new
// parallelization levels).  Here the subspace matrix lives on the GPU and
// is diagonalised by a cyclic two-sided Jacobi method (Hermitian case),
// chosen because every rotation of one round is independent:
//
//   round r pairs the indices (p, q) by the round-robin (circle) schedule;
//   phase 1 computes each pair's unitary J = D R, with D = diag(1, e^{-i phi})
//           taking a_pq = |a_pq| e^{i phi} to a real number and R the real
//           rotation (c, s) that zeroes it (t = tan of the smaller angle);
//   phase 2 applies  A <- J^H A J  block by block (each 2x2 block (a, b)
//           becomes J_a^H A_ab J_b) and accumulates  Z <- Z J.
// A sweep is m'-1 rounds (m' = m rounded up to even; a padding index has a
// zero row so its rotations are the identity).  Sweeps repeat until the
// off-diagonal mass is at the rounding level (4 m eps^2 of the total) or
// below a caller's absolute target, at most kMaxSweeps; elements below
// eps sqrt(|a_pp a_qq|) are not rotated.  The block variant can also count
// only the pairs that touch the lowest few diagonal entries, which is all a
// Davidson step needs of the subspace problem.
//
// Small matrices (m' <= 64) run in one workgroup with A and Z in LDS.
// Larger ones run by blocks of 16 indices: each block pair's 32 x 32
// sub-problem is solved in LDS by one workgroup, and the pair unitaries are
// then applied to the whole matrix and to Z (see the block-Jacobi section).
// Both are bounded: every wave leaves after at most kMaxSweeps sweeps.
//
// Also here: eigenvalue sort / Ritz-vector selection, Cholesky of a small
// Hermitian positive matrix with breakdown detection, the inverse of its
// triangular factor, and the small elementwise kernels of a Davidson step.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "common.h"

namespace pw {

constexpr int kMaxSweeps = 40;
// Stop when the off-diagonal mass is at most 4 m eps^2 of the total: after
// convergence every off-diagonal element sits at the rounding level eps |a|
// of its row, which leaves about m eps^2 of relative mass that no further
// sweep can remove.
constexpr double kOffRel = 4.0 * 4.93e-32;

struct Rot {
  double c, s, er, ei;  // J = [[c, s], [-s e, c e]],  e = er + i ei = e^{-i phi}
};

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cmc(double2 a, double2 b) {  // conj(a) * b
  return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }

__device__ __forceinline__ Rot make_rot(double alpha, double gamma, double2 beta) {
  Rot r{1.0, 0.0, 1.0, 0.0};
  const double ab = sqrt(beta.x * beta.x + beta.y * beta.y);
  // threshold Jacobi: an element below the rounding level of its diagonal
  // pair is left alone (no rotation), so converged matrices stop changing
  if (ab == 0.0 || ab <= 1e-300 || ab <= 1e-16 * sqrt(fabs(alpha * gamma))) return r;
  const double tau = (gamma - alpha) / (2.0 * ab);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t);
  r.c = c;
  r.s = t * c;
  r.er = beta.x / ab;   // e^{-i phi} = conj(beta) / |beta|
  r.ei = -beta.y / ab;
  return r;
}

// The same rotation from the hardware reciprocal and reciprocal square root,
// each refined by one Newton step (a few ulps instead of correct rounding):
// a shorter dependency chain for solves that stop at a target well above
// the rounding level.  The threshold test is done on squares.
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ Rot make_rot_fast(double alpha, double gamma, double2 beta) {
  const double ab2 = beta.x * beta.x + beta.y * beta.y;
  // branch-free: the identity is selected at the end (the inputs of every
  // rotation can then be read together)
  const bool id = !(ab2 > 1e-300) || ab2 <= 1e-32 * fabs(alpha * gamma);
  const double ab2s = id ? 1.0 : ab2;
  // with d = gamma - alpha and rho = sqrt(d^2 + 4 |beta|^2): cos 2theta =
  // |d| / rho, c = sqrt((1 + cos 2theta) / 2), s = sign(d) |beta| / (rho c)
  // -- the angle of t = tan theta above, with no cancellation
  const double d = id ? 0.0 : gamma - alpha;
  const double rab = rsq_nr(ab2s);
  const double rrho = rsq_nr(fma(d, d, 4.0 * ab2s));
  const double h = fma(0.5 * fabs(d), rrho, 0.5);
  const double rh = rsq_nr(h);
  Rot r;
  r.c = id ? 1.0 : h * rh;
  r.s = id ? 0.0 : (d >= 0.0 ? 1.0 : -1.0) * (ab2s * rab) * rrho * rh;
  r.er = id ? 1.0 : beta.x * rab;
  r.ei = id ? 0.0 : -beta.y * rab;
  return r;
}

// J entries: j11 = c, j12 = s, j21 = -s e, j22 = c e.
__device__ __forceinline__ void rot_entries(const Rot &r, double2 &j11, double2 &j12, double2 &j21,
                                            double2 &j22) {
  j11 = double2{r.c, 0.0};
  j12 = double2{r.s, 0.0};
  j21 = double2{-r.s * r.er, -r.s * r.ei};
  j22 = double2{r.c * r.er, r.c * r.ei};
}

// Indices of pair k in round r for m' (even) indices.
__device__ __forceinline__ void pair_of(int k, int r, int mp, int *p, int *q) {
  const int n1 = mp - 1;
  // 0 <= r < n1 and 0 <= k < mp / 2, so each sum needs at most one wrap
  if (k == 0) {
    *p = 0;
    *q = 1 + r;
  } else {
    const int a = k + r;
    *p = 1 + (a >= n1 ? a - n1 : a);
    *q = 1 + (r >= k ? r - k : n1 - k + r);
  }
}

// New 2x2 block = Ja^H [a b; c d] Jb, with [a b; c d] = A[{pa,qa}][{pb,qb}].
__device__ __forceinline__ void update_block(double2 &a, double2 &b, double2 &c, double2 &d,
                                             const Rot &ra, const Rot &rb) {
  double2 a11, a12, a21, a22, b11, b12, b21, b22;
  rot_entries(ra, a11, a12, a21, a22);
  rot_entries(rb, b11, b12, b21, b22);
  // T = X Jb
  const double2 t11 = cadd(cm(a, b11), cm(b, b21));
  const double2 t12 = cadd(cm(a, b12), cm(b, b22));
  const double2 t21 = cadd(cm(c, b11), cm(d, b21));
  const double2 t22 = cadd(cm(c, b12), cm(d, b22));
  // Ja^H T: (Ja^H)_11 = conj(a11), _12 = conj(a21), _21 = conj(a12), _22 = conj(a22)
  a = cadd(cmc(a11, t11), cmc(a21, t21));
  b = cadd(cmc(a11, t12), cmc(a21, t22));
  c = cadd(cmc(a12, t11), cmc(a22, t21));
  d = cadd(cmc(a12, t12), cmc(a22, t22));
}

__device__ __forceinline__ void update_zrow(double2 &zp, double2 &zq, const Rot &r) {
  double2 j11, j12, j21, j22;
  rot_entries(r, j11, j12, j21, j22);
  const double2 np = cadd(cm(zp, j11), cm(zq, j21));
  const double2 nq = cadd(cm(zp, j12), cm(zq, j22));
  zp = np;
  zq = nq;
}

// X <- J_a^H X J_b for the 2x2 block X = [a b; c d] (rows p_a, q_a; columns
// p_b, q_b).  J = diag(1, e) R with R = [[c, s], [-s, c]] real, so the phase
// scales row q_a by conj(e_a) and column q_b by e_b, then the real rotations
// mix the rows and the columns.
__device__ __forceinline__ void rotate_block(double2 &a, double2 &b, double2 &c, double2 &d, const Rot &ra,
                                             const Rot &rb) {
  const double2 eb{rb.er, rb.ei}, eac{ra.er, -ra.ei};
  b = cm(b, eb);
  d = cm(eac, cm(d, eb));
  c = cm(eac, c);
  // columns: (x, y) -> (c x - s y, s x + c y)
  const double2 a1{rb.c * a.x - rb.s * b.x, rb.c * a.y - rb.s * b.y};
  const double2 b1{rb.s * a.x + rb.c * b.x, rb.s * a.y + rb.c * b.y};
  const double2 c1{rb.c * c.x - rb.s * d.x, rb.c * c.y - rb.s * d.y};
  const double2 d1{rb.s * c.x + rb.c * d.x, rb.s * c.y + rb.c * d.y};
  // rows: (u, v) -> (c u - s v, s u + c v)
  a = double2{ra.c * a1.x - ra.s * c1.x, ra.c * a1.y - ra.s * c1.y};
  c = double2{ra.s * a1.x + ra.c * c1.x, ra.s * a1.y + ra.c * c1.y};
  b = double2{ra.c * b1.x - ra.s * d1.x, ra.c * b1.y - ra.s * d1.y};
  d = double2{ra.s * b1.x + ra.c * d1.x, ra.s * b1.y + ra.c * d1.y};
}

// (z_p, z_q) <- (z_p, z_q) J for one row of the accumulated unitary
__device__ __forceinline__ void rotate_cols(double2 &zp, double2 &zq, const Rot &r) {
  const double2 y = cm(zq, double2{r.er, r.ei});
  const double2 x = zp;
  zp = double2{r.c * x.x - r.s * y.x, r.c * x.y - r.s * y.y};
  zq = double2{r.s * x.x + r.c * y.x, r.s * x.y + r.c * y.y};
}

// ---------------------------------------------------------------- LDS Jacobi
// A: m x m (lda), Hermitian; on exit w[i] = eigenvalue i (unsorted), Z (ldz)
// the eigenvectors (column i) and A overwritten by Z^H A Z.  mp = m rounded
// up to even <= 64.  Sweeps stop at the rounding level or once the
// off-diagonal mass is at most off_abs^2 (off_abs > 0 also selects the
// short-chain rotations).  A round's (np)^2 2 x 2 block updates and mp np
// eigenvector updates are spread over kJacThreads threads: 1024 above 16
// rows (one block and two eigenvector pairs each at m = 64), else 256.
template <int kJacThreads>
__global__ __launch_bounds__(kJacThreads) void k_jacobi_lds(double2 *__restrict__ Ain, int64_t lda,
                                                    int m, double *__restrict__ w,
                                                    double2 *__restrict__ Z, int64_t ldz,
                                                    int *__restrict__ sweeps_out, double off_abs) {
  constexpr int MP = 64;
  __shared__ double2 A[MP][MP + 1];
  __shared__ double2 Zs[MP][MP + 1];
  __shared__ Rot rot[MP / 2];
  __shared__ double red[2 * (kJacThreads / 64)];
  __shared__ int done;
  const int tid = threadIdx.x;
  const int mp = (m + 1) & ~1;
  const int np = mp / 2;
  for (int e = tid; e < mp * mp; e += kJacThreads) {
    const int i = e % mp, j = e / mp;
    A[i][j] = (i < m && j < m) ? Ain[i + j * lda] : double2{0.0, 0.0};
    Zs[i][j] = double2{i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    // convergence test on the current matrix
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < mp * mp; e += kJacThreads) {
      const int i = e % mp, j = e / mp;
      const double v = A[i][j].x * A[i][j].x + A[i][j].y * A[i][j].y;
      tot += v;
      if (i != j) off += v;
    }
    // summed within each wave by shuffles, then over the waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = off;
      red[kJacThreads / 64 + (tid >> 6)] = tot;
    }
    __syncthreads();
    if (tid == 0) {
      double offs = 0.0, tots = 0.0;
      for (int v = 0; v < kJacThreads / 64; ++v) {
        offs += red[v];
        tots += red[kJacThreads / 64 + v];
      }
      done = (offs <= fmax(kOffRel * (double)mp * tots, off_abs * off_abs)) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < mp - 1; ++r) {
      if (tid < np) {
        int p, q;
        pair_of(tid, r, mp, &p, &q);
        rot[tid] = off_abs > 0.0 ? make_rot_fast(A[p][p].x, A[q][q].x, A[p][q])
                                 : make_rot(A[p][p].x, A[q][q].x, A[p][q]);
      }
      __syncthreads();
      for (int e = tid; e < np * np; e += kJacThreads) {
        const int ka = e % np, kb = e / np;
        int pa, qa, pb, qb;
        pair_of(ka, r, mp, &pa, &qa);
        pair_of(kb, r, mp, &pb, &qb);
        double2 a = A[pa][pb], b = A[pa][qb], c = A[qa][pb], d = A[qa][qb];
        rotate_block(a, b, c, d, rot[ka], rot[kb]);
        A[pa][pb] = a;
        A[pa][qb] = b;
        A[qa][pb] = c;
        A[qa][qb] = d;
      }
      for (int e = tid; e < mp * np; e += kJacThreads) {
        const int i = e % mp, kb = e / mp;
        int pb, qb;
        pair_of(kb, r, mp, &pb, &qb);
        rotate_cols(Zs[i][pb], Zs[i][qb], rot[kb]);
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < m; i += kJacThreads) w[i] = A[i][i].x;
  for (int e = tid; e < m * m; e += kJacThreads) {
    const int i = e % m, j = e / m;
    Z[i + j * ldz] = Zs[i][j];
    Ain[i + j * lda] = A[i][j];
  }
  if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}


// ---------------------------------------------------------------- block Jacobi
// Indices are grouped into blocks of kBJ.  A sweep is one intra round, which
// pairs blocks 2P and 2P+1 and diagonalises each pair's 2kBJ x 2kBJ
// sub-matrix with one full sweep of scalar rotations (every index pair
// inside a block is rotated there), followed by 2k-1 cross rounds, which
// pair the 2k blocks by the circle schedule and rotate only index pairs
// (i in I, j in J), kBJ steps of kBJ disjoint rotations.  Together every
// off-diagonal index pair is rotated at least once per sweep, as in a cyclic
// scalar sweep (the pairs across blocks 2P and 2P+1 twice: a circle round
// pairs those blocks again), at half the steps of diagonalising every pair
// problem in full.
//   k_bj_inner  (one workgroup per block pair) runs the steps in LDS and
//               stores the pair's accumulated unitary U_P;
//   k_bj_apply  replaces every 2kBJ x 2kBJ block A_PQ (P <= Q) by
//               U_P^H A_PQ U_Q, mirrors it into A_QP, and every row chunk of
//               Z[:, Q] by Z[:, Q] U_Q (each block owned by one workgroup, so
//               the update is in place).
constexpr int kBJ = 16;
constexpr int kSub = 2 * kBJ;

// Blocks (I, J) of pair p in round r: r < 0 is the intra round (2p, 2p+1),
// otherwise the circle schedule over the nblk blocks.
__device__ __forceinline__ void bj_pair(int p, int r, int nblk, int *I, int *J) {
  if (r < 0) {
    *I = 2 * p;
    *J = 2 * p + 1;
  } else {
    pair_of(p, r, nblk, I, J);
  }
}

// global index of local index i (< kBJ: block I, else block J)
__device__ __forceinline__ int bj_row(int I, int J, int i) { return i < kBJ ? I * kBJ + i : J * kBJ + i - kBJ; }

// Rotation k at step st of a pair solve.  CROSS: index k of block I with
// index (k + st) mod kBJ of block J; otherwise the circle schedule over all
// 2kBJ indices.
template <bool CROSS>
__device__ __forceinline__ void step_pair(int k, int st, int *p, int *q) {
  if (CROSS) {
    *p = k;
    *q = kBJ + ((k + st) & (kBJ - 1));
  } else {
    pair_of(k, st, kSub, p, q);
  }
}

// Sum over the 256 threads of a block (4 waves) of two values.
__device__ __forceinline__ void block_sum256x2(double &u, double &v, double (*part)[4]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    u += __shfl_xor(u, o, 64);
    v += __shfl_xor(v, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = u;
    part[1][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  u = part[0][0] + part[0][1] + part[0][2] + part[0][3];
  v = part[1][0] + part[1][1] + part[1][2] + part[1][3];
}

// One block pair: the 2kBJ x 2kBJ sub-matrix S of A in LDS, 256 threads.
// Thread (ka, kb) = (tid / kBJ, tid % kBJ) owns, at each step, the 2x2 block
// of S at rotations (ka, kb) and the rows ka, ka + kBJ of the accumulated
// unitary at rotation kb; it recomputes the two rotations it needs from the
// current S (every thread gets the same bits), reads S from one LDS buffer
// and writes the other, so a step costs one barrier.
// A pair whose off-diagonal mass (CROSS: of the block A_IJ) is at most
// skip2, or at the rounding level, is left alone: rotated[p] = 0 and its U
// is not written; k_bj_apply then skips every block whose transforms are
// all identities.
static_assert(kSub == 32 && kBJ * kBJ == 256, "k_bj_inner maps one thread to each rotation pair");
template <bool CROSS, bool FAST>
__global__ __launch_bounds__(256) void k_bj_inner(const double2 *__restrict__ A, int64_t lda, int nblk,
                                                  int r, double2 *__restrict__ U, double skip2,
                                                  int *__restrict__ rotated) {
  __shared__ double2 S[2][kSub][kSub + 1];
  __shared__ double2 Q[kSub][kSub + 1];
  __shared__ double part[2][4];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  int I, J;
  bj_pair(p, r, nblk, &I, &J);
  double off = 0.0, tot = 0.0;
#pragma unroll
  for (int q = 0; q < kSub * kSub / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = e % kSub, j = e / kSub;
    const double2 v = A[bj_row(I, J, i) + (int64_t)bj_row(I, J, j) * lda];
    S[0][i][j] = v;
    Q[i][j] = double2{i == j ? 1.0 : 0.0, 0.0};
    const double v2 = v.x * v.x + v.y * v.y;
    tot += v2;
    if (CROSS ? ((i < kBJ) != (j < kBJ)) : (i != j)) off += v2;
  }
  block_sum256x2(off, tot, part);
  const bool skip = off <= kOffRel * (double)kSub * tot || off <= skip2;
  if (skip) {
    if (tid == 0) rotated[p] = 0;
    return;  // identity: U is not needed
  }
  if (tid == 0) rotated[p] = 1;
  constexpr int nsteps = CROSS ? kBJ : kSub - 1;
  const int ka = tid / kBJ, kb = tid % kBJ;
  int cur = 0;
  for (int st = 0; st < nsteps; ++st) {
    int pa, qa, pb, qb;
    step_pair<CROSS>(ka, st, &pa, &qa);
    step_pair<CROSS>(kb, st, &pb, &qb);
    const double2 (*Sc)[kSub + 1] = S[cur];
    double2 (*Sn)[kSub + 1] = S[cur ^ 1];
    // every LDS read of the step is issued before any arithmetic
    const double2 ba = Sc[pa][qa], bb = Sc[pb][qb];
    const double aa = Sc[pa][pa].x, ga = Sc[qa][qa].x, ab = Sc[pb][pb].x, gb = Sc[qb][qb].x;
    double2 a = Sc[pa][pb], b = Sc[pa][qb], c = Sc[qa][pb], d = Sc[qa][qb];
    double2 z0 = Q[ka][pb], z1 = Q[ka][qb], z2 = Q[ka + kBJ][pb], z3 = Q[ka + kBJ][qb];
    const Rot ra = FAST ? make_rot_fast(aa, ga, ba) : make_rot(aa, ga, ba);
    const Rot rb = FAST ? make_rot_fast(ab, gb, bb) : make_rot(ab, gb, bb);
    rotate_block(a, b, c, d, ra, rb);
    rotate_cols(z0, z1, rb);
    rotate_cols(z2, z3, rb);
    Sn[pa][pb] = a;
    Sn[pa][qb] = b;
    Sn[qa][pb] = c;
    Sn[qa][qb] = d;
    Q[ka][pb] = z0;
    Q[ka][qb] = z1;
    Q[ka + kBJ][pb] = z2;
    Q[ka + kBJ][qb] = z3;
    __syncthreads();
    cur ^= 1;
  }
  double2 *Up = U + (int64_t)p * kSub * kSub;
#pragma unroll
  for (int q = 0; q < kSub * kSub / 256; ++q) {
    const int e = tid + 256 * q;
    Up[e] = Q[e % kSub][e / kSub];
  }
}

// Workgroups 0 .. nA-1 (nA = npair (npair + 1) / 2) update the A blocks
// (P, Q), P <= Q, in row-major order; the next npair^2 update the Z row
// chunks (rows 2kBJ P .. +2kBJ, columns of pair Q).  Each thread computes a
// 2 x 2 tile of the 2kBJ x 2kBJ products from LDS; results leave through LDS
// so that every global store is along a column.
__global__ __launch_bounds__(256) void k_bj_apply(double2 *__restrict__ A, int64_t lda,
                                                  double2 *__restrict__ Z, int64_t ldz, int nblk, int r,
                                                  const double2 *__restrict__ U,
                                                  const int *__restrict__ rotated) {
  __shared__ double2 X[kSub][kSub + 1];   // X[col][row]: the block, then T, then the result
  __shared__ double2 UQ[kSub][kSub + 1];  // UQ[k][j] = U_Q(k, j)
  __shared__ double2 UP[kSub][kSub + 1];  // UP[k][i] = U_P(k, i)
  const int npair = nblk / 2;
  const int nA = npair * (npair + 1) / 2;
  int b = blockIdx.x;
  const bool isZ = b >= nA;
  int P, Qp;
  if (isZ) {
    b -= nA;
    P = b % npair;
    Qp = b / npair;
  } else {
    P = 0;
    while (b >= npair - P) {
      b -= npair - P;
      ++P;
    }
    Qp = P + b;
  }
  const bool rq = rotated[Qp] != 0;
  const bool rp = !isZ && rotated[P] != 0;
  // identity transforms leave the block as it is
  if (!rq && !rp) return;
  int QI, QJ, PI = 0, PJ = 0;
  bj_pair(Qp, r, nblk, &QI, &QJ);
  if (!isZ) bj_pair(P, r, nblk, &PI, &PJ);
  const int tid = threadIdx.x;
  const double2 *uq = U + (int64_t)Qp * kSub * kSub;
  const double2 *up = U + (int64_t)P * kSub * kSub;
#pragma unroll
  for (int q = 0; q < kSub * kSub / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = e % kSub, j = e / kSub;
    if (rq) UQ[i][j] = uq[e];
    if (rp) UP[i][j] = up[e];
    const int col = bj_row(QI, QJ, j);
    X[j][i] = isZ ? Z[(int64_t)P * kSub + i + (int64_t)col * ldz] : A[bj_row(PI, PJ, i) + (int64_t)col * lda];
  }
  __syncthreads();
  const int i0 = 2 * (tid % kBJ), j0 = 2 * (tid / kBJ);
  double2 t00, t01, t10, t11;
  if (rq) {
    // T = X U_Q
    t00 = t01 = t10 = t11 = double2{0.0, 0.0};
    // operands of 8 k at a time are read before they are used
#pragma unroll
    for (int k0 = 0; k0 < kSub; k0 += 8) {
      double2 x0[8], x1[8], u0[8], u1[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        x0[k] = X[k0 + k][i0];
        x1[k] = X[k0 + k][i0 + 1];
        u0[k] = UQ[k0 + k][j0];
        u1[k] = UQ[k0 + k][j0 + 1];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        t00 = cadd(t00, cm(x0[k], u0[k]));
        t01 = cadd(t01, cm(x0[k], u1[k]));
        t10 = cadd(t10, cm(x1[k], u0[k]));
        t11 = cadd(t11, cm(x1[k], u1[k]));
      }
    }
    __syncthreads();
    X[j0][i0] = t00;
    X[j0 + 1][i0] = t01;
    X[j0][i0 + 1] = t10;
    X[j0 + 1][i0 + 1] = t11;
    __syncthreads();
  }
  if (rp) {
    // out = U_P^H T
    t00 = t01 = t10 = t11 = double2{0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < kSub; k0 += 8) {
      double2 u0[8], u1[8], x0[8], x1[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        u0[k] = UP[k0 + k][i0];
        u1[k] = UP[k0 + k][i0 + 1];
        x0[k] = X[j0][k0 + k];
        x1[k] = X[j0 + 1][k0 + k];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        t00 = cadd(t00, cmc(u0[k], x0[k]));
        t01 = cadd(t01, cmc(u0[k], x1[k]));
        t10 = cadd(t10, cmc(u1[k], x0[k]));
        t11 = cadd(t11, cmc(u1[k], x1[k]));
      }
    }
    __syncthreads();
    X[j0][i0] = t00;
    X[j0 + 1][i0] = t01;
    X[j0][i0 + 1] = t10;
    X[j0 + 1][i0 + 1] = t11;
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kSub * kSub / 256; ++q) {
    const int e = tid + 256 * q;
    const int i = e % kSub, j = e / kSub;
    const int col = bj_row(QI, QJ, j);
    if (isZ) {
      Z[(int64_t)P * kSub + i + (int64_t)col * ldz] = X[j][i];
    } else {
      A[bj_row(PI, PJ, i) + (int64_t)col * lda] = X[j][i];
      // mirror: A_QP(i, j) = conj(A_PQ(j, i))
      if (P != Qp) {
        const double2 v = X[i][j];
        A[bj_row(QI, QJ, i) + (int64_t)bj_row(PI, PJ, j) * lda] = double2{v.x, -v.y};
      }
    }
  }
}

// off-diagonal and total mass of the mpb x mpb matrix -> acc[0..1] (acc zeroed by caller)
// (only pairs (i, j) with min(a_ii, a_jj) <= thr count as off-diagonal)
__global__ __launch_bounds__(256) void k_offnorm(const double2 *__restrict__ A, int64_t lda, int n,
                                                 double *__restrict__ acc, double thr) {
  __shared__ double red[2][256];
  double off = 0.0, tot = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double2 v = A[i + (int64_t)j * lda];
    const double a2 = v.x * v.x + v.y * v.y;
    tot += a2;
    if (i != j && fmin(A[i + (int64_t)i * lda].x, A[j + (int64_t)j * lda].x) <= thr) off += a2;
  }
  red[0][threadIdx.x] = off;
  red[1][threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], red[0][0]);
    atomicAdd(&acc[1], red[1][0]);
  }
}

// pad to mpb (multiple of 2 kBJ): zero rows / columns m .. mpb-1, identity Z
__global__ void k_bj_init(double2 *__restrict__ A, int64_t lda, int m, int mpb, double2 *__restrict__ Z,
                          int64_t ldz) {
  const int64_t tot = (int64_t)mpb * mpb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mpb), j = (int)(e / mpb);
    if (i >= m || j >= m) A[i + (int64_t)j * lda] = double2{0.0, 0.0};
    Z[i + (int64_t)j * ldz] = double2{i == j ? 1.0 : 0.0, 0.0};
  }
}

__global__ void k_diag_out(const double2 *__restrict__ A, int64_t lda, int m, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) w[i] = A[i + (int64_t)i * lda].x;
}

// ---------------------------------------------------------------- sort / select
// rank of each eigenvalue (ties by index); idx[rank] = i for rank < nsel.
__global__ void k_eig_rank(const double *__restrict__ w, int m, int nsel, double *__restrict__ wsel,
                           int *__restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double wi = w[i];
  int r = 0;
  for (int j = 0; j < m; ++j) {
    const double wj = w[j];
    r += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
  }
  if (r < nsel) {
    wsel[r] = wi;
    idx[r] = i;
  }
}

// Y[:, r] = Z[:, idx[r]] for r < nsel (Y: m x nsel, ldy).
__global__ void k_gather_cols(const double2 *__restrict__ Z, int64_t ldz, const int *__restrict__ idx,
                              int m, int nsel, double2 *__restrict__ Y, int64_t ldy) {
  const int64_t tot = (int64_t)m * nsel;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / m), i = (int)(e % m);
    Y[i + r * ldy] = Z[i + (int64_t)idx[r] * ldz];
  }
}

// H[r + r' ldh] = A[idx[r] + idx[r'] lda] for r, r' < m: the transformed
// matrix in the order of the selected eigenvalues.
__global__ void k_perm_sym(const double2 *__restrict__ A, int64_t lda, const int *__restrict__ idx, int m,
                           double2 *__restrict__ H, int64_t ldh) {
  const int64_t tot = (int64_t)m * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    H[r + c * ldh] = A[idx[r] + (int64_t)idx[c] * lda];
  }
}

// ---------------------------------------------------------------- Cholesky
// S (lds) Hermitian positive n x n -> L lower (ldl, upper part zeroed).
// flag[0] = first column whose pivot fell to <= rel * S_jj (or was not
// finite) + 1, else 0.  One workgroup.
__global__ __launch_bounds__(1024) void k_cholesky(const double2 *__restrict__ S, int64_t lds, int n,
                                                   double2 *__restrict__ L, int64_t ldl, double rel,
                                                   int *__restrict__ flag) {
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int64_t e = tid; e < (int64_t)n * n; e += blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    L[i + j * ldl] = (i >= j) ? S[i + j * lds] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double d = L[j + j * ldl].x;
      for (int k = 0; k < j; ++k) {
        const double2 v = L[j + k * ldl];
        d -= v.x * v.x + v.y * v.y;
      }
      const double s0 = S[j + j * lds].x;
      if (!(d > rel * s0) || !isfinite(d)) {
        if (!bad) bad = j + 1;
        d = 1.0;
      }
      piv = sqrt(d);
      L[j + j * ldl] = double2{piv, 0.0};
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int i = j + 1 + tid; i < n; i += blockDim.x) {
      double2 acc = L[i + j * ldl];
      for (int k = 0; k < j; ++k) {
        const double2 a = L[i + k * ldl], b = L[j + k * ldl];  // a * conj(b)
        acc.x -= a.x * b.x + a.y * b.y;
        acc.y -= a.y * b.x - a.x * b.y;
      }
      L[i + j * ldl] = double2{acc.x * inv, acc.y * inv};
    }
    __syncthreads();
  }
  if (tid == 0) *flag = bad;
}

// Blocked Cholesky in one workgroup (n <= kCholMaxN): right-looking over
// panels of kCholPB columns.  The panel (all rows below its top) is factored
// in LDS column by column; the trailing lower triangle is then updated from
// global memory with the panel's outer product.  Breakdown rule as in
// k_cholesky (pivot <= rel * S_jj or not finite: flag = column + 1, pivot 1).
constexpr int kCholPB = 16;
constexpr int kCholMaxN = 512;
__global__ __launch_bounds__(1024) void k_cholesky_blk(const double2 *__restrict__ S, int64_t lds, int n,
                                                       double2 *__restrict__ L, int64_t ldl, double rel,
                                                       int *__restrict__ flag) {
  extern __shared__ __align__(16) unsigned char smem_c[];
  double2 *P = reinterpret_cast<double2 *>(smem_c);  // [n][kCholPB + 1]
  constexpr int PS = kCholPB + 1;
  __shared__ double inv_piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    const int i = (int)(e % n), j = (int)(e / n);
    L[i + j * ldl] = (i >= j) ? S[i + j * lds] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += kCholPB) {
    const int jb = min(kCholPB, n - j0), nr = n - j0;
    for (int e = tid; e < nr * jb; e += 1024) {
      const int r = e % nr, c = e / nr;
      P[r * PS + c] = L[(j0 + r) + (int64_t)(j0 + c) * ldl];
    }
    __syncthreads();
    for (int c = 0; c < jb; ++c) {
      if (tid == 0) {
        double d = P[c * PS + c].x;
        const double s0 = S[(j0 + c) + (int64_t)(j0 + c) * lds].x;
        if (!(d > rel * s0) || !isfinite(d)) {
          if (!bad) bad = j0 + c + 1;
          d = 1.0;
        }
        const double piv = sqrt(d);
        P[c * PS + c] = double2{piv, 0.0};
        inv_piv = 1.0 / piv;
      }
      __syncthreads();
      const double iv = inv_piv;
      for (int r = c + 1 + tid; r < nr; r += 1024) {
        const double2 v = P[r * PS + c];
        P[r * PS + c] = double2{v.x * iv, v.y * iv};
      }
      __syncthreads();
      const int w = jb - c - 1;
      if (w > 0) {
        const int rows = nr - c - 1;
        for (int e = tid; e < rows * w; e += 1024) {
          const int r = c + 1 + e % rows, c2 = c + 1 + e / rows;
          if (r < c2) continue;
          const double2 a = P[r * PS + c], b = P[c2 * PS + c];  // a * conj(b)
          double2 t = P[r * PS + c2];
          t.x -= a.x * b.x + a.y * b.y;
          t.y -= a.y * b.x - a.x * b.y;
          P[r * PS + c2] = t;
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < nr * jb; e += 1024) {
      const int r = e % nr, c = e / nr;
      L[(j0 + r) + (int64_t)(j0 + c) * ldl] = (r >= c) ? P[r * PS + c] : double2{0.0, 0.0};
    }
    const int nt = nr - jb;
    for (int64_t e = tid; e < (int64_t)nt * nt; e += 1024) {
      const int i = (int)(e % nt), k = (int)(e / nt);
      if (i < k) continue;
      double2 acc = L[(j0 + jb + i) + (int64_t)(j0 + jb + k) * ldl];
      const double2 *pi = P + (jb + i) * PS, *pk = P + (jb + k) * PS;
      for (int c = 0; c < jb; ++c) {
        const double2 a = pi[c], b = pk[c];
        acc.x -= a.x * b.x + a.y * b.y;
        acc.y -= a.y * b.x - a.x * b.y;
      }
      L[(j0 + jb + i) + (int64_t)(j0 + jb + k) * ldl] = acc;
    }
    __syncthreads();
  }
  if (tid == 0) *flag = bad;
}

constexpr int kTriBS = 16;

// X = L^{-1} and B = X^H by block columns, one workgroup per block column
// J of kTriBS columns (they are independent): forward substitution over the
// block rows, X_JJ = L_JJ^{-1} and X_IJ = -L_II^{-1} sum_{K=J..I-1} L_IK X_KJ
// for I > J, with the block column held in LDS (dynamic, n x kTriBS) and
// each diagonal solve by one thread per column.  Block rows above J are
// zero.
__global__ __launch_bounds__(256) void k_trinv_cols(const double2 *__restrict__ L, int64_t ldl, int n,
                                                    double2 *__restrict__ X, int64_t ldx,
                                                    double2 *__restrict__ B, int64_t ldb) {
  constexpr int BS = kTriBS;
  extern __shared__ __align__(16) unsigned char smem_t[];
  double2 *Xc = reinterpret_cast<double2 *>(smem_t);  // [n][BS + 1], row i = global row i
  constexpr int XS = BS + 1;
  __shared__ double2 T[BS][BS + 1];
  __shared__ double2 Ld[BS][BS + 1];  // the diagonal block L_II
  const int J = blockIdx.x;
  const int nbk = (n + BS - 1) / BS;
  const int tid = threadIdx.x;
  const int r = tid / BS, c = tid % BS;  // element (r, c) of a BS x BS block
  const int j0 = J * BS;
  const int jc = j0 + c;                  // global column of this thread's element
  for (int I = J; I < nbk; ++I) {
    const int i0 = I * BS;
    // T = delta_IJ I - sum_{K=J..I-1} L_IK X_KJ (element (r, c))
    double2 acc = double2{(I == J && r == c) ? 1.0 : 0.0, 0.0};
    const int gi = i0 + r;
    if (gi < n && jc < n) {
      for (int k = j0; k < i0; ++k) {
        const double2 a = L[gi + (int64_t)k * ldl], x = Xc[k * XS + c];
        acc.x -= a.x * x.x - a.y * x.y;
        acc.y -= a.x * x.y + a.y * x.x;
      }
    }
    T[r][c] = acc;
    if (gi < n && i0 + c < n && c <= r) Ld[r][c] = L[gi + (int64_t)(i0 + c) * ldl];
    __syncthreads();
    // X_IJ = L_II^{-1} T: thread c < BS solves column c down the block rows
    // (L_II from LDS, so the solve's chain waits on no global read)
    if (tid < BS) {
      for (int rr = 0; rr < BS && i0 + rr < n; ++rr) {
        const int g = i0 + rr;
        double2 v = T[rr][tid];
        for (int k = 0; k < rr; ++k) {
          const double2 a = Ld[rr][k], x = Xc[(i0 + k) * XS + tid];
          v.x -= a.x * x.x - a.y * x.y;
          v.y -= a.x * x.y + a.y * x.x;
        }
        const double dinv = 1.0 / Ld[rr][rr].x;
        Xc[g * XS + tid] = double2{v.x * dinv, v.y * dinv};
      }
    }
    __syncthreads();
  }
  // X[:, J] (zero above the diagonal block) and B = X^H (rows J of B)
  for (int e = tid; e < n * BS; e += 256) {
    const int i = e % n, cc = e / n, col = j0 + cc;
    if (col >= n) continue;
    const double2 x = i >= j0 ? Xc[i * XS + cc] : double2{0.0, 0.0};
    const double2 xv = i >= col ? x : double2{0.0, 0.0};
    X[i + (int64_t)col * ldx] = xv;
    B[col + (int64_t)i * ldb] = double2{xv.x, -xv.y};
  }
}

// B = (L^{-1})^H (upper triangular, ldb): column c of X = L^{-1} e_c by
// forward substitution, one thread per column; B[c][i] = conj(X[i][c]).
__global__ void k_trinv_h(const double2 *__restrict__ L, int64_t ldl, int n, double2 *__restrict__ X,
                          int64_t ldx, double2 *__restrict__ B, int64_t ldb) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = 0; i < c; ++i) X[i + (int64_t)c * ldx] = double2{0.0, 0.0};
  for (int i = c; i < n; ++i) {
    double2 acc = double2{i == c ? 1.0 : 0.0, 0.0};
    for (int k = c; k < i; ++k) {
      const double2 a = L[i + k * ldl], x = X[k + (int64_t)c * ldx];
      acc.x -= a.x * x.x - a.y * x.y;
      acc.y -= a.x * x.y + a.y * x.x;
    }
    const double d = L[i + i * ldl].x;
    X[i + (int64_t)c * ldx] = double2{acc.x / d, acc.y / d};
  }
  for (int i = 0; i < n; ++i) {
    const double2 x = X[i + (int64_t)c * ldx];
    B[c + (int64_t)i * ldb] = double2{x.x, -x.y};
  }
}

// ---------------------------------------------------------------- small kernels
// R = HX - X diag(theta);  rho[n] = ||R_n||, xn2[n] = ||X_n||^2 if xn2 is
// given (one block per band).
__global__ __launch_bounds__(256) void k_residual(const double2 *__restrict__ X,
                                                  const double2 *__restrict__ HX,
                                                  const double *__restrict__ theta,
                                                  double2 *__restrict__ R, int64_t ld, int64_t npw,
                                                  double *__restrict__ rho, double *__restrict__ xn2) {
  __shared__ double red[256], redx[256];
  const int b = blockIdx.x;
  const double th = theta[b];
  double s = 0.0, q = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += 256) {
    const double2 x = X[b * ld + g], h = HX[b * ld + g];
    const double2 r = double2{h.x - th * x.x, h.y - th * x.y};
    R[b * ld + g] = r;
    s += r.x * r.x + r.y * r.y;
    q += x.x * x.x + x.y * x.y;
  }
  red[threadIdx.x] = s;
  redx[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      redx[threadIdx.x] += redx[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rho[b] = sqrt(red[0]);
    if (xn2) xn2[b] = redx[0];
  }
}

// nrm2[b] = sum_g |T[b][g]|^2, one workgroup per column
template <bool ROOT>
__global__ __launch_bounds__(256) void k_colnorm2(const double2 *__restrict__ T, int64_t ld, int64_t npw,
                                                  double *__restrict__ nrm2) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += 256) {
    const double2 x = T[b * ld + g];
    s += x.x * x.x + x.y * x.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm2[b] = ROOT ? sqrt(red[0]) : red[0];
}

// Hermitise the new columns [m0, m1) of H (ldh): mirror the off-diagonal
// rectangle into rows, average the new diagonal block with its adjoint.
__global__ void k_hermitize(double2 *__restrict__ H, int64_t ldh, int m0, int m1) {
  const int64_t nn = (int64_t)(m1 - m0) * m1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = m0 + (int)(e / m1);
    const int i = (int)(e % m1);
    if (i < m0) {
      const double2 v = H[i + j * ldh];
      H[j + i * ldh] = double2{v.x, -v.y};
    } else if (i < j) {
      const double2 a = H[i + j * ldh], b = H[j + i * ldh];
      const double2 v = double2{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
      H[i + j * ldh] = v;
      H[j + i * ldh] = double2{v.x, -v.y};
    } else if (i == j) {
      H[i + j * ldh].y = 0.0;
    }
  }
}

// H[0:n, 0:n] = diag(theta)

// dst (m x n, ldd) = src (m x n, lds)
__global__ void k_copy_mat(const double2 *__restrict__ src, int64_t lds, double2 *__restrict__ dst,
                           int64_t ldd, int m, int n) {
  const int64_t nn = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    dst[i + j * ldd] = src[i + j * lds];
  }
}

// B[:, c] = U[:, keep[c]] / sqrt(lam[keep[c]]) (rank-revealing orthonormalisation)
__global__ void k_scaled_cols(const double2 *__restrict__ U, int64_t ldu, const double *__restrict__ lam,
                              const int *__restrict__ keep, int n, int nk, double2 *__restrict__ B,
                              int64_t ldb) {
  const int64_t nn = (int64_t)n * nk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    const int k = keep[c];
    const double s = 1.0 / sqrt(lam[k]);
    const double2 u = U[i + (int64_t)k * ldu];
    B[i + (int64_t)c * ldb] = double2{u.x * s, u.y * s};
  }
}

// T[i] = K(t/T_{idx[i]}) R[idx[i]] (TPA, or K = 1); tn from k_band_kinetic over X.
__device__ __forceinline__ double tpa_k2(double x) {
  const double num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0));
  const double x2 = x * x;
  return num / (num + 16.0 * x2 * x2);
}
__global__ void k_precond_idx(const double *__restrict__ kin, const double *__restrict__ tn,
                              const int *__restrict__ idx, const double2 *__restrict__ R, int64_t ldr,
                              double2 *__restrict__ T, int64_t ldt, int64_t npw, int kind) {
  const int i = blockIdx.y;
  const int n = idx[i];
  const double inv = 1.0 / tn[n];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = R[(int64_t)n * ldr + g];
    const double k = (kind == PW_PRECOND_TPA) ? tpa_k2(kin[g] * inv) : 1.0;
    T[(int64_t)i * ldt + g] = double2{k * v.x, k * v.y};
  }
}

// ---------------------------------------------------------------- launchers
static int grid_for(int64_t n, int bs = 256, int cap = 2048) {
  int64_t b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}


// Block Jacobi driver: A (lda >= mpb, mpb = m rounded up to 2 kBJ) is
// overwritten; Z (ldz >= mpb) receives the eigenvectors; uws holds the
// per-pair unitaries (mpb/kBJ/2 * (2 kBJ)^2 complex) and flags; acc >= 2
// doubles.  One host sync per sweep reads the off-diagonal mass.
// PW_BJ_CROSS=0 replaces the intra + cross rounds by 2k-1 rounds of full
// pair solves (every pair problem diagonalised by one scalar sweep).
static int bj_cross() {
  static const int v = env_switch("PW_BJ_CROSS", 1);
  return v;
}

template <bool FAST>
static void bj_round(bool cross, int npair, int nblk, int r, double2 *A, int64_t lda, double2 *Z, int64_t ldz,
                     double2 *U, double skip2, int *rotated, hipStream_t s) {
  if (cross)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_bj_inner<true, FAST>), dim3(npair), dim3(256), 0, s, A, lda, nblk, r, U,
                       skip2, rotated);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_bj_inner<false, FAST>), dim3(npair), dim3(256), 0, s, A, lda, nblk, r,
                       U, skip2, rotated);
  const int nA = npair * (npair + 1) / 2;
  hipLaunchKernelGGL(k_bj_apply, dim3(nA + npair * npair), dim3(256), 0, s, A, lda, Z, ldz, nblk, r, U, rotated);
}

static int eig_block(double2 *A, int64_t lda, int m, double *w, double2 *Z, int64_t ldz, void *uws,
                     double *acc, double *h_acc, hipStream_t s, double off_abs, int nwant) {
  std::vector<double> h_diag(nwant > 0 ? m : 0);
  const int mpb = (m + kSub - 1) / kSub * kSub;
  const int nblk = mpb / kBJ;
  const int npair = nblk / 2;
  double2 *U = static_cast<double2 *>(uws);
  int *rotated = reinterpret_cast<int *>(U + (int64_t)npair * kSub * kSub);
  const bool cross = bj_cross() != 0;
  // a pair below this mass is skipped: the pair problems of one sweep
  // (npair intra + nblk (nblk - 1) / 2 cross, or the latter alone) together
  // stay below the target
  const int nprob = cross ? npair + nblk * (nblk - 1) / 2 : nblk * (nblk - 1) / 2;
  const double skip2 = off_abs * off_abs / (double)std::max(1, nprob);
  // a target far above the rounding level allows the short-chain rotations
  const bool fast = off_abs > 0.0;
  hipLaunchKernelGGL(k_bj_init, dim3(grid_for((int64_t)mpb * mpb)), dim3(256), 0, s, A, lda, m, mpb, Z, ldz);
  if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (hipMemsetAsync(acc, 0, 2 * sizeof(double), s) != hipSuccess) return PW_ERR_HIP;
    double thr = INFINITY;
    if (nwant > 0 && nwant < m) {
      // the nwant-th smallest diagonal entry: pairs above it on both sides
      // are not counted
      hipLaunchKernelGGL(k_diag_out, dim3((m + 255) / 256), dim3(256), 0, s, A, lda, m, w);
      if (hipMemcpyAsync(h_diag.data(), w, m * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return PW_ERR_HIP;
      std::nth_element(h_diag.begin(), h_diag.begin() + (nwant - 1), h_diag.begin() + m);
      thr = h_diag[nwant - 1];
    }
    hipLaunchKernelGGL(k_offnorm, dim3(grid_for((int64_t)mpb * mpb, 256, 256)), dim3(256), 0, s, A, lda,
                       mpb, acc, thr);
    if (hipMemcpyAsync(h_acc, acc, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PW_ERR_HIP;
    // converged to the rounding level, or to the caller's target (or NaN)
    if (!(h_acc[0] > std::max(kOffRel * (double)mpb * h_acc[1], off_abs * off_abs))) break;
    // the intra round (r = -1) runs full pair solves; the circle rounds then
    // rotate the cross pairs only
    for (int r = cross ? -1 : 0; r < nblk - 1; ++r) {
      const bool c = cross && r >= 0;
      if (fast)
        bj_round<true>(c, npair, nblk, r, A, lda, Z, ldz, U, skip2, rotated, s);
      else
        bj_round<false>(c, npair, nblk, r, A, lda, Z, ldz, U, skip2, rotated, s);
    }
    if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  }
  hipLaunchKernelGGL(k_diag_out, dim3((m + 255) / 256), dim3(256), 0, s, A, lda, m, w);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// rot_ws: the per-pair unitaries of the block solver (lda x lda complex
// is enough).  Both solvers leave Z^H A Z in A.

// h_acc: two host doubles (pinned or pageable) owned by the caller, where the
// block solver reads back the off-diagonal and total mass once per sweep.
int eig_herm(double2 *A, int64_t lda, int m, double *w, double2 *Z, int64_t ldz, void *rot_ws,
             double *acc_ws, double *h_acc, int *sweeps, hipStream_t s, double off_abs, int nwant) {
  if (m <= 0) return PW_OK;
  const int mp = (m + 1) & ~1;
  if (mp <= 64) {
    if (mp > 16)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_jacobi_lds<1024>), dim3(1), dim3(1024), 0, s, A, lda, m, w, Z, ldz,
                         sweeps, off_abs);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_jacobi_lds<256>), dim3(1), dim3(256), 0, s, A, lda, m, w, Z, ldz,
                         sweeps, off_abs);
    return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
  }
  return eig_block(A, lda, m, w, Z, ldz, rot_ws, acc_ws, h_acc, s, off_abs, nwant);
}


int eig_select(const double *w, int m, int nsel, double *wsel, int *idx, const double2 *Z, int64_t ldz,
               double2 *Y, int64_t ldy, hipStream_t s, const double2 *A, int64_t lda, double2 *H,
               int64_t ldh) {
  hipLaunchKernelGGL(k_eig_rank, dim3((m + 255) / 256), dim3(256), 0, s, w, m, nsel, wsel, idx);
  if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  if (A && nsel == m) {
    hipLaunchKernelGGL(k_perm_sym, dim3(grid_for((int64_t)m * m)), dim3(256), 0, s, A, lda, idx, m, H, ldh);
    if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  }
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for((int64_t)m * nsel)), dim3(256), 0, s, Z, ldz, idx, m,
                     nsel, Y, ldy);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// PW_CHOL_IMPL=1 keeps the unblocked kernels (the path above kCholMaxN) at every size
static int chol_impl() {
  static const int v = env_switch("PW_CHOL_IMPL", 0);
  return v;
}

int cholesky(const double2 *S, int64_t lds, int n, double2 *L, int64_t ldl, double rel, int *flag,
             hipStream_t s) {
  if (n <= 0) return PW_OK;
  if (chol_impl() == 0 && n <= kCholMaxN) {
    const size_t lds_bytes = sizeof(double2) * (size_t)n * (kCholPB + 1);
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(k_cholesky_blk),
                                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                                        (int)(sizeof(double2) * kCholMaxN * (kCholPB + 1)));
    if (attr != hipSuccess) return PW_ERR_HIP;
    hipLaunchKernelGGL(k_cholesky_blk, dim3(1), dim3(1024), lds_bytes, s, S, lds, n, L, ldl, rel, flag);
  } else {
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, S, lds, n, L, ldl, rel, flag);
  }
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int trinv_h(const double2 *L, int64_t ldl, int n, double2 *X, int64_t ldx, double2 *B, int64_t ldb,
            hipStream_t s) {
  if (n <= 0) return PW_OK;
  if (chol_impl() == 0 && n <= kCholMaxN) {
    const size_t lds = sizeof(double2) * (size_t)n * (kTriBS + 1);
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(k_trinv_cols),
                                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                                        (int)(sizeof(double2) * kCholMaxN * (kTriBS + 1)));
    if (attr != hipSuccess) return PW_ERR_HIP;
    hipLaunchKernelGGL(k_trinv_cols, dim3((n + kTriBS - 1) / kTriBS), dim3(256), lds, s, L, ldl, n, X, ldx, B,
                       ldb);
  } else
    hipLaunchKernelGGL(k_trinv_h, dim3((n + 63) / 64), dim3(64), 0, s, L, ldl, n, X, ldx, B, ldb);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int col_norms2(const double2 *T, int64_t ld, int64_t npw, int n, double *nrm2, hipStream_t s) {
  if (n <= 0) return PW_OK;
  hipLaunchKernelGGL(k_colnorm2<false>, dim3(n), dim3(256), 0, s, T, ld, npw, nrm2);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// Y[:, r] = Z[:, idx[r]] for r < nsel, rows 0 .. m-1 (Y and Z distinct)
int gather_cols(const double2 *Z, int64_t ldz, const int *idx, int64_t m, int nsel, double2 *Y, int64_t ldy,
                hipStream_t s) {
  if (nsel <= 0 || m <= 0) return PW_OK;
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(m * nsel)), dim3(256), 0, s, Z, ldz, idx, (int)m, nsel, Y, ldy);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int col_norms(const double2 *T, int64_t ld, int64_t npw, int n, double *nrm, hipStream_t s) {
  if (n <= 0) return PW_OK;
  hipLaunchKernelGGL(k_colnorm2<true>, dim3(n), dim3(256), 0, s, T, ld, npw, nrm);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int residual(const double2 *X, const double2 *HX, const double *theta, double2 *R, int64_t ld,
             int64_t npw, int nb, double *rho, double *xn2, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, s, X, HX, theta, R, ld, npw, rho, xn2);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int hermitize(double2 *H, int64_t ldh, int m0, int m1, hipStream_t s) {
  hipLaunchKernelGGL(k_hermitize, dim3(grid_for((int64_t)(m1 - m0) * m1)), dim3(256), 0, s, H, ldh, m0, m1);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}


int copy_mat(const double2 *src, int64_t lds, double2 *dst, int64_t ldd, int m, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_mat, dim3(grid_for((int64_t)m * n)), dim3(256), 0, s, src, lds, dst, ldd, m, n);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int scaled_cols(const double2 *U, int64_t ldu, const double *lam, const int *keep, int n, int nk,
                double2 *B, int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_scaled_cols, dim3(grid_for((int64_t)n * nk)), dim3(256), 0, s, U, ldu, lam, keep,
                     n, nk, B, ldb);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int precond_idx(const double *kin, const double *tn, const int *idx, const double2 *R, int64_t ldr,
                double2 *T, int64_t ldt, int64_t npw, int nu, int kind, hipStream_t s) {
  if (nu <= 0) return PW_OK;
  int bx = (int)((npw + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_precond_idx, dim3(bx, nu), dim3(256), 0, s, kin, tn, idx, R, ldr, T, ldt, npw, kind);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

static_assert(kSub == kEighPad && kMaxSweeps == kEighMaxSweeps, "eigh_ws_bytes in common.h");

// The eigensolver on a workspace laid out as eigh_ws_bytes(m) describes.
// Every region is written before it is read (the copy of A, the identity
// start of Z, the padding of A, the accumulators cleared per sweep), so the
// workspace's earlier contents do not matter.
int eigh_impl(const void *A, int64_t lda, int m, double *w, void *Z, int64_t ldz, void *work,
              hipStream_t s) {
  const int64_t mp = (m + kSub - 1) / kSub * kSub;
  double2 *Ac = static_cast<double2 *>(work);
  double2 *Bw = Ac + mp * mp;
  double2 *Zw = Bw + mp * mp;
  double *wu = reinterpret_cast<double *>(Zw + mp * mp);
  double *acc = wu + mp;
  int *idx = reinterpret_cast<int *>(acc + 2 * kMaxSweeps + 2);
  int rc = copy_mat(static_cast<const double2 *>(A), lda, Ac, mp, m, m, s);
  double h_acc[2];
  if (rc == PW_OK) rc = eig_herm(Ac, mp, m, wu, Zw, mp, Bw, acc, h_acc, nullptr, s, 0.0, 0);
  if (rc == PW_OK)
    rc = eig_select(wu, m, m, w, idx, Zw, mp, static_cast<double2 *>(Z), ldz, s, nullptr, 0, nullptr, 0);
  return rc;
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_eigh_workspace(int32_t m, size_t *bytes) {
  PW_CHECK_ARG(m >= 1 && bytes, PW_ERR_INVALID, "pw_eigh_workspace: bad argument");
  *bytes = eigh_ws_bytes(m);
  return PW_OK;
}

pw_status pw_eigh(const void *A, int64_t lda, int32_t m, double *w, void *Z, int64_t ldz, void *work,
                  size_t work_bytes, void *stream) {
  PW_CHECK_ARG(A && w && Z && work && m >= 1 && lda >= m && ldz >= m, PW_ERR_INVALID,
               "pw_eigh: bad argument");
  PW_CHECK_ARG(work_bytes >= eigh_ws_bytes(m), PW_ERR_INVALID, "pw_eigh: workspace too small");
  const int rc = eigh_impl(A, lda, m, w, Z, ldz, work, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_eigh: launch failed");
  return rc;
}

}  // extern "C"
