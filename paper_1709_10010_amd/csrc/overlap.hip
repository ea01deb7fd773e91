// Overlap S = 1 + sum_I sum_mn q_I,mn |beta_m^I><beta_n^I| of the generalized
// Kohn-Sham problem (H - eps S) psi = 0, the paper's general form
// (eq. pauli_ks), with the augmentation written on the same projectors as
// the nonlocal term.
//
// S differs from 1 only on the span of the projectors, so its inverse
// square root is exact and cheap: with beta = Q_b L^H (Cholesky-QR, Q_b
// orthonormal), S = 1 + Q_b M Q_b^H with M = L^H C L (C the block-diagonal
// q), M = W diag(lambda) W^H, and K = Q_b W (orthonormal columns):
//   S = 1 + K diag(lambda) K^H,   S^{-1/2} = 1 + K diag(f) K^H,
//   f = (1 + lambda)^{-1/2} - 1.
// K and f are built once at create (GEMMs, Cholesky and the subspace
// eigensolver, all on the GPU).  The Davidson then solves the standard
// problem of S^{-1/2} H S^{-1/2} for y = S^{1/2} x: a y-space that is
// orthonormal is an x-space that is S-orthonormal, and the Ritz values are
// those of the pencil (H, S).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace pw {

int cholesky(const double2 *S, int64_t lds, int n, double2 *L, int64_t ldl, double rel, int *flag,
             hipStream_t s);
int trinv_h(const double2 *L, int64_t ldl, int n, double2 *X, int64_t ldx, double2 *B, int64_t ldb,
            hipStream_t s);
int hermitize(double2 *H, int64_t ldh, int m0, int m1, hipStream_t s);

// Q[n][j] = f[j] P[n][j]  (P, Q [nb][nproj])
__global__ void k_scale_rows(const double2 *__restrict__ P, const double *__restrict__ f,
                             double2 *__restrict__ Q, int64_t nproj, int64_t nb) {
  const int64_t tot = nproj * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const double s = f[e % nproj];
    Q[e] = double2{s * P[e].x, s * P[e].y};
  }
}

// split-K factor of a K-long product that fits the handle's partials
static int fitting_splits(const pw_problem *p, int64_t M, int64_t N, int64_t K) {
  int splits = choose_splits(M, N, K);
  while (splits > 1 && (size_t)splits * M * N * 16 > p->part_bytes) --splits;
  return splits;
}

// Workspace regions of the overlap transform, carved by carve_problem when
// the problem has augmentation: K [nproj][ldb], f [nproj], and the set-up
// scratch (Q_b [nproj][ldb], five nproj^2 complex matrices, the
// eigensolver's workspace, one word).
void carve_overlap(pw_problem *p, Carve &c) {
  const size_t np = (size_t)p->nproj;
  p->d_K = c.take<double2>(np * p->ldb);
  p->d_sfac = c.take<double>(np);
  p->d_qij = c.take<double>(np * np);  // largest possible size of the concatenated blocks
  p->d_ov_qb = c.take<double2>(np * p->ldb);
  p->d_ov_mat = c.take<double2>(5 * np * np);
  p->d_ov_eig = c.take<char>(eigh_ws_bytes((int)np));
  p->d_ov_flag = c.take<int>(1);
}

int overlap_setup(pw_problem *p, const std::vector<double> &qblocks, const std::vector<int32_t> &poff,
                  hipStream_t s) {
  const int64_t np = p->nproj, npw = p->npw, ldb = p->ldb;
  double2 *G = p->d_ov_mat, *L = G + np * np, *Xi = L + np * np, *Bi = Xi + np * np, *C = Bi + np * np;
  double2 *Qb = p->d_ov_qb;
  int rc;
  PW_HIP(hipMemcpyAsync(p->d_qij, qblocks.data(), qblocks.size() * sizeof(double), hipMemcpyHostToDevice, s));
  // Gram matrix of the projectors and its Cholesky factor: beta = Q_b L^H
  if ((rc = zgemm_cn(np, np, npw, p->d_beta, ldb, p->d_beta, ldb, G, np, fitting_splits(p, np, np, npw),
                     p->d_part, s)) != PW_OK)
    return rc;
  if ((rc = cholesky(G, np, (int)np, L, np, 1e-12, p->d_ov_flag, s)) != PW_OK) return rc;
  int flag = 0;
  PW_HIP(hipMemcpyAsync(&flag, p->d_ov_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  PW_CHECK_ARG(flag == 0, PW_ERR_NUMERIC,
               "pw_problem_create: the projectors are linearly dependent on the sphere (their Gram matrix "
               "is singular), so the overlap cannot be factorised");
  if ((rc = trinv_h(L, np, (int)np, Xi, np, Bi, np, s)) != PW_OK) return rc;  // Bi = L^{-H}
  if ((rc = zgemm_nn(npw, np, np, 1.0, p->d_beta, ldb, Bi, np, 0.0, Qb, ldb, s)) != PW_OK) return rc;
  // C: the block-diagonal q as a dense complex matrix; M = L^H C L
  {
    std::vector<double2> Ch((size_t)np * np, double2{0.0, 0.0});
    int64_t off = 0;
    for (size_t a = 0; a + 1 < poff.size(); ++a) {
      const int o = poff[a], n = poff[a + 1] - poff[a];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ch[(size_t)(o + i) + (size_t)(o + j) * np] = double2{qblocks[off + i * n + j], 0.0};
      off += (int64_t)n * n;
    }
    PW_HIP(hipMemcpyAsync(C, Ch.data(), Ch.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    PW_HIP(hipStreamSynchronize(s));
  }
  if ((rc = zgemm_nn(np, np, np, 1.0, C, np, L, np, 0.0, Xi, np, s)) != PW_OK) return rc;        // C L
  if ((rc = zgemm_cn(np, np, np, L, np, Xi, np, G, np, 1, p->d_part, s)) != PW_OK) return rc;    // L^H C L
  if ((rc = hermitize(G, np, 0, (int)np, s)) != PW_OK) return rc;
  double *lam = reinterpret_cast<double *>(Bi);  // Bi is free again
  if ((rc = eigh_impl(G, np, (int)np, lam, C, np, p->d_ov_eig, s)) != PW_OK) return rc;         // M = W diag W^H
  if ((rc = zgemm_nn(npw, np, np, 1.0, Qb, ldb, C, np, 0.0, p->d_K, ldb, s)) != PW_OK) return rc;  // K = Q_b W
  std::vector<double> lh(np), f(np);
  PW_HIP(hipMemcpyAsync(lh.data(), lam, np * sizeof(double), hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  for (int64_t j = 0; j < np; ++j) {
    PW_CHECK_ARG(std::isfinite(lh[j]) && 1.0 + lh[j] > 1e-12, PW_ERR_NUMERIC,
                 "pw_problem_create: the overlap S = 1 + sum q |beta><beta| is not positive definite");
    f[j] = 1.0 / std::sqrt(1.0 + lh[j]) - 1.0;
  }
  PW_HIP(hipMemcpyAsync(p->d_sfac, f.data(), np * sizeof(double), hipMemcpyHostToDevice, s));
  PW_HIP(hipStreamSynchronize(s));
  return PW_OK;
}

// y = S^{-1/2} x = x + K diag(f) K^H x for nb bands (x and y distinct).
int sinvhalf(pw_problem *p, const void *x, int64_t ldx, void *y, int64_t ldy, int64_t nb, hipStream_t s) {
  if (nb <= 0) return PW_OK;
  const int64_t np = p->nproj, npw = p->npw;
  int rc = zgemm_cn(np, nb, npw, p->d_K, p->ldb, x, ldx, p->d_P, np, fitting_splits(p, np, nb, npw), p->d_part, s);
  if (rc != PW_OK) return rc;
  int64_t blocks = (np * nb + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const double2 *>(p->d_P),
                     p->d_sfac, static_cast<double2 *>(p->d_Q), np, nb);
  PW_HIP(hipGetLastError());
  PW_HIP(hipMemcpy2DAsync(y, ldy * sizeof(double2), x, ldx * sizeof(double2), npw * sizeof(double2), nb,
                          hipMemcpyDeviceToDevice, s));
  return zgemm_nn(npw, nb, np, 1.0, p->d_K, p->ldb, p->d_Q, np, 1.0, y, ldy, s);
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_spsi(pw_problem *p, const void *psi, int64_t ld_psi, void *spsi, int64_t ld_spsi, int64_t nbands,
                  void *stream) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_spsi: null handle");
  PW_CHECK_ARG(nbands >= 0 && nbands <= p->max_bands, PW_ERR_INVALID, "pw_spsi: nbands must be in 0 .. max_bands");
  if (nbands == 0) return PW_OK;
  PW_CHECK_ARG(psi && spsi && ld_psi >= p->npw && ld_spsi >= p->npw, PW_ERR_INVALID,
               "pw_spsi: null pointer or ld < npw");
  PW_CHECK_ARG(psi != spsi, PW_ERR_INVALID, "pw_spsi: psi and spsi must not be the same block");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t npw = p->npw, np = p->nproj;
  PW_HIP(hipMemcpy2DAsync(spsi, ld_spsi * sizeof(double2), psi, ld_psi * sizeof(double2), npw * sizeof(double2),
                          nbands, hipMemcpyDeviceToDevice, s));
  if (!p->gen) return PW_OK;
  int rc = zgemm_cn(np, nbands, npw, p->d_beta, p->ldb, psi, ld_psi, p->d_P, np, fitting_splits(p, np, nbands, npw),
                    p->d_part, s);
  if (rc == PW_OK)
    rc = launch_apply_d(p->d_qij, p->d_pj_atom, p->d_proj_off, p->d_dij_off, p->d_P, p->d_Q, np, (int)nbands, s);
  if (rc == PW_OK) rc = zgemm_nn(npw, nbands, np, 1.0, p->d_beta, p->ldb, p->d_Q, np, 1.0, spsi, ld_spsi, s);
  if (rc != PW_OK) set_error("pw_spsi: launch failed");
  return rc;
}

}  // extern "C"
