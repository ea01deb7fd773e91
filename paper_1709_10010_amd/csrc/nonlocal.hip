// Nonlocal coefficients and the diagonal preconditioner.
//
//  k_apply_d : Q[n][j] = sum_{j' of atom(j)} D_a(j, j') P[n][j'] -- the
//              block-diagonal D_I,mn of eq. pauli_ks (one real symmetric
//              block per atom) applied to the projections p = <beta|psi>.
//  k_band_kinetic / k_tpa : Teter-Payne-Allan (1989) preconditioner
//              K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4),
//              x = t(G)/T_n, T_n = <x_n|t|x_n>/<x_n|x_n> (not in the paper:
//              the paper names the iterative diagonalisation but not its
//              preconditioner).
#include "common.h"

namespace pw {

__global__ void k_apply_d(const double *__restrict__ dij, const int32_t *__restrict__ pj_atom,
                          const int32_t *__restrict__ proj_off, const int32_t *__restrict__ dij_off,
                          const double2 *__restrict__ P, double2 *__restrict__ Q, int64_t nproj,
                          int nb) {
  const int64_t tot = nproj * (int64_t)nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e / nproj;
    const int j = (int)(e - n * nproj);
    const int a = pj_atom[j];
    const int o = proj_off[a];
    const int na = proj_off[a + 1] - o;
    const double *d = dij + dij_off[a] + (int64_t)(j - o) * na;
    const double2 *p = P + n * nproj + o;
    double re = 0.0, im = 0.0;
    for (int jj = 0; jj < na; ++jj) {
      re += d[jj] * p[jj].x;
      im += d[jj] * p[jj].y;
    }
    Q[e] = double2{re, im};
  }
}

int launch_apply_d(const double *dij, const int32_t *pj_atom, const int32_t *proj_off,
                   const int32_t *dij_off, const void *P, void *Q, int64_t nproj, int nb,
                   hipStream_t s) {
  const int64_t tot = nproj * (int64_t)nb;
  if (tot <= 0) return PW_OK;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_apply_d, dim3((unsigned)blocks), dim3(256), 0, s, dij, pj_atom, proj_off,
                     dij_off, static_cast<const double2 *>(P), static_cast<double2 *>(Q), nproj, nb);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// T_n = sum_G t(G)|x(G)|^2 / sum_G |x(G)|^2, one workgroup per band.
__global__ __launch_bounds__(256) void k_band_kinetic(const double *__restrict__ kin,
                                                      const double2 *__restrict__ x, int64_t ld,
                                                      int64_t npw, double *__restrict__ tn) {
  __shared__ double s_num[256], s_den[256];
  const int b = blockIdx.x;
  const double2 *xb = x + (int64_t)b * ld;
  double num = 0.0, den = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += 256) {
    const double2 v = xb[g];
    const double a2 = v.x * v.x + v.y * v.y;
    num += kin[g] * a2;
    den += a2;
  }
  s_num[threadIdx.x] = num;
  s_den[threadIdx.x] = den;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_num[threadIdx.x] += s_num[threadIdx.x + w];
      s_den[threadIdx.x] += s_den[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) tn[b] = s_num[0] / s_den[0];
}

__device__ __forceinline__ double tpa_k(double x) {
  const double num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0));
  const double x2 = x * x;
  return num / (num + 16.0 * x2 * x2);
}

__global__ void k_tpa(const double *__restrict__ kin, const double *__restrict__ tn,
                      const double2 *__restrict__ r, double2 *__restrict__ t, int64_t ld,
                      int64_t npw, int kind) {
  const int b = blockIdx.y;
  const double inv = 1.0 / tn[b];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = r[(int64_t)b * ld + g];
    const double k = (kind == PW_PRECOND_TPA) ? tpa_k(kin[g] * inv) : 1.0;
    t[(int64_t)b * ld + g] = double2{k * v.x, k * v.y};
  }
}

int band_kinetic(const double *kin, const void *x, int64_t ld, int64_t npw, int nb, double *tn,
                 hipStream_t s) {
  if (nb <= 0) return PW_OK;
  hipLaunchKernelGGL(k_band_kinetic, dim3(nb), dim3(256), 0, s, kin, static_cast<const double2 *>(x),
                     ld, npw, tn);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int launch_tpa(const double *kin, const void *x, const void *r, void *t, int64_t ld, int64_t npw,
               int nb, int kind, double *tn_work, hipStream_t s) {
  if (nb <= 0) return PW_OK;
  hipLaunchKernelGGL(k_band_kinetic, dim3(nb), dim3(256), 0, s, kin,
                     static_cast<const double2 *>(x), ld, npw, tn_work);
  if (hipGetLastError() != hipSuccess) return PW_ERR_HIP;
  int bx = (int)((npw + 255) / 256);
  if (bx > 512) bx = 512;
  hipLaunchKernelGGL(k_tpa, dim3(bx, nb), dim3(256), 0, s, kin, tn_work,
                     static_cast<const double2 *>(r), static_cast<double2 *>(t), ld, npw, kind);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

}  // namespace pw
