// Exact (Fock) exchange and its adaptively compressed form (CDNA4 / gfx950).
//
// The paper's exact-exchange section (eqs. Vx, Poisson, Vxace): for a state
// phi and the occupied states psi_j (spin-unpolarised, Hartree units),
//   (V_x phi)(r) = - sum_j w_j psi_j(r) v_j(r),  v_j(G) = 4 pi rho_j(G) / |G|^2,
//   rho_j(r) = psi_j^*(r) phi(r),
// and ACE: V_x ~ xi M^-1 xi^H with xi = V_x psi, M = <psi | xi>.  Gamma point
// only; the G = 0 term of the kernel is dropped, as for the Hartree potential.
//
// Every occupied state is brought to the full grid once (inverse 3D
// transforms, batched); the pair densities of one phi with a chunk of
// occupied states are formed, transformed, multiplied by the kernel and
// transformed back as one batch, and their products with the occupied states
// are summed in a fixed order.  For ACE, -M = L L^H (M is negative definite)
// and zeta = -xi L^-H, so that V_ace = xi M^-1 xi^H = -zeta zeta^H: in H psi
// the term costs the two GEMMs of a rank-nocc projector, like the nonlocal
// term, instead of nocc pair transforms per band.
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

namespace {

constexpr int kPairBatch = 16;  // pair densities transformed per batch

struct Recip3 {
  double b[9];
};

int64_t grid_len3(const pw_problem *p) { return (int64_t)p->nr[0] * p->nr[1] * p->nr[2]; }

double volume3(const pw_problem *p) {
  const double *a = p->A;
  return std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                   a[2] * (a[3] * a[7] - a[4] * a[6]));
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }

__global__ void k_zero_c(double2 *a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = double2{0.0, 0.0};
}

// grids[b][gfull[g]] = psi[b][g] for nb bands (the grids are zero elsewhere)
__global__ void k_scatter_full(const double2 *__restrict__ psi, int64_t ld, const int *__restrict__ gfull,
                               int64_t npw, double2 *__restrict__ grids, int64_t glen, int nb) {
  const int64_t tot = npw * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / npw, g = e - b * npw;
    grids[b * glen + gfull[g]] = psi[b * ld + g];
  }
}

// out[g] = sign * grid[gfull[g]] (+ out[g] with acc)
__global__ void k_gather_full(const double2 *__restrict__ grid, const int *__restrict__ gfull, int64_t npw,
                              double sign, int acc, double2 *__restrict__ out) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw; g += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = grid[gfull[g]];
    double2 o = double2{sign * v.x, sign * v.y};
    if (acc) {
      const double2 c = out[g];
      o.x += c.x;
      o.y += c.y;
    }
    out[g] = o;
  }
}

// 4 pi / |G|^2 at every grid point (signed indices), 0 at G = 0
__global__ void k_coulomb(double *__restrict__ kern, int n0, int n1, int n2, Recip3 B) {
  const int64_t len = (int64_t)n0 * n1 * n2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(i % n2);
    const int64_t r = i / n2;
    const int y = (int)(r % n1);
    const int x = (int)(r / n1);
    const double h = x <= n0 / 2 ? x : x - n0;
    const double k = y <= n1 / 2 ? y : y - n1;
    const double l = z <= n2 / 2 ? z : z - n2;
    const double gx = h * B.b[0] + k * B.b[3] + l * B.b[6];
    const double gy = h * B.b[1] + k * B.b[4] + l * B.b[7];
    const double gz = h * B.b[2] + k * B.b[5] + l * B.b[8];
    const double g2 = gx * gx + gy * gy + gz * gz;
    kern[i] = g2 > 0.0 ? 4.0 * M_PI / g2 : 0.0;
  }
}

// rho[b][r] = conj(U[b][r]) u[r] / Omega for nj occupied states
__global__ void k_pair_rho(const double2 *__restrict__ u, const double2 *__restrict__ U, int64_t glen, int nj,
                           double inv_omega, double2 *__restrict__ rho) {
  const int64_t tot = glen * nj;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % glen;
    const double2 a = U[e], b = u[r];
    rho[e] = double2{(a.x * b.x + a.y * b.y) * inv_omega, (a.x * b.y - a.y * b.x) * inv_omega};
  }
}

// rho[b][r] *= kern[r]
__global__ void k_kern_mul(double2 *__restrict__ rho, const double *__restrict__ kern, int64_t glen, int nj) {
  const int64_t tot = glen * nj;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const double k = kern[e % glen];
    rho[e] = double2{k * rho[e].x, k * rho[e].y};
  }
}

// acc[r] -= sum_{b < nj} w[b] U[b][r] v[b][r], in order of b
__global__ void k_exx_acc(double2 *__restrict__ acc, const double2 *__restrict__ U, const double2 *__restrict__ v,
                          const double *__restrict__ w, int64_t glen, int nj) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < glen; r += (int64_t)gridDim.x * blockDim.x) {
    double2 a = acc[r];
    for (int b = 0; b < nj; ++b) {
      const double2 x = U[(int64_t)b * glen + r], y = v[(int64_t)b * glen + r];
      const double wb = w[b];
      a.x -= wb * (x.x * y.x - x.y * y.y);
      a.y -= wb * (x.x * y.y + x.y * y.x);
    }
    acc[r] = a;
  }
}

// the workspace of the direct operator: kernel, the occupied states on the
// grid, one phi on the grid, one batch of pair potentials, the accumulator,
// the weights
struct VxWork {
  double *kern;
  double2 *U, *u, *rho, *acc;
  double *w;
};

VxWork carve_vx(const pw_problem *p, int64_t nocc, Carve &c) {
  const int64_t glen = grid_len3(p);
  VxWork v;
  v.kern = c.take<double>((size_t)glen);
  v.U = c.take<double2>((size_t)glen * nocc);
  v.u = c.take<double2>((size_t)glen);
  v.rho = c.take<double2>((size_t)glen * kPairBatch);
  v.acc = c.take<double2>((size_t)glen);
  v.w = c.take<double>((size_t)nocc);
  return v;
}

size_t vx_bytes(const pw_problem *p, int64_t nocc) {
  Carve c(nullptr);
  carve_vx(p, nocc, c);
  return c.size();
}

// out[i] = sign * V_x phi_i (+ out[i] with acc) for nphi bands
int vx_impl(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w_host,
            const void *phi, int64_t ld_phi, int64_t nphi, void *out, int64_t ld_out, double sign, void *work,
            hipStream_t s, bool acc = false) {
  const int64_t glen = grid_len3(p), npw = p->npw;
  Carve c(work);
  VxWork v = carve_vx(p, nocc, c);
  PW_HIP(hipMemcpyAsync(v.w, w_host, sizeof(double) * nocc, hipMemcpyHostToDevice, s));
  PW_HIP(hipStreamSynchronize(s));
  Recip3 B;
  std::copy(p->B, p->B + 9, B.b);
  hipLaunchKernelGGL(k_coulomb, dim3(blocks_for(glen)), dim3(256), 0, s, v.kern, p->nr[0], p->nr[1], p->nr[2], B);
  hipLaunchKernelGGL(k_zero_c, dim3(blocks_for(glen * nocc)), dim3(256), 0, s, v.U, glen * nocc);
  hipLaunchKernelGGL(k_scatter_full, dim3(blocks_for(npw * nocc)), dim3(256), 0, s,
                     static_cast<const double2 *>(psi_occ), ld_occ, p->d_gfull, npw, v.U, glen, (int)nocc);
  PW_HIP(hipGetLastError());
  int rc = launch_grid_fft(p->fft, v.U, (int)nocc, glen, true, s);
  if (rc != PW_OK) return rc;
  const double inv_omega = 1.0 / volume3(p);
  for (int64_t i = 0; i < nphi; ++i) {
    hipLaunchKernelGGL(k_zero_c, dim3(blocks_for(glen)), dim3(256), 0, s, v.u, glen);
    hipLaunchKernelGGL(k_scatter_full, dim3(blocks_for(npw)), dim3(256), 0, s,
                       static_cast<const double2 *>(phi) + i * ld_phi, ld_phi, p->d_gfull, npw, v.u, glen, 1);
    PW_HIP(hipGetLastError());
    if ((rc = launch_grid_fft(p->fft, v.u, 1, 0, true, s)) != PW_OK) return rc;
    hipLaunchKernelGGL(k_zero_c, dim3(blocks_for(glen)), dim3(256), 0, s, v.acc, glen);
    for (int64_t j0 = 0; j0 < nocc; j0 += kPairBatch) {
      const int nj = (int)std::min<int64_t>(kPairBatch, nocc - j0);
      const double2 *Uj = v.U + j0 * glen;
      hipLaunchKernelGGL(k_pair_rho, dim3(blocks_for(glen * nj)), dim3(256), 0, s, v.u, Uj, glen, nj, inv_omega,
                         v.rho);
      PW_HIP(hipGetLastError());
      if ((rc = launch_grid_fft(p->fft, v.rho, nj, glen, false, s)) != PW_OK) return rc;
      hipLaunchKernelGGL(k_kern_mul, dim3(blocks_for(glen * nj)), dim3(256), 0, s, v.rho, v.kern, glen, nj);
      PW_HIP(hipGetLastError());
      if ((rc = launch_grid_fft(p->fft, v.rho, nj, glen, true, s)) != PW_OK) return rc;
      hipLaunchKernelGGL(k_exx_acc, dim3(blocks_for(glen)), dim3(256), 0, s, v.acc, Uj, v.rho, v.w + j0, glen, nj);
      PW_HIP(hipGetLastError());
    }
    if ((rc = launch_grid_fft(p->fft, v.acc, 1, 0, false, s)) != PW_OK) return rc;
    hipLaunchKernelGGL(k_gather_full, dim3(blocks_for(npw)), dim3(256), 0, s, v.acc, p->d_gfull, npw, sign,
                       acc ? 1 : 0, static_cast<double2 *>(out) + i * ld_out);
    PW_HIP(hipGetLastError());
  }
  return PW_OK;
}

// split-K factor of a K-long product that fits the handle's partials
int fit_splits(const pw_problem *p, int64_t M, int64_t N, int64_t K) {
  int splits = choose_splits(M, N, K);
  while (splits > 1 && (size_t)splits * M * N * 16 > p->part_bytes) --splits;
  return splits;
}

// ACE build scratch: the direct operator's, then xi' = -V_x psi [nocc][ld],
// M' = -M, L, and the triangular inverse's two nocc x nocc matrices, a flag
size_t ace_bytes(const pw_problem *p, int64_t nocc) {
  Carve c(nullptr);
  carve_vx(p, nocc, c);
  const int64_t ld = (p->npw + 63) / 64 * 64;
  c.take<double2>((size_t)nocc * ld);
  c.take<double2>((size_t)4 * nocc * nocc);
  c.take<int>(1);
  return c.size();
}

}  // namespace

int ace_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi, int64_t ld_hpsi, int64_t nbands,
             hipStream_t s) {
  const int64_t no = p->ace_nocc, npw = p->npw;
  int rc = zgemm_cn(no, nbands, npw, p->ace_zeta, p->ace_ldz, psi, ld_psi, p->ace_proj, no,
                    fit_splits(p, no, nbands, npw), p->d_part, s);
  if (rc != PW_OK) return rc;
  return zgemm_nn(npw, nbands, no, -p->ace_alpha, p->ace_zeta, p->ace_ldz, p->ace_proj, no, 1.0, hpsi, ld_hpsi, s);
}

// Build ACE from nocc occupied states and attach alpha V_ace to the problem;
// e_xx (may be null) receives sum_i w_i <psi_i | V_x psi_i> = sum_i w_i M_ii.
int ace_build(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w, double alpha,
              void *zeta, int64_t ldz, void *proj, void *work, double *e_xx, hipStream_t s) {
  Carve c(work);
  carve_vx(p, nocc, c);
  const int64_t ld = (p->npw + 63) / 64 * 64, npw = p->npw;
  double2 *xi = c.take<double2>((size_t)nocc * ld);
  double2 *Mm = c.take<double2>((size_t)4 * nocc * nocc);
  double2 *L = Mm + nocc * nocc, *Xi = L + nocc * nocc, *Bi = Xi + nocc * nocc;
  int *flag = c.take<int>(1);
  int rc;
  // xi' = -V_x psi, M' = psi^H xi' = -M (positive definite)
  if ((rc = vx_impl(p, psi_occ, ld_occ, nocc, w, psi_occ, ld_occ, nocc, xi, ld, -1.0, work, s)) != PW_OK) goto fail;
  if ((rc = zgemm_cn(nocc, nocc, npw, psi_occ, ld_occ, xi, ld, Mm, nocc, fit_splits(p, nocc, nocc, npw), p->d_part,
                     s)) != PW_OK)
    goto fail;
  if ((rc = hermitize(Mm, nocc, 0, (int)nocc, s)) != PW_OK) goto fail;
  if (e_xx) {
    std::vector<double2> m((size_t)nocc * nocc);
    PW_HIP(hipMemcpyAsync(m.data(), Mm, m.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    PW_HIP(hipStreamSynchronize(s));
    double acc = 0.0;
    for (int64_t i = 0; i < nocc; ++i) acc -= w[i] * m[(size_t)i * nocc + i].x;
    *e_xx = acc;
  }
  if ((rc = cholesky(Mm, nocc, (int)nocc, L, nocc, 1e-12, flag, s)) != PW_OK) goto fail;
  {
    int h = 0;
    PW_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PW_HIP(hipStreamSynchronize(s));
    PW_CHECK_ARG(h == 0, PW_ERR_NUMERIC,
                 "pw_ace_set: <psi|V_x psi> is not negative definite (dependent or zero-weight occupied states)");
  }
  if ((rc = trinv_h(L, nocc, (int)nocc, Xi, nocc, Bi, nocc, s)) != PW_OK) goto fail;  // Bi = L^-H
  if ((rc = zgemm_nn(npw, nocc, nocc, 1.0, xi, ld, Bi, nocc, 0.0, zeta, ldz, s)) != PW_OK) goto fail;
  p->ace_zeta = static_cast<const double2 *>(zeta);
  p->ace_ldz = ldz;
  p->ace_nocc = nocc;
  p->ace_alpha = alpha;
  p->ace_proj = static_cast<double2 *>(proj);
  p->ace_owner = nullptr;
  p->exx_occ = nullptr;
  p->exx_nocc = 0;
  PW_HIP(hipStreamSynchronize(s));
  return PW_OK;
fail:
  set_error("pw_ace_set: launch failed");
  return rc;
}

int exx_direct_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi, int64_t ld_hpsi, int64_t nbands,
                    hipStream_t s) {
  return vx_impl(p, p->exx_occ, p->exx_ldo, p->exx_nocc, p->exx_w.data(), psi, ld_psi, nbands, hpsi, ld_hpsi,
                 p->exx_alpha, p->exx_work, s, true);
}

// e_xx = sum_i w_i <psi_i | V_x psi_i> from the diagonal of psi^H (V_x psi)
static int exx_energy(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                      void *work, double *e_xx, hipStream_t s) {
  Carve c(work);
  carve_vx(p, nocc, c);
  const int64_t ld = (p->npw + 63) / 64 * 64, npw = p->npw;
  double2 *xi = c.take<double2>((size_t)nocc * ld);
  double2 *Mm = c.take<double2>((size_t)4 * nocc * nocc);
  int rc = vx_impl(p, psi_occ, ld_occ, nocc, w, psi_occ, ld_occ, nocc, xi, ld, 1.0, work, s);
  if (rc != PW_OK) return rc;
  if ((rc = zgemm_cn(nocc, nocc, npw, psi_occ, ld_occ, xi, ld, Mm, nocc, fit_splits(p, nocc, nocc, npw),
                     p->d_part, s)) != PW_OK)
    return rc;
  std::vector<double2> d((size_t)nocc);
  PW_HIP(hipMemcpy2DAsync(d.data(), sizeof(double2), Mm, (size_t)(nocc + 1) * sizeof(double2), sizeof(double2),
                          nocc, hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int64_t i = 0; i < nocc; ++i) acc += w[i] * d[(size_t)i].x;
  *e_xx = acc;
  return PW_OK;
}

int exx_direct_build(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                     double alpha, void *occ, int64_t ldo, void *work, double *e_xx, hipStream_t s) {
  int rc = PW_OK;
  if (occ != psi_occ)
    PW_HIP(hipMemcpy2DAsync(occ, ldo * sizeof(double2), psi_occ, ld_occ * sizeof(double2), p->npw * sizeof(double2),
                            nocc, hipMemcpyDeviceToDevice, s));
  if (e_xx && (rc = exx_energy(p, occ, ldo, nocc, w, work, e_xx, s)) != PW_OK) {
    set_error("pw_vx_attach: launch failed");
    return rc;
  }
  p->ace_zeta = nullptr;
  p->ace_proj = nullptr;
  p->ace_nocc = 0;
  p->exx_occ = static_cast<const double2 *>(occ);
  p->exx_ldo = ldo;
  p->exx_nocc = nocc;
  p->exx_alpha = alpha;
  p->exx_w.assign(w, w + nocc);
  p->exx_work = work;
  p->ace_owner = nullptr;
  PW_HIP(hipStreamSynchronize(s));
  return PW_OK;
}

size_t ace_build_bytes(const pw_problem *p, int64_t nocc) { return ace_bytes(p, nocc); }

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_vx_workspace_size(const pw_problem *p, int64_t nocc, size_t *bytes) {
  PW_CHECK_ARG(p && bytes && nocc >= 1, PW_ERR_INVALID, "pw_vx_workspace_size: bad argument");
  *bytes = vx_bytes(p, nocc);
  return PW_OK;
}

static int exx_checks(const pw_problem *p, const char *who, const void *psi_occ, int64_t ld_occ, int64_t nocc,
                      const double *w) {
  PW_CHECK_ARG(p && psi_occ && w, PW_ERR_INVALID, std::string(who) + ": null argument");
  PW_CHECK_ARG(p->precision == PW_FP64, PW_ERR_INVALID, std::string(who) + ": the problem must be FP64");
  PW_CHECK_ARG(p->kpt[0] == 0.0 && p->kpt[1] == 0.0 && p->kpt[2] == 0.0, PW_ERR_INVALID,
               std::string(who) + ": exact exchange is implemented at the Gamma point only");
  PW_CHECK_ARG(!p->gen, PW_ERR_INVALID, std::string(who) + ": problems with overlap augmentation are not supported");
  PW_CHECK_ARG(nocc >= 1 && ld_occ >= p->npw, PW_ERR_INVALID, std::string(who) + ": need nocc >= 1 and ld >= npw");
  for (int64_t j = 0; j < nocc; ++j)
    PW_CHECK_ARG(std::isfinite(w[j]), PW_ERR_INVALID, std::string(who) + ": weights must be finite");
  return PW_OK;
}

pw_status pw_vx(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                const void *phi, int64_t ld_phi, int64_t nphi, void *out, int64_t ld_out, void *work,
                size_t work_bytes, void *stream) {
  int rc = exx_checks(p, "pw_vx", psi_occ, ld_occ, nocc, w);
  if (rc != PW_OK) return rc;
  PW_CHECK_ARG(nphi >= 0 && (nphi == 0 || (phi && out && ld_phi >= p->npw && ld_out >= p->npw)), PW_ERR_INVALID,
               "pw_vx: null phi / out or ld < npw");
  PW_CHECK_ARG(work && (reinterpret_cast<uintptr_t>(work) & 255) == 0 && work_bytes >= vx_bytes(p, nocc),
               PW_ERR_INVALID, "pw_vx: work must be 256-byte aligned and pw_vx_workspace_size bytes");
  if (nphi == 0) return PW_OK;
  rc = vx_impl(p, psi_occ, ld_occ, nocc, w, phi, ld_phi, nphi, out, ld_out, 1.0, work,
               static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_vx: launch failed");
  return rc;
}

pw_status pw_ace_workspace_size(const pw_problem *p, int64_t nocc, size_t *bytes) {
  PW_CHECK_ARG(p && bytes && nocc >= 1, PW_ERR_INVALID, "pw_ace_workspace_size: bad argument");
  *bytes = ace_bytes(p, nocc);
  return PW_OK;
}

pw_status pw_ace_set(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                     double alpha, void *zeta, int64_t ldz, void *proj, void *work, size_t work_bytes,
                     void *stream) {
  int rc = exx_checks(p, "pw_ace_set", psi_occ, ld_occ, nocc, w);
  if (rc != PW_OK) return rc;
  PW_CHECK_ARG(zeta && proj && ldz >= p->npw && std::isfinite(alpha), PW_ERR_INVALID,
               "pw_ace_set: null zeta / proj, ldz < npw or alpha not finite");
  PW_CHECK_ARG(nocc <= p->npw, PW_ERR_INVALID, "pw_ace_set: more occupied states than plane waves");
  PW_CHECK_ARG(work && (reinterpret_cast<uintptr_t>(work) & 255) == 0 && work_bytes >= ace_bytes(p, nocc),
               PW_ERR_INVALID, "pw_ace_set: work must be 256-byte aligned and pw_ace_workspace_size bytes");
  return ace_build(p, psi_occ, ld_occ, nocc, w, alpha, zeta, ldz, proj, work, nullptr,
                   static_cast<hipStream_t>(stream));
}

pw_status pw_vx_attach(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                       double alpha, void *work, size_t work_bytes, void *stream) {
  int rc = exx_checks(p, "pw_vx_attach", psi_occ, ld_occ, nocc, w);
  if (rc != PW_OK) return rc;
  PW_CHECK_ARG(std::isfinite(alpha), PW_ERR_INVALID, "pw_vx_attach: alpha not finite");
  PW_CHECK_ARG(work && (reinterpret_cast<uintptr_t>(work) & 255) == 0 && work_bytes >= vx_bytes(p, nocc),
               PW_ERR_INVALID, "pw_vx_attach: work must be 256-byte aligned and pw_vx_workspace_size bytes");
  return exx_direct_build(p, psi_occ, ld_occ, nocc, w, alpha, const_cast<void *>(psi_occ), ld_occ, work, nullptr,
                          static_cast<hipStream_t>(stream));
}

pw_status pw_ace_clear(pw_problem *p) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_ace_clear: null handle");
  p->ace_zeta = nullptr;
  p->ace_proj = nullptr;
  p->ace_nocc = 0;
  p->ace_alpha = 0.0;
  p->exx_occ = nullptr;
  p->exx_nocc = 0;
  p->exx_w.clear();
  p->exx_work = nullptr;
  p->ace_owner = nullptr;
  return PW_OK;
}

}  // extern "C"
