// Self-consistent field loop around the solver (CDNA4 / gfx950).
//
// The Kohn-Sham potential is V_ion + V_H[n] + V_x[n] (the paper writes V_LOC
// as the sum of the local, Hartree and exchange-correlation potentials in
// its relativistic PAW section; its exact-exchange section describes the
// outer loop that rebuilds the operator from the bands until it stops
// changing).  On the scalar, spin-unpolarised path, in Hartree units:
//   n(r)   = Omega^-1 sum_k w_k sum_n f_nk |u_nk(r)|^2
//   V_H(G) = 4 pi n(G) / |G|^2 (G != 0), V_H(0) = 0
//   V_x(r) = -(3 n(r) / pi)^{1/3}
//   f_nk   = 2 / (1 + exp((eps_nk - mu) / sigma)), sum_k w_k sum_n f_nk = N_el
//   n_in  <- n_in + alpha (n_out - n_in), or with the Kerker weight
//            alpha G^2 / (G^2 + q0^2) on each Fourier component of the residual
//
// Everything on the grid runs here: the band densities reuse the z passes
// of H*psi and a plane pass that stops after the inverse x transform, the
// Poisson solve runs on full-grid transforms, the reductions are fixed-order
// block trees.  The host only picks mu (bisection over a few thousand
// eigenvalues) and drives the Davidson solves.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace pw {

namespace {

constexpr int kRedBlocks = 512;   // fixed number of partial sums per reduction
constexpr int kRedThreads = 256;
constexpr int kRhoGroups = 16;    // partial density planes (bands per group = ceil(nb / 16))

__global__ void k_fill(double *a, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// fixed-order tree over the block; thread 0 writes the block's sum
__device__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}

// n[x][y][z] += scale * sum_{g < ng} part[g][z][x][y]: a 32 x 32 tile of
// (xy, z) per workgroup, read along xy, written along z through LDS
__global__ void k_rho_reduce(const double *__restrict__ part, int ng, int64_t npl, int n2, double scale,
                             double *__restrict__ n) {
  __shared__ double t[32][33];
  const int64_t xy0 = (int64_t)blockIdx.x * 32;
  const int z0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int z = z0 + j;
    const int64_t xy = xy0 + tx;
    double acc = 0.0;
    if (z < n2 && xy < npl)
      for (int g = 0; g < ng; ++g) acc += part[((int64_t)g * n2 + z) * npl + xy];
    t[j][tx] = acc;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t xy = xy0 + j;
    const int z = z0 + tx;
    if (z < n2 && xy < npl) n[xy * n2 + z] += scale * t[tx][j];
  }
}

// vplanes[z][x][y] = scale * v[x][y][z], the same tiling the other way
__global__ void k_to_planes(const double *__restrict__ v, int64_t npl, int n2, double scale,
                            double *__restrict__ vp) {
  __shared__ double t[32][33];
  const int64_t xy0 = (int64_t)blockIdx.x * 32;
  const int z0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int j = ty; j < 32; j += 8) {
    const int64_t xy = xy0 + j;
    const int z = z0 + tx;
    t[j][tx] = (z < n2 && xy < npl) ? v[xy * n2 + z] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int z = z0 + j;
    const int64_t xy = xy0 + tx;
    if (z < n2 && xy < npl) vp[(int64_t)z * npl + xy] = scale * t[tx][j];
  }
}

// partial sums of a (op 0), |a - b| (op 1)
__global__ __launch_bounds__(kRedThreads) void k_sum(const double *__restrict__ a, const double *__restrict__ b,
                                                     int64_t n, int op, double *__restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    acc += op == 0 ? a[i] : fabs(a[i] - b[i]);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_to_complex(const double *__restrict__ n, int64_t len, double2 *__restrict__ c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = double2{n[i], 0.0};
}

struct Recip {
  double b[9];  // rows b_i, a_i . b_j = 2 pi delta_ij
};

// c(G) <- 4 pi c(G) / |G|^2 (0 at G = 0) on the whole grid, signed indices
// h = j for j <= N/2 else j - N; partial sums of 4 pi |c(G)|^2 / |G|^2
__global__ __launch_bounds__(kRedThreads) void k_poisson(double2 *__restrict__ c, int n0, int n1, int n2, Recip B,
                                                         double *__restrict__ out) {
  __shared__ double sh[kRedThreads];
  const int64_t len = (int64_t)n0 * n1 * n2;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < len; i += (int64_t)gridDim.x * kRedThreads) {
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
    const double2 v = c[i];
    if (g2 > 0.0) {
      const double f = 4.0 * M_PI / g2;
      acc += f * (v.x * v.x + v.y * v.y);
      c[i] = double2{f * v.x, f * v.y};
    } else {
      c[i] = double2{0.0, 0.0};
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// v[r] = (vion[r] if given) + Re c[r] + xfrac v_x(n[r]); partial sums of
// xfrac n eps_x (out) and xfrac n v_x (out + kRedBlocks)
__global__ __launch_bounds__(kRedThreads) void k_hxc(const double2 *__restrict__ c, const double *__restrict__ n,
                                                     const double *__restrict__ vion, int64_t len, double xfrac,
                                                     double *__restrict__ v, double *__restrict__ out) {
  __shared__ double sh[kRedThreads];
  double ae = 0.0, av = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < len; i += (int64_t)gridDim.x * kRedThreads) {
    const double ni = n[i];
    const double cb = ni > 0.0 ? cbrt(3.0 * ni / M_PI) : 0.0;
    const double vx = -xfrac * cb;
    ae += ni * (-0.75 * xfrac * cb);
    av += ni * vx;
    v[i] = (vion ? vion[i] : 0.0) + c[i].x + vx;
  }
  const double se = block_sum(ae, sh);
  __syncthreads();
  const double sv = block_sum(av, sh);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = se;
    out[kRedBlocks + blockIdx.x] = sv;
  }
}

// c = (a - b) + 0i
__global__ void k_diff_complex(const double *__restrict__ a, const double *__restrict__ b, int64_t len,
                               double2 *__restrict__ c) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = double2{a[i] - b[i], 0.0};
}

// c(G) *= alpha G^2 / (G^2 + q0^2), alpha at G = 0 (signed indices as k_poisson)
__global__ void k_kerker(double2 *__restrict__ c, int n0, int n1, int n2, Recip B, double alpha, double q0sq) {
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
    const double w = g2 > 0.0 ? alpha * g2 / (g2 + q0sq) : alpha;
    c[i] = double2{w * c[i].x, w * c[i].y};
  }
}

// a += Re c
__global__ void k_add_real(double *__restrict__ a, const double2 *__restrict__ c, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    a[i] += c[i].x;
}

// n_in += alpha (n_out - n_in)
__global__ void k_mix(double *__restrict__ nin, const double *__restrict__ nout, int64_t len, double alpha) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    nin[i] += alpha * (nout[i] - nin[i]);
}

int64_t grid_len(const pw_problem *p) { return (int64_t)p->nr[0] * p->nr[1] * p->nr[2]; }

double cell_volume(const pw_problem *p) {
  const double *a = p->A;
  return std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                   a[2] * (a[3] * a[7] - a[4] * a[6]));
}

int fill(double *a, int64_t n, double v, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
  if (blocks <= 0) return PW_OK;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, a, n, v);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

// host sum, in order, of kRedBlocks partials (synchronises the stream)
int host_sum(const double *dpart, int count, double *out, hipStream_t s) {
  std::vector<double> h((size_t)count);
  PW_HIP(hipMemcpyAsync(h.data(), dpart, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (double x : h) acc += x;
  *out = acc;
  return PW_OK;
}

// sum of a (op 0) or of |a - b| (op 1) over n values, through nparts partials
int sum_grid(const double *a, const double *b, int64_t n, int op, double *dpart, int nparts, double *out,
             hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(nparts), dim3(kRedThreads), 0, s, a, b, n, op, dpart);
  PW_HIP(hipGetLastError());
  return host_sum(dpart, nparts, out, s);
}

size_t density_ws(const pw_problem *p) {
  Carve c(nullptr);
  c.take<double>((size_t)kRhoGroups * grid_len(p));
  c.take<double>((size_t)p->max_bands);
  return c.size();
}

size_t hxc_ws(const pw_problem *p) {
  Carve c(nullptr);
  c.take<double2>((size_t)grid_len(p));
  c.take<double>(2 * kRedBlocks);
  return c.size();
}

int density_impl(pw_problem *p, const void *psi, int64_t ld, int64_t nbands, const double *f, double *n,
                 void *work, hipStream_t s) {
  const int64_t len = grid_len(p), npl = (int64_t)p->nr[0] * p->nr[1];
  Carve c(work);
  double *part = c.take<double>((size_t)kRhoGroups * len);
  double *w = c.take<double>((size_t)p->max_bands);
  // the caller's host weights are read before the call returns
  PW_HIP(hipMemcpyAsync(w, f, sizeof(double) * nbands, hipMemcpyHostToDevice, s));
  PW_HIP(hipStreamSynchronize(s));
  int rc = fill(part, (int64_t)kRhoGroups * len, 0.0, s);
  if (rc != PW_OK) return rc;
  for (int64_t b0 = 0; b0 < nbands; b0 += p->band_chunk) {
    const int nb = (int)std::min<int64_t>(p->band_chunk, nbands - b0);
    const double2 *ps = static_cast<const double2 *>(psi) + b0 * ld;
    if ((rc = launch_zfft_inv(p->fft, PW_FP64, ps, ld, p->d_sticks, nb, s)) != PW_OK) return rc;
    const int group = (nb + kRhoGroups - 1) / kRhoGroups;
    if ((rc = launch_rho_plane(p->fft, p->d_sticks, nb, group, w + b0, part, s)) != PW_OK) return rc;
  }
  dim3 grid((unsigned)((npl + 31) / 32), (unsigned)((p->nr[2] + 31) / 32));
  hipLaunchKernelGGL(k_rho_reduce, grid, dim3(32, 8), 0, s, part, kRhoGroups, npl, p->nr[2],
                     1.0 / cell_volume(p), n);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

// v = (vion) + V_H[n] + xfrac V_x[n]; e[0..2] = E_H, xfrac E_x, xfrac int v_x n
int hxc_impl(pw_problem *p, const double *n, const double *vion, double xfrac, double *v, double *e, void *work,
             hipStream_t s) {
  const int64_t len = grid_len(p);
  Carve c(work);
  double2 *g = c.take<double2>((size_t)len);
  double *red = c.take<double>(2 * kRedBlocks);
  const int64_t blocks = std::min<int64_t>(4096, (len + 255) / 256);
  hipLaunchKernelGGL(k_to_complex, dim3((unsigned)blocks), dim3(256), 0, s, n, len, g);
  PW_HIP(hipGetLastError());
  int rc = launch_grid_fft(p->fft, g, 1, 0, false, s);
  if (rc != PW_OK) return rc;
  Recip B;
  std::copy(p->B, p->B + 9, B.b);
  hipLaunchKernelGGL(k_poisson, dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, p->nr[0], p->nr[1], p->nr[2], B, red);
  PW_HIP(hipGetLastError());
  double eh = 0.0;
  if ((rc = host_sum(red, kRedBlocks, &eh, s)) != PW_OK) return rc;
  if ((rc = launch_grid_fft(p->fft, g, 1, 0, true, s)) != PW_OK) return rc;
  hipLaunchKernelGGL(k_hxc, dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, n, vion, len, xfrac, v, red);
  PW_HIP(hipGetLastError());
  double ex = 0.0, evx = 0.0;
  if ((rc = host_sum(red, kRedBlocks, &ex, s)) != PW_OK) return rc;
  if ((rc = host_sum(red + kRedBlocks, kRedBlocks, &evx, s)) != PW_OK) return rc;
  const double omega = cell_volume(p);
  e[0] = 0.5 * omega * eh;
  e[1] = ex * omega / (double)len;
  e[2] = evx * omega / (double)len;
  return PW_OK;
}

// dpart: nparts doubles of device scratch for the mean of V
int set_vloc_impl(pw_problem *p, const double *v, double *dpart, int nparts, hipStream_t s) {
  const int64_t len = grid_len(p), npl = (int64_t)p->nr[0] * p->nr[1];
  dim3 grid((unsigned)((npl + 31) / 32), (unsigned)((p->nr[2] + 31) / 32));
  hipLaunchKernelGGL(k_to_planes, grid, dim3(32, 8), 0, s, v, npl, p->nr[2], 1.0 / (double)len,
                     static_cast<double *>(p->d_vplanes));
  PW_HIP(hipGetLastError());
  double sum = 0.0;
  const int rc = sum_grid(v, nullptr, len, 0, dpart, nparts, &sum, s);
  if (rc == PW_OK) p->vavg = sum / (double)len;
  return rc;
}

// occupations f = 2 / (1 + exp((eps - mu) / sigma)) with the weighted count
// nel, by bisection on mu; returns mu and the entropy S
double fermi(const std::vector<std::vector<double>> &eps, const std::vector<double> &kw, double nel,
             double sigma, std::vector<std::vector<double>> *f, double *entropy) {
  auto occ = [&](double mu, size_t k, size_t n) {
    const double x = std::min(700.0, std::max(-700.0, (eps[k][n] - mu) / sigma));
    return 2.0 / (1.0 + std::exp(x));
  };
  auto count = [&](double mu) {
    double c = 0.0;
    for (size_t k = 0; k < eps.size(); ++k) {
      double ck = 0.0;
      for (size_t n = 0; n < eps[k].size(); ++n) ck += occ(mu, k, n);
      c += kw[k] * ck;
    }
    return c;
  };
  double lo = 1e300, hi = -1e300;
  for (const auto &e : eps)
    for (double x : e) {
      lo = std::min(lo, x);
      hi = std::max(hi, x);
    }
  lo -= 50.0 * sigma;
  hi += 50.0 * sigma;
  while (hi - lo > 1e-14) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (count(mid) < nel)
      lo = mid;
    else
      hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  f->assign(eps.size(), {});
  double ent = 0.0;
  for (size_t k = 0; k < eps.size(); ++k) {
    (*f)[k].resize(eps[k].size());
    double ek = 0.0;
    for (size_t n = 0; n < eps[k].size(); ++n) {
      const double fn = occ(mu, k, n);
      (*f)[k][n] = fn;
      const double g = std::min(1.0, std::max(1e-300, fn / 2.0));
      const double h = std::min(1.0, std::max(1e-300, 1.0 - fn / 2.0));
      ek += g * std::log(g) + h * std::log(h);
    }
    ent -= kw[k] * 2.0 * ek;
  }
  *entropy = ent;
  return mu;
}

}  // namespace
}  // namespace pw

using namespace pw;

struct pw_scf {
  hipStream_t s = nullptr;
  std::vector<pw_problem *> probs;
  std::vector<pw_davidson *> davs;
  pw_batch_dav *batch = nullptr;
  std::vector<double> kw;
  const double *vion = nullptr;
  double nel = 0, sigma = 0, alpha = 0, q0 = 0;
  int64_t len = 0, ldx = 0;
  int nbmax = 0;
  double *n_in = nullptr, *n_out = nullptr, *v = nullptr, *red = nullptr;
  double2 *X = nullptr;
  void *dwork = nullptr, *hwork = nullptr;
  int step = 0;
  double e_h = 0, e_x = 0, e_vxn = 0;  // of the potential the current solves use
  // hybrid functional: exx_alpha of the Fock operator through ACE, the local
  // exchange scaled by xfrac = 1 - exx_alpha once the first ACE is attached
  double exx_alpha = 0, exx_tol = 0, xfrac = 1.0, e_xx = 0;
  bool exx_direct = false;  // V_x applied directly instead of through ACE
  int outer = 0;
  double2 *zeta = nullptr, *proj = nullptr;
  void *awork = nullptr;
  pw_problem *ace_prob = nullptr;  // the problem the loop's ACE is attached to
};

namespace pw {

void scf_forget_problem(pw_scf *s, const pw_problem *p) {
  if (s && s->ace_prob == p) s->ace_prob = nullptr;
}

namespace {

int check_desc(const pw_scf_desc *d, int64_t *ldx, int *nbmax) {
  PW_CHECK_ARG(d && d->nk >= 1 && d->probs && d->davs && d->kweights && d->vion, PW_ERR_INVALID,
               "pw_scf: null descriptor field or nk < 1");
  PW_CHECK_ARG(d->nel > 0 && d->sigma > 0 && d->alpha > 0 && d->alpha <= 1 && std::isfinite(d->nel) &&
                   std::isfinite(d->sigma) && d->kerker_q0 >= 0 && std::isfinite(d->kerker_q0),
               PW_ERR_INVALID, "pw_scf: need nel > 0, sigma > 0, 0 < alpha <= 1 and kerker_q0 >= 0");
  const pw_problem *p0 = d->probs[0];
  PW_CHECK_ARG(p0, PW_ERR_INVALID, "pw_scf: null problem");
  int64_t ld = 0;
  int nb = 0;
  double nsum = 0;
  for (int k = 0; k < d->nk; ++k) {
    const pw_problem *p = d->probs[k];
    const pw_davidson *dv = d->davs[k];
    PW_CHECK_ARG(p && dv, PW_ERR_INVALID, "pw_scf: null problem or Davidson state");
    PW_CHECK_ARG(p->precision == PW_FP64, PW_ERR_INVALID, "pw_scf: the problems must be FP64");
    PW_CHECK_ARG(!p->gen, PW_ERR_INVALID, "pw_scf: problems with overlap augmentation are not supported");
    PW_CHECK_ARG(p->nr[0] == p0->nr[0] && p->nr[1] == p0->nr[1] && p->nr[2] == p0->nr[2], PW_ERR_INVALID,
                 "pw_scf: every problem must be on the same grid");
    for (int i = 0; i < 9; ++i)
      PW_CHECK_ARG(p->A[i] == p0->A[i], PW_ERR_INVALID, "pw_scf: every problem must be in the same cell");
    PW_CHECK_ARG(dav_problem(dv) == p, PW_ERR_INVALID, "pw_scf: davs[k] must solve probs[k]");
    PW_CHECK_ARG(dav_inited(dv), PW_ERR_INVALID, "pw_scf: every Davidson state must be initialised");
    PW_CHECK_ARG(d->kweights[k] > 0 && std::isfinite(d->kweights[k]), PW_ERR_INVALID,
                 "pw_scf: k-point weights must be positive");
    ld = std::max<int64_t>(ld, (p->npw + 63) / 64 * 64);
    nb = std::max(nb, dav_nbands(dv));
    nsum += 2.0 * dav_nbands(dv) * d->kweights[k];
  }
  PW_CHECK_ARG(d->nel < nsum, PW_ERR_INVALID, "pw_scf: more electrons than the bands can hold");
  PW_CHECK_ARG(d->exx_alpha >= 0 && d->exx_alpha <= 1 && std::isfinite(d->exx_alpha), PW_ERR_INVALID,
               "pw_scf: need 0 <= exx_alpha <= 1");
  if (d->exx_alpha > 0) {
    PW_CHECK_ARG(d->nk == 1 && p0->kpt[0] == 0.0 && p0->kpt[1] == 0.0 && p0->kpt[2] == 0.0, PW_ERR_INVALID,
                 "pw_scf: exact exchange is implemented at the Gamma point only (one k-point, k = 0)");
    PW_CHECK_ARG(d->exx_tol > 0 && std::isfinite(d->exx_tol), PW_ERR_INVALID, "pw_scf: need exx_tol > 0");
  }
  PW_CHECK_ARG(d->exx_direct == 0 || (d->exx_direct == 1 && d->exx_alpha > 0), PW_ERR_INVALID,
               "pw_scf: exx_direct is 0 or 1, and 1 only with exx_alpha > 0");
  *ldx = ld;
  *nbmax = nb;
  return PW_OK;
}

size_t scf_carve(const pw_scf_desc *d, int64_t ldx, int nbmax, Carve &c, pw_scf *s) {
  const pw_problem *p0 = d->probs[0];
  const int64_t len = grid_len(p0);
  size_t dws = 0, hws = hxc_ws(p0);
  for (int k = 0; k < d->nk; ++k) dws = std::max(dws, density_ws(d->probs[k]));
  double *a = c.take<double>((size_t)len);
  double *b = c.take<double>((size_t)len);
  double *v = c.take<double>((size_t)len);
  double *r = c.take<double>(2 * kRedBlocks);
  double2 *x = c.take<double2>((size_t)nbmax * ldx);
  char *dw = c.take<char>(dws);
  char *hw = c.take<char>(hws);
  double2 *zt = nullptr, *pj = nullptr;
  char *aw = nullptr;
  if (d->exx_alpha > 0) {
    zt = c.take<double2>((size_t)nbmax * ldx);
    pj = c.take<double2>((size_t)nbmax * p0->max_bands);
    aw = c.take<char>(ace_build_bytes(p0, nbmax));
  }
  if (s) {
    s->zeta = zt;
    s->proj = pj;
    s->awork = aw;
    s->n_in = a;
    s->n_out = b;
    s->v = v;
    s->red = r;
    s->X = x;
    s->dwork = dw;
    s->hwork = hw;
  }
  return c.size();
}

}  // namespace
}  // namespace pw

extern "C" {

pw_status pw_density_workspace_size(const pw_problem *p, size_t *bytes) {
  PW_CHECK_ARG(p && bytes, PW_ERR_INVALID, "pw_density_workspace_size: null argument");
  *bytes = density_ws(p);
  return PW_OK;
}

pw_status pw_density(pw_problem *p, const void *psi, int64_t ld, int64_t nbands, const double *f, double *n,
                     void *work, size_t work_bytes, void *stream) {
  PW_CHECK_ARG(p && n && f, PW_ERR_INVALID, "pw_density: null argument");
  PW_CHECK_ARG(p->precision == PW_FP64, PW_ERR_INVALID, "pw_density: the problem must be FP64");
  PW_CHECK_ARG(nbands >= 0 && nbands <= p->max_bands, PW_ERR_INVALID, "pw_density: nbands must be in 0 .. max_bands");
  if (nbands == 0) return PW_OK;
  PW_CHECK_ARG(psi && ld >= p->npw, PW_ERR_INVALID, "pw_density: null psi or ld < npw");
  PW_CHECK_ARG(work && (reinterpret_cast<uintptr_t>(work) & 255) == 0 && work_bytes >= density_ws(p),
               PW_ERR_INVALID, "pw_density: work must be 256-byte aligned and pw_density_workspace_size bytes");
  for (int64_t b = 0; b < nbands; ++b)
    PW_CHECK_ARG(std::isfinite(f[b]), PW_ERR_INVALID, "pw_density: weights must be finite");
  const int rc = density_impl(p, psi, ld, nbands, f, n, work, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_density: launch failed");
  return rc;
}

pw_status pw_hxc_workspace_size(const pw_problem *p, size_t *bytes) {
  PW_CHECK_ARG(p && bytes, PW_ERR_INVALID, "pw_hxc_workspace_size: null argument");
  *bytes = hxc_ws(p);
  return PW_OK;
}

pw_status pw_hxc(pw_problem *p, const double *n, const double *vion, double *v, double *energies, void *work,
                 size_t work_bytes, void *stream) {
  PW_CHECK_ARG(p && n && v && energies, PW_ERR_INVALID, "pw_hxc: null argument");
  PW_CHECK_ARG(p->precision == PW_FP64, PW_ERR_INVALID, "pw_hxc: the problem must be FP64");
  PW_CHECK_ARG(work && (reinterpret_cast<uintptr_t>(work) & 255) == 0 && work_bytes >= hxc_ws(p), PW_ERR_INVALID,
               "pw_hxc: work must be 256-byte aligned and pw_hxc_workspace_size bytes");
  const int rc = hxc_impl(p, n, vion, 1.0, v, energies, work, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_hxc: launch failed");
  return rc;
}

pw_status pw_problem_set_vloc(pw_problem *p, const double *v, void *stream) {
  PW_CHECK_ARG(p && v, PW_ERR_INVALID, "pw_problem_set_vloc: null argument");
  PW_CHECK_ARG(p->precision == PW_FP64, PW_ERR_INVALID, "pw_problem_set_vloc: the problem must be FP64");
  // the mean of V goes through the handle's per-band scratch (max_bands doubles)
  const int nparts = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, p->max_bands));
  const int rc = set_vloc_impl(p, v, p->d_tn, nparts, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_problem_set_vloc: launch failed");
  return rc;
}

pw_status pw_scf_workspace_size(const pw_scf_desc *d, size_t *bytes) {
  PW_CHECK_ARG(bytes, PW_ERR_INVALID, "pw_scf_workspace_size: null argument");
  int64_t ldx = 0;
  int nb = 0;
  const int rc = check_desc(d, &ldx, &nb);
  if (rc != PW_OK) return rc;
  Carve c(nullptr);
  *bytes = scf_carve(d, ldx, nb, c, nullptr);
  return PW_OK;
}

pw_status pw_scf_create(const pw_scf_desc *d, void *workspace, size_t ws_bytes, void *stream, pw_scf **out) {
  PW_CHECK_ARG(out, PW_ERR_INVALID, "pw_scf_create: null output");
  *out = nullptr;
  int64_t ldx = 0;
  int nb = 0;
  int rc = check_desc(d, &ldx, &nb);
  if (rc != PW_OK) return rc;
  Carve cnt(nullptr);
  const size_t need = scf_carve(d, ldx, nb, cnt, nullptr);
  PW_CHECK_ARG(workspace && (reinterpret_cast<uintptr_t>(workspace) & 255) == 0 && ws_bytes >= need,
               PW_ERR_INVALID, "pw_scf_create: workspace must be 256-byte aligned and pw_scf_workspace_size bytes");
  pw_scf *s = new pw_scf;
  s->s = static_cast<hipStream_t>(stream);
  s->probs.assign(d->probs, d->probs + d->nk);
  s->davs.assign(d->davs, d->davs + d->nk);
  s->batch = d->batch;
  s->kw.assign(d->kweights, d->kweights + d->nk);
  s->vion = d->vion;
  s->nel = d->nel;
  s->sigma = d->sigma;
  s->alpha = d->alpha;
  s->q0 = d->kerker_q0;
  s->exx_alpha = d->exx_alpha;
  s->exx_tol = d->exx_tol;
  s->exx_direct = d->exx_direct != 0;
  s->len = grid_len(d->probs[0]);
  s->ldx = ldx;
  s->nbmax = nb;
  Carve c(workspace);
  scf_carve(d, ldx, nb, c, s);
  // step 0 solves with V_ion alone (and, in a hybrid loop, without a Fock term)
  if (s->exx_alpha > 0) pw_ace_clear(s->probs[0]);
  rc = fill(s->n_in, s->len, 0.0, s->s);
  for (int k = 0; k < d->nk && rc == PW_OK; ++k) {
    rc = set_vloc_impl(s->probs[k], s->vion, s->red, kRedBlocks, s->s);
    if (rc == PW_OK) rc = pw_davidson_set_problem(s->davs[k], s->probs[k], stream);
  }
  // the solves may run on other streams (a batch): the refreshed states must be complete
  if (rc == PW_OK && hipStreamSynchronize(s->s) != hipSuccess) rc = PW_ERR_HIP;
  if (rc != PW_OK) {
    delete s;
    set_error("pw_scf_create: set-up failed");
    return rc;
  }
  *out = s;
  return PW_OK;
}

pw_status pw_scf_destroy(pw_scf *s) {
  // the Fock term the loop attached lives in the loop's workspace; a problem
  // destroyed before the loop has already told it (scf_forget_problem)
  if (s && s->ace_prob && s->ace_prob->ace_owner == s) pw_ace_clear(s->ace_prob);
  delete s;
  return PW_OK;
}

pw_status pw_scf_step(pw_scf *s, double dav_tol, int32_t dav_max_iter, double tol, double *out,
                      int32_t *converged) {
  PW_CHECK_ARG(s && out && dav_tol > 0 && dav_max_iter >= 1 && tol > 0, PW_ERR_INVALID,
               "pw_scf_step: bad argument");
  hipStream_t st = s->s;
  const int nk = (int)s->probs.size();
  int rc;
  // 1. the bands of every k-point in the current potential
  for (int k = 0; k < nk; ++k)
    if ((rc = pw_davidson_set_tol(s->davs[k], dav_tol)) != PW_OK) return rc;
  if (s->batch) {
    rc = pw_batch_davidson_run(s->batch, nullptr, nullptr, dav_max_iter, PW_PRECOND_TPA, nullptr, nullptr);
    if (rc < 0) return rc;
  } else {
    for (int k = 0; k < nk; ++k) {
      rc = pw_davidson_run(s->davs[k], dav_max_iter, PW_PRECOND_TPA, nullptr, st, nullptr);
      if (rc < 0) return rc;
    }
  }
  // 2. occupations
  std::vector<std::vector<double>> eps((size_t)nk), f;
  for (int k = 0; k < nk; ++k) {
    eps[k].resize((size_t)dav_nbands(s->davs[k]));
    if ((rc = pw_davidson_query(s->davs[k], eps[k].data(), nullptr, nullptr, nullptr, st)) != PW_OK) return rc;
  }
  double ent = 0.0;
  const double mu = fermi(eps, s->kw, s->nel, s->sigma, &f, &ent);
  // 3. output density
  if ((rc = fill(s->n_out, s->len, 0.0, st)) != PW_OK) return rc;
  for (int k = 0; k < nk; ++k) {
    pw_problem *p = s->probs[k];
    const int nb = dav_nbands(s->davs[k]);
    std::vector<double> w((size_t)nb);
    for (int n = 0; n < nb; ++n) w[n] = s->kw[k] * f[k][n];
    if ((rc = pw_davidson_vectors(s->davs[k], s->X, s->ldx, st)) != PW_OK) return rc;
    if ((rc = density_impl(p, s->X, s->ldx, nb, w.data(), s->n_out, s->dwork, st)) != PW_OK) return rc;
  }
  // 4. distance from the input density, energies of this step
  const double dv = cell_volume(s->probs[0]) / (double)s->len;
  double drho = -1.0;
  if (s->step > 0) {
    double sum = 0.0;
    if ((rc = sum_grid(s->n_out, s->n_in, s->len, 1, s->red, kRedBlocks, &sum, st)) != PW_OK) return rc;
    drho = sum * dv / s->nel;
  }
  double eband = 0.0;
  for (int k = 0; k < nk; ++k) {
    double ek = 0.0;
    for (size_t n = 0; n < eps[k].size(); ++n) ek += f[k][n] * eps[k][n];
    eband += s->kw[k] * ek;
  }
  const double exx_att = s->outer > 0 ? s->e_xx : 0.0;
  const double etot = eband - s->exx_alpha * exx_att - s->e_h + s->e_x - s->e_vxn;
  out[0] = drho;
  out[1] = mu;
  out[2] = eband;
  out[3] = s->e_h;
  out[4] = s->e_x;
  out[5] = s->e_vxn;
  out[6] = etot;
  out[7] = etot - s->sigma * ent;
  out[8] = exx_att;
  out[9] = (double)s->outer;
  bool conv = s->step > 0 && drho < tol;
  if (conv && s->exx_alpha > 0) {
    // outer step of the double loop: V_ace from the occupied orbitals of the
    // converged inner loop (weights f/2 above 1e-8, a prefix of the ascending bands)
    pw_problem *p0 = s->probs[0];
    const int nb = dav_nbands(s->davs[0]);
    std::vector<double> w;
    for (int n = 0; n < nb && f[0][n] / 2.0 > 1e-8; ++n) w.push_back(f[0][n] / 2.0);
    double e_new = 0.0;
    if (s->exx_direct)
      rc = exx_direct_build(p0, s->X, s->ldx, (int64_t)w.size(), w.data(), s->exx_alpha, s->zeta, s->ldx,
                            s->awork, &e_new, st);
    else
      rc = ace_build(p0, s->X, s->ldx, (int64_t)w.size(), w.data(), s->exx_alpha, s->zeta, s->ldx, s->proj,
                     s->awork, &e_new, st);
    if (rc != PW_OK) return rc;
    p0->ace_owner = s;
    s->ace_prob = p0;
    if (s->outer >= 1 && std::fabs(e_new - s->e_xx) < s->exx_tol) {
      // converged: the operator rebuilt from these orbitals is the one they solve
      if (converged) *converged = 1;
      return PW_OK;
    }
    s->e_xx = e_new;
    s->xfrac = 1.0 - s->exx_alpha;
    ++s->outer;
    conv = false;
    // the inner loop continues from the same input density with the new operator
    double e[3];
    if ((rc = hxc_impl(p0, s->n_in, s->vion, s->xfrac, s->v, e, s->hwork, st)) != PW_OK) return rc;
    s->e_h = e[0];
    s->e_x = e[1];
    s->e_vxn = e[2];
    if ((rc = set_vloc_impl(p0, s->v, s->red, kRedBlocks, st)) != PW_OK) return rc;
    if ((rc = pw_davidson_set_problem(s->davs[0], p0, st)) != PW_OK) return rc;
    ++s->step;
    if (converged) *converged = 0;
    PW_HIP(hipStreamSynchronize(st));
    return PW_OK;
  }
  if (converged) *converged = conv ? 1 : 0;
  if (conv) return PW_OK;
  // 5. the next input density and its potential on every problem
  if (s->step == 0) {
    PW_HIP(hipMemcpyAsync(s->n_in, s->n_out, sizeof(double) * s->len, hipMemcpyDeviceToDevice, st));
  } else if (s->q0 > 0.0) {
    // Kerker: the residual through the full-grid transforms (the Hartree scratch)
    pw_problem *p0 = s->probs[0];
    double2 *g = static_cast<double2 *>(s->hwork);
    const int64_t blocks = std::min<int64_t>(4096, (s->len + 255) / 256);
    hipLaunchKernelGGL(k_diff_complex, dim3((unsigned)blocks), dim3(256), 0, st, s->n_out, s->n_in, s->len, g);
    PW_HIP(hipGetLastError());
    if ((rc = launch_grid_fft(p0->fft, g, 1, 0, false, st)) != PW_OK) return rc;
    Recip B;
    std::copy(p0->B, p0->B + 9, B.b);
    hipLaunchKernelGGL(k_kerker, dim3((unsigned)blocks), dim3(256), 0, st, g, p0->nr[0], p0->nr[1], p0->nr[2], B,
                       s->alpha, s->q0 * s->q0);
    PW_HIP(hipGetLastError());
    if ((rc = launch_grid_fft(p0->fft, g, 1, 0, true, st)) != PW_OK) return rc;
    hipLaunchKernelGGL(k_add_real, dim3((unsigned)blocks), dim3(256), 0, st, s->n_in, g, s->len);
    PW_HIP(hipGetLastError());
  } else {
    const int64_t blocks = std::min<int64_t>(4096, (s->len + 255) / 256);
    hipLaunchKernelGGL(k_mix, dim3((unsigned)blocks), dim3(256), 0, st, s->n_in, s->n_out, s->len, s->alpha);
    PW_HIP(hipGetLastError());
  }
  double e[3];
  if ((rc = hxc_impl(s->probs[0], s->n_in, s->vion, s->xfrac, s->v, e, s->hwork, st)) != PW_OK) return rc;
  s->e_h = e[0];
  s->e_x = e[1];
  s->e_vxn = e[2];
  for (int k = 0; k < nk; ++k) {
    if ((rc = set_vloc_impl(s->probs[k], s->v, s->red, kRedBlocks, st)) != PW_OK) return rc;
    if ((rc = pw_davidson_set_problem(s->davs[k], s->probs[k], st)) != PW_OK) return rc;
  }
  ++s->step;
  // the next solves may run on other streams (a batch)
  PW_HIP(hipStreamSynchronize(st));
  return PW_OK;
}

pw_status pw_scf_density(pw_scf *s, double *n_in, double *n_out, void *stream) {
  PW_CHECK_ARG(s, PW_ERR_INVALID, "pw_scf_density: null state");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (n_in) PW_HIP(hipMemcpyAsync(n_in, s->n_in, sizeof(double) * s->len, hipMemcpyDeviceToDevice, st));
  if (n_out) PW_HIP(hipMemcpyAsync(n_out, s->n_out, sizeof(double) * s->len, hipMemcpyDeviceToDevice, st));
  return PW_OK;
}

pw_status pw_scf_potential(pw_scf *s, double *v, void *stream) {
  PW_CHECK_ARG(s && v, PW_ERR_INVALID, "pw_scf_potential: null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double *src = s->step == 0 ? s->vion : s->v;
  PW_HIP(hipMemcpyAsync(v, src, sizeof(double) * s->len, hipMemcpyDeviceToDevice, st));
  return PW_OK;
}

}  // extern "C"
