// Lanczos recursion on H and the continued fraction of its resolvent.
//
// The paper's section on dynamic perturbations computes a diagonal element
// of a resolvent, g_v(w) = <v|(w - L)^{-1} v> (eq. resolvent), from the
// chain q_0 = 0, q_1 = v, alpha_n = <q_n|L q_n>, beta_{n+1} q_{n+1} =
// (L - alpha_n) q_n - beta_n q_{n-1} with |q_{n+1}| = 1 (eqs. rec1 - rec4),
// as the continued fraction of the tridiagonal T_M (eqs. tridiagonal,
// continuedfraction); only three vectors per chain are ever kept.  Here
// L = H, applied by pw_hpsi, and many chains (start vectors) advance in
// lockstep: one step is one batched H*psi over the chains plus one kernel
// that, per chain, forms alpha, the three-term update, beta and the
// normalised next vector.  alpha and beta stay on the device; a run of
// steps has no host synchronisation.
//
// The chain starts from q_1 = v / |v| (beta_1 = |v| is kept, g_v = |v|^2
// times the fraction).  It ends at beta_{n+1} <= 1e-12 |H q_n| (breakdown:
// an invariant subspace, the remaining residual being rounding error):
// beta_{n+1} and q_{n+1} are then zero, and so is every later alpha and
// beta, which ends the fraction there.
#include <cmath>

#include "common.h"

namespace pw {

constexpr int kLzThreads = 256;
constexpr double kLzBreakdown = 1e-12;

// Sum over the workgroup of one double per thread (fixed-order tree).
__device__ __forceinline__ double wg_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kLzThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// Per chain c (one workgroup): beta[c][0] = |v_c|, q_c = v_c / |v_c| (zero
// for a zero start), q_prev = 0.
__global__ __launch_bounds__(kLzThreads) void k_lz_start(const double2 *__restrict__ v, int64_t ldv,
                                                         double2 *__restrict__ q, double2 *__restrict__ qp,
                                                         int64_t ld, int64_t npw, double *__restrict__ beta,
                                                         int64_t ldb) {
  __shared__ double red[kLzThreads];
  const int64_t c = blockIdx.x;
  const double2 *vc = v + c * ldv;
  double s = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kLzThreads) s += vc[g].x * vc[g].x + vc[g].y * vc[g].y;
  const double nrm = sqrt(wg_sum(s, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kLzThreads) {
    q[c * ld + g] = double2{vc[g].x * inv, vc[g].y * inv};
    qp[c * ld + g] = double2{0.0, 0.0};
  }
  if (threadIdx.x == 0) beta[c * ldb] = nrm;
}

// Step n of chain c (one workgroup), hq = H q_n given:
//   alpha_n = Re <q_n|H q_n>;  w = H q_n - alpha_n q_n - beta_n q_{n-1}
//   (written over q_{n-1});  beta_{n+1} = |w| (zero at breakdown);
//   q_{n+1} = w / beta_{n+1} (zero at breakdown).
// alpha[c][n] and beta[c][n + 1] are stored; beta[c][n] holds beta_n (for
// n = 0 the start norm, multiplying q_0 = 0).
__global__ __launch_bounds__(kLzThreads) void k_lz_step(const double2 *__restrict__ hq,
                                                        const double2 *__restrict__ q,
                                                        double2 *__restrict__ qp, int64_t ld, int64_t npw,
                                                        double *__restrict__ alpha, int64_t lda,
                                                        double *__restrict__ beta, int64_t ldb, int n) {
  __shared__ double red[kLzThreads];
  const int64_t c = blockIdx.x;
  const double2 *h = hq + c * ld;
  const double2 *x = q + c * ld;
  double2 *y = qp + c * ld;
  double sa = 0.0, sh = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kLzThreads) {
    sa += x[g].x * h[g].x + x[g].y * h[g].y;
    sh += h[g].x * h[g].x + h[g].y * h[g].y;
  }
  const double a = wg_sum(sa, red);
  const double hnorm = sqrt(wg_sum(sh, red));
  const double bp = beta[c * ldb + n];
  double sw = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kLzThreads) {
    const double2 w = double2{h[g].x - a * x[g].x - bp * y[g].x, h[g].y - a * x[g].y - bp * y[g].y};
    y[g] = w;
    sw += w.x * w.x + w.y * w.y;
  }
  double bn = sqrt(wg_sum(sw, red));
  if (bn <= kLzBreakdown * hnorm) bn = 0.0;
  const double inv = bn > 0.0 ? 1.0 / bn : 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += kLzThreads) y[g] = double2{y[g].x * inv, y[g].y * inv};
  if (threadIdx.x == 0) {
    alpha[c * lda + n] = a;
    beta[c * ldb + n + 1] = bn;
  }
}

// g[c][k] = beta_1^2 / (z_k - alpha_1 - beta_2^2 / (z_k - alpha_2 - ... / (z_k - alpha_M))),
// evaluated from the bottom up, one thread per (chain, z).
__global__ void k_lz_cfrac(const double *__restrict__ alpha, int64_t lda, const double *__restrict__ beta,
                           int64_t ldb, int m, const double2 *__restrict__ z, int nz, int64_t nch,
                           double2 *__restrict__ g) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nch * nz) return;
  const int64_t c = e / nz;
  const int k = (int)(e - c * nz);
  const double *a = alpha + c * lda;
  const double *b = beta + c * ldb;
  const double zr = z[k].x, zi = z[k].y;
  // r = 1 / (z - alpha_M)
  double dr = zr - a[m - 1], di = zi;
  double den = dr * dr + di * di;
  double rr = dr / den, ri = -di / den;
  for (int n = m - 2; n >= 0; --n) {
    const double b2 = b[n + 1] * b[n + 1];
    dr = zr - a[n] - b2 * rr;
    di = zi - b2 * ri;
    den = dr * dr + di * di;
    rr = dr / den;
    ri = -di / den;
  }
  const double s = b[0] * b[0];
  g[c * nz + k] = double2{s * rr, s * ri};
}

}  // namespace pw

using namespace pw;

struct pw_lanczos {
  pw_problem *p = nullptr;
  int64_t nch = 0, ld = 0;
  int max_steps = 0, n = 0;
  bool started = false;
  double2 *qp = nullptr, *q = nullptr, *hq = nullptr;  // [nch][ld] each
  double *alpha = nullptr;                              // [nch][max_steps]
  double *beta = nullptr;                               // [nch][max_steps + 1]
};

namespace {

void carve_lz(pw_lanczos *l, Carve &c) {
  const size_t vec = (size_t)l->nch * l->ld;
  l->qp = c.take<double2>(vec);
  l->q = c.take<double2>(vec);
  l->hq = c.take<double2>(vec);
  l->alpha = c.take<double>((size_t)l->nch * l->max_steps);
  l->beta = c.take<double>((size_t)l->nch * (l->max_steps + 1));
}

int lz_shape(pw_problem *p, int64_t nchains, int32_t max_steps, const char *who) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, std::string(who) + ": null problem");
  PW_CHECK_ARG(nchains >= 1 && nchains <= p->max_bands, PW_ERR_INVALID,
               std::string(who) + ": nchains must be in 1 .. the problem's max_bands");
  PW_CHECK_ARG(max_steps >= 1 && max_steps <= (1 << 20), PW_ERR_INVALID,
               std::string(who) + ": max_steps must be in 1 .. 2^20");
  return PW_OK;
}

}  // namespace

extern "C" {

pw_status pw_lanczos_workspace_size(pw_problem *p, int64_t nchains, int32_t max_steps, size_t *bytes) {
  PW_CHECK_ARG(bytes, PW_ERR_INVALID, "pw_lanczos_workspace_size: null bytes");
  *bytes = 0;
  const int rc = lz_shape(p, nchains, max_steps, "pw_lanczos_workspace_size");
  if (rc != PW_OK) return rc;
  pw_lanczos l;
  l.nch = nchains;
  l.ld = (p->npw + 63) / 64 * 64;
  l.max_steps = max_steps;
  Carve c(nullptr);
  carve_lz(&l, c);
  *bytes = c.size();
  return PW_OK;
}

pw_status pw_lanczos_create(pw_problem *p, int64_t nchains, int32_t max_steps, void *workspace, size_t ws_bytes,
                            pw_lanczos **out) {
  PW_CHECK_ARG(out, PW_ERR_INVALID, "pw_lanczos_create: null out");
  *out = nullptr;
  const int rc = lz_shape(p, nchains, max_steps, "pw_lanczos_create");
  if (rc != PW_OK) return rc;
  pw_lanczos *l = new pw_lanczos();
  l->p = p;
  l->nch = nchains;
  l->ld = (p->npw + 63) / 64 * 64;
  l->max_steps = max_steps;
  Carve count(nullptr);
  carve_lz(l, count);
  if (!workspace || ws_bytes < count.size() || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
    delete l;
    set_error("pw_lanczos_create: workspace must be 256-byte aligned device memory of at least "
              "pw_lanczos_workspace_size() = " + std::to_string(count.size()) + " bytes");
    return PW_ERR_INVALID;
  }
  Carve c(workspace);
  carve_lz(l, c);
  *out = l;
  return PW_OK;
}

pw_status pw_lanczos_destroy(pw_lanczos *l) {
  delete l;
  return PW_OK;
}

pw_status pw_lanczos_start(pw_lanczos *l, const void *v, int64_t ld, void *stream) {
  PW_CHECK_ARG(l && v && ld >= l->p->npw, PW_ERR_INVALID, "pw_lanczos_start: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // alpha and beta cleared: a chain read before its steps exist reads zeros
  PW_HIP(hipMemsetAsync(l->alpha, 0, (size_t)l->nch * l->max_steps * sizeof(double), s));
  PW_HIP(hipMemsetAsync(l->beta, 0, (size_t)l->nch * (l->max_steps + 1) * sizeof(double), s));
  hipLaunchKernelGGL(k_lz_start, dim3((unsigned)l->nch), dim3(kLzThreads), 0, s, static_cast<const double2 *>(v),
                     ld, l->q, l->qp, l->ld, l->p->npw, l->beta, (int64_t)(l->max_steps + 1));
  PW_HIP(hipGetLastError());
  l->n = 0;
  l->started = true;
  return PW_OK;
}

pw_status pw_lanczos_run(pw_lanczos *l, int32_t nsteps, void *stream) {
  PW_CHECK_ARG(l && l->started, PW_ERR_INVALID, "pw_lanczos_run: start the chains first");
  PW_CHECK_ARG(nsteps >= 0 && nsteps <= l->max_steps - l->n, PW_ERR_INVALID,
               "pw_lanczos_run: nsteps exceeds the steps left (max_steps - steps done)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int t = 0; t < nsteps; ++t) {
    const int rc = pw_hpsi(l->p, l->q, l->ld, l->hq, l->ld, l->nch, PW_TERM_ALL, stream);
    if (rc != PW_OK) return rc;
    {
      ProfScope ps(&l->p->prof, PW_STAGE_VEC, s);
      hipLaunchKernelGGL(k_lz_step, dim3((unsigned)l->nch), dim3(kLzThreads), 0, s, l->hq, l->q, l->qp, l->ld,
                         l->p->npw, l->alpha, (int64_t)l->max_steps, l->beta, (int64_t)(l->max_steps + 1), l->n);
    }
    PW_HIP(hipGetLastError());
    std::swap(l->q, l->qp);  // q_{n+1} was written over q_{n-1}
    ++l->n;
  }
  return PW_OK;
}

pw_status pw_lanczos_coefficients(pw_lanczos *l, double *alpha, double *beta, int32_t *nsteps, void *stream) {
  PW_CHECK_ARG(l, PW_ERR_INVALID, "pw_lanczos_coefficients: null chain set");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (alpha)
    PW_HIP(hipMemcpyAsync(alpha, l->alpha, (size_t)l->nch * l->max_steps * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  if (beta)
    PW_HIP(hipMemcpyAsync(beta, l->beta, (size_t)l->nch * (l->max_steps + 1) * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  if (nsteps) *nsteps = l->n;
  return PW_OK;
}

pw_status pw_lanczos_resolvent(pw_lanczos *l, const void *z, int32_t nz, void *g, void *stream) {
  PW_CHECK_ARG(l && l->started && z && g && nz >= 1, PW_ERR_INVALID, "pw_lanczos_resolvent: bad argument");
  PW_CHECK_ARG(l->n >= 1, PW_ERR_INVALID, "pw_lanczos_resolvent: run at least one step first");
  const int64_t tot = l->nch * (int64_t)nz;
  hipLaunchKernelGGL(k_lz_cfrac, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     l->alpha, (int64_t)l->max_steps, l->beta, (int64_t)(l->max_steps + 1), l->n,
                     static_cast<const double2 *>(z), nz, l->nch, static_cast<double2 *>(g));
  PW_HIP(hipGetLastError());
  return PW_OK;
}

}  // extern "C"
