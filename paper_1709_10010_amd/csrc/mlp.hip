// Learned diagonal preconditioner: features, network, training, Adam (FP32).
//
// Not in the paper (it names the iterative diagonalisation, not its
// preconditioner); the workload defines it.  Per sample (G, n):
//   f = (t(G)/T_n, theta_n, |R_n(G)| sqrt(npw) / ||R_n||, <V_LOC>), standardised,
//   with T_n = <x_n|t|x_n> / <x_n|x_n> the band's kinetic energy, so the
//   first feature is the TPA argument and carries over between cutoffs
//   z = W3 silu(W2 silu(W1 f + b1) + b2) + b3                (4 -> 64 -> 64 -> 1)
//   s = S_LO + (S_HI - S_LO) sigmoid(z),  S_LO = 1/4, S_HI = 4
//   T_n(G) = s K_TPA(t(G)/T_n) R_n(G): the network learns a per-G scale on
//   top of the Teter-Payne-Allan diagonal (s = 1 reproduces TPA).  The
//   bounded range keeps the learned operator spectrally equivalent to TPA
//   (condition number of the ratio at most 16): an unbounded scale learns to
//   switch G components off, and a Davidson space never regains them.  A band
//   with any non-finite s falls back to plain TPA.
// Training minimises, per band sample, 1 - |<d, sR>|^2 / (||d||^2 ||sR||^2)
// (d: the part outside the current Ritz vectors of the move from the
// iterate to its converged cluster), averaged
// over the bands of a batch, with Adam (Kingma & Ba 2015).
//
// Parameters live in one packed float array (see kOff*).  Gradients are
// accumulated per workgroup and summed by a second kernel in a fixed order,
// so a training step is bitwise reproducible.
#include <cmath>
#include <cstring>

#include "common.h"

namespace pw {

constexpr int H = 64;
constexpr int kOffW1 = 0;             // [64][4]
constexpr int kOffB1 = kOffW1 + H * 4;  // [64]
constexpr int kOffW2 = kOffB1 + H;      // [64][64]
constexpr int kOffB2 = kOffW2 + H * H;  // [64]
constexpr int kOffW3 = kOffB2 + H;      // [64]
constexpr int kOffB3 = kOffW3 + H;      // [1]
constexpr int kNParam = kOffB3 + 1;     // 4545
constexpr int kTrainBlocks = 512;
constexpr int kChunk = 64;              // samples per training sub-step (one per thread)

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}
constexpr float kSLo = 0.25f, kSHi = 4.0f;
__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float scale_out(float z) { return kSLo + (kSHi - kSLo) * sigm(z); }
__device__ __forceinline__ float dscale_out(float z) {
  const float q = sigm(z);
  return (kSHi - kSLo) * q * (1.0f - q);
}

// standardised features of sample (g, n)
__device__ __forceinline__ void features(const double *kin, int64_t g, double itn, double theta,
                                         double2 r, double rnorm, double sqrt_npw, double vavg,
                                         const float *scaler, float f[4]) {
  const double amp = sqrt(r.x * r.x + r.y * r.y) * sqrt_npw / rnorm;
  const double raw[4] = {kin[g] * itn, theta, amp, vavg};
#pragma unroll
  for (int k = 0; k < 4; ++k) f[k] = (float)((raw[k] - (double)scaler[k]) * (double)scaler[4 + k]);
}

// forward of one sample with weights in LDS; returns z3 (before the output map)
__device__ __forceinline__ float mlp_z3(const float *W, const float f[4]) {
  float a1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float *w = W + kOffW1 + 4 * i;
    a1[i] = silu(W[kOffB1 + i] + w[0] * f[0] + w[1] * f[1] + w[2] * f[2] + w[3] * f[3]);
  }
  float z3 = W[kOffB3];
#pragma unroll 1
  for (int i = 0; i < H; ++i) {
    const float4 *w2 = reinterpret_cast<const float4 *>(W + kOffW2 + H * i);
    float z = W[kOffB2 + i];
#pragma unroll
    for (int j4 = 0; j4 < H / 4; ++j4) {
      const float4 w = w2[j4];
      z += w.x * a1[4 * j4] + w.y * a1[4 * j4 + 1] + w.z * a1[4 * j4 + 2] + w.w * a1[4 * j4 + 3];
    }
    z3 += W[kOffW3 + i] * silu(z);
  }
  return z3;
}

__device__ __forceinline__ void load_weights(float *Ws, const float *W) {
  for (int i = threadIdx.x; i < kNParam; i += blockDim.x) Ws[i] = W[i];
  __syncthreads();
}

// ---------------------------------------------------------------- features (raw)
// F[(i*npw + g)] = raw features of band idx[i] (idx may be null: i itself).
__global__ void k_features(const double *__restrict__ kin, const double *__restrict__ tn,
                           const double *__restrict__ theta, const double2 *__restrict__ R, int64_t ld,
                           const double *__restrict__ rnorm, const int *__restrict__ idx, int64_t npw,
                           double vavg, float4 *__restrict__ F) {
  const int i = blockIdx.y;
  const int n = idx ? idx[i] : i;
  const double sq = sqrt((double)npw);
  const double th = theta[n], rn = rnorm[n], itn = 1.0 / tn[n];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double2 r = R[(int64_t)n * ld + g];
    const double amp = sqrt(r.x * r.x + r.y * r.y) * sq / rn;
    F[(int64_t)i * npw + g] = float4{(float)(kin[g] * itn), (float)th, (float)amp, (float)vavg};
  }
}

// ---------------------------------------------------------------- inference
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ W,
                                                     const float *__restrict__ scaler,
                                                     const float4 *__restrict__ F, int64_t n,
                                                     float *__restrict__ s) {
  __shared__ __align__(16) float Ws[kNParam + 3];
  load_weights(Ws, W);
  const float mu[4] = {scaler[0], scaler[1], scaler[2], scaler[3]};
  const float is[4] = {scaler[4], scaler[5], scaler[6], scaler[7]};
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float4 r = F[e];
    const float f[4] = {(r.x - mu[0]) * is[0], (r.y - mu[1]) * is[1], (r.z - mu[2]) * is[2],
                        (r.w - mu[3]) * is[3]};
    s[e] = scale_out(mlp_z3(Ws, f));
  }
}

__device__ __forceinline__ double tpa_k3(double x);

// T[i](G) = s(G, idx[i]) K_TPA R[idx[i]](G); bad[i] = 1 if any s of the band is not finite
__global__ __launch_bounds__(256) void k_mlp_precond(const float *__restrict__ W,
                                                     const float *__restrict__ scaler,
                                                     const double *__restrict__ kin,
                                                     const double *__restrict__ theta,
                                                     const double2 *__restrict__ R, int64_t ld,
                                                     const double *__restrict__ rnorm,
                                                     const int *__restrict__ idx, int64_t npw,
                                                     double vavg, const double *__restrict__ tn,
                                                     double2 *__restrict__ T, int64_t ldt,
                                                     int *__restrict__ bad) {
  __shared__ __align__(16) float Ws[kNParam + 3];
  load_weights(Ws, W);
  const int i = blockIdx.y;
  const int n = idx[i];
  const double sq = sqrt((double)npw);
  const double th = theta[n], rn = rnorm[n], itn = 1.0 / tn[n];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double2 r = R[(int64_t)n * ld + g];
    float f[4];
    features(kin, g, itn, th, r, rn, sq, vavg, scaler, f);
    const float sv = scale_out(mlp_z3(Ws, f));
    if (!isfinite(sv)) bad[i] = 1;
    const double k = (double)sv * tpa_k3(kin[g] * itn);
    T[(int64_t)i * ldt + g] = double2{k * r.x, k * r.y};
  }
}

// bands flagged bad: T = TPA(R)
__device__ __forceinline__ double tpa_k3(double x) {
  const double num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0));
  const double x2 = x * x;
  return num / (num + 16.0 * x2 * x2);
}
__global__ void k_precond_fallback(const int *__restrict__ bad, const double *__restrict__ kin,
                                   const double *__restrict__ tn, const int *__restrict__ idx,
                                   const double2 *__restrict__ R, int64_t ld, double2 *__restrict__ T,
                                   int64_t ldt, int64_t npw) {
  const int i = blockIdx.y;
  if (!bad[i]) return;
  const int n = idx[i];
  const double inv = 1.0 / tn[n];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = R[(int64_t)n * ld + g];
    const double k = tpa_k3(kin[g] * inv);
    T[(int64_t)i * ldt + g] = double2{k * v.x, k * v.y};
  }
}

// ---------------------------------------------------------------- training
// per band b (samples off[b] .. off[b+1]): a = sum conj(d) s r, nu = sum s^2 |r|^2,
// nd = sum |d|^2, loss = 1 - |a|^2 / (nd nu).  stats[b] = (a.re, a.im, nu, nd, loss)
__global__ __launch_bounds__(256) void k_band_stats(const float *__restrict__ s,
                                                    const double2 *__restrict__ R,
                                                    const double2 *__restrict__ D,
                                                    const int64_t *__restrict__ off,
                                                    double *__restrict__ stats) {
  __shared__ double red[4][256];
  const int b = blockIdx.x;
  double ar = 0, ai = 0, nu = 0, nd = 0;
  for (int64_t e = off[b] + threadIdx.x; e < off[b + 1]; e += 256) {
    const double sv = s[e];
    const double2 r = R[e], d = D[e];
    // conj(d) * s r
    ar += sv * (d.x * r.x + d.y * r.y);
    ai += sv * (d.x * r.y - d.y * r.x);
    nu += sv * sv * (r.x * r.x + r.y * r.y);
    nd += d.x * d.x + d.y * d.y;
  }
  red[0][threadIdx.x] = ar;
  red[1][threadIdx.x] = ai;
  red[2][threadIdx.x] = nu;
  red[3][threadIdx.x] = nd;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = stats + 5 * (int64_t)b;
    o[0] = red[0][0];
    o[1] = red[1][0];
    o[2] = red[2][0];
    o[3] = red[3][0];
    o[4] = 1.0 - (red[0][0] * red[0][0] + red[1][0] * red[1][0]) / (red[3][0] * red[2][0]);
  }
}

// One wave per block; each 64-sample chunk: thread t runs sample t forward
// and backward into LDS, then thread t owns gradient entries t, t+64, ...
// and sums them over the chunk.  Block partials go to part[block][kNParam].
__global__ __launch_bounds__(64) void k_train_bwd(const float *__restrict__ W,
                                                  const float *__restrict__ scaler,
                                                  const float4 *__restrict__ F,
                                                  const double2 *__restrict__ R,
                                                  const double2 *__restrict__ D,
                                                  const float *__restrict__ s,
                                                  const int *__restrict__ band_of,
                                                  const double *__restrict__ stats, int64_t n,
                                                  double inv_nbands, float *__restrict__ part) {
  __shared__ __align__(16) float Ws[kNParam + 3];
  __shared__ float Gs[kNParam + 3];
  __shared__ float A1[kChunk][H + 1], A2[kChunk][H + 1], DZ1[kChunk][H + 1], DZ2[kChunk][H + 1];
  __shared__ float Fs[kChunk][4], DZ3[kChunk];
  load_weights(Ws, W);
  for (int i = threadIdx.x; i < kNParam; i += 64) Gs[i] = 0.0f;
  const int t = threadIdx.x;
  const float mu[4] = {scaler[0], scaler[1], scaler[2], scaler[3]};
  const float is[4] = {scaler[4], scaler[5], scaler[6], scaler[7]};
  const int64_t nchunk = (n + kChunk - 1) / kChunk;
  for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const int64_t e = c * kChunk + t;
    float dz3 = 0.0f;
    if (e < n) {
      const float4 r4 = F[e];
      float f[4] = {(r4.x - mu[0]) * is[0], (r4.y - mu[1]) * is[1], (r4.z - mu[2]) * is[2],
                    (r4.w - mu[3]) * is[3]};
      float z1[H];
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const float *w = Ws + kOffW1 + 4 * i;
        z1[i] = Ws[kOffB1 + i] + w[0] * f[0] + w[1] * f[1] + w[2] * f[2] + w[3] * f[3];
        A1[t][i] = silu(z1[i]);
      }
      float z3 = Ws[kOffB3];
      float z2s[H];
#pragma unroll 4
      for (int i = 0; i < H; ++i) {
        float z = Ws[kOffB2 + i];
#pragma unroll 8
        for (int j = 0; j < H; ++j) z += Ws[kOffW2 + H * i + j] * A1[t][j];
        z2s[i] = z;
        const float a2 = silu(z);
        A2[t][i] = a2;
        z3 += Ws[kOffW3 + i] * a2;
      }
      // dL/ds for this sample
      const int b = band_of[e];
      const double *st = stats + 5 * (int64_t)b;
      const double sv = s[e];
      const double2 r = R[e], d = D[e];
      const double a2abs = st[0] * st[0] + st[1] * st[1];
      // d|a|^2/ds = 2 Re(conj(a) conj(d) r)
      const double cdr_re = d.x * r.x + d.y * r.y, cdr_im = d.x * r.y - d.y * r.x;
      const double da2 = 2.0 * (st[0] * cdr_re + st[1] * cdr_im);
      const double dnu = 2.0 * sv * (r.x * r.x + r.y * r.y);
      const double ds = -(da2 * st[2] - a2abs * dnu) / (st[3] * st[2] * st[2]) * inv_nbands;
      dz3 = (float)ds * dscale_out(z3);
      float dz2[H];
      for (int i = 0; i < H; ++i) {
        dz2[i] = dz3 * Ws[kOffW3 + i] * dsilu(z2s[i]);
        DZ2[t][i] = dz2[i];
      }
#pragma unroll 1
      for (int j = 0; j < H; ++j) {
        float dh = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) dh += Ws[kOffW2 + H * i + j] * dz2[i];
        DZ1[t][j] = dh * dsilu(z1[j]);
      }
      for (int k = 0; k < 4; ++k) Fs[t][k] = f[k];
    } else {
      for (int i = 0; i < H; ++i) A1[t][i] = A2[t][i] = DZ1[t][i] = DZ2[t][i] = 0.0f;
      for (int k = 0; k < 4; ++k) Fs[t][k] = 0.0f;
    }
    DZ3[t] = dz3;
    __syncthreads();
    for (int p = t; p < kNParam; p += 64) {
      float acc = 0.0f;
      if (p < kOffB1) {
        const int i = p / 4, k = p % 4;
        for (int q = 0; q < kChunk; ++q) acc += DZ1[q][i] * Fs[q][k];
      } else if (p < kOffW2) {
        const int i = p - kOffB1;
        for (int q = 0; q < kChunk; ++q) acc += DZ1[q][i];
      } else if (p < kOffB2) {
        const int i = (p - kOffW2) / H, j = (p - kOffW2) % H;
        for (int q = 0; q < kChunk; ++q) acc += DZ2[q][i] * A1[q][j];
      } else if (p < kOffW3) {
        const int i = p - kOffB2;
        for (int q = 0; q < kChunk; ++q) acc += DZ2[q][i];
      } else if (p < kOffB3) {
        const int j = p - kOffW3;
        for (int q = 0; q < kChunk; ++q) acc += DZ3[q] * A2[q][j];
      } else {
        for (int q = 0; q < kChunk; ++q) acc += DZ3[q];
      }
      Gs[p] += acc;
    }
    __syncthreads();
  }
  for (int p = t; p < kNParam; p += 64) part[(int64_t)blockIdx.x * kNParam + p] = Gs[p];
}

__global__ void k_sum_partials(const float *__restrict__ part, int nblk, float *__restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParam) return;
  float acc = 0.0f;
  for (int b = 0; b < nblk; ++b) acc += part[(int64_t)b * kNParam + p];
  grad[p] = acc;
}

__global__ void k_adam(float *__restrict__ W, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParam) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / c1, vh = vp / c2;
  W[p] -= lr * mh / (sqrtf(vh) + eps);
}

// mean / inverse std of raw features -> scaler
__global__ __launch_bounds__(256) void k_fit_scaler(const float4 *__restrict__ F, int64_t n,
                                                    float *__restrict__ scaler) {
  __shared__ double red[8][256];
  double s[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0};
  for (int64_t e = threadIdx.x; e < n; e += 256) {
    const float4 f = F[e];
    const double v[4] = {f.x, f.y, f.z, f.w};
    for (int k = 0; k < 4; ++k) {
      s[k] += v[k];
      q[k] += v[k] * v[k];
    }
  }
  for (int k = 0; k < 4; ++k) {
    red[k][threadIdx.x] = s[k];
    red[4 + k][threadIdx.x] = q[k];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) {
      const double mu = red[k][0] / (double)n;
      const double var = red[4 + k][0] / (double)n - mu * mu;
      scaler[k] = (float)mu;
      scaler[4 + k] = var > 1e-20 ? (float)(1.0 / sqrt(var)) : 0.0f;
    }
  }
}

// targets: Dt[n] = y_n / ||y_n|| - x_n with y = Xc Cm, Cm = masked Xc^H x
__global__ void k_cluster_mask(double2 *__restrict__ C, int ldc, int nb, const int *__restrict__ cid) {
  const int64_t tot = (int64_t)nb * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(e % nb), n = (int)(e / nb);
    if (cid[m] != cid[n]) C[m + (int64_t)n * ldc] = double2{0.0, 0.0};
  }
}
__global__ __launch_bounds__(256) void k_target_finish(const double2 *__restrict__ X,
                                                       double2 *__restrict__ Y, int64_t ld,
                                                       int64_t npw) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int64_t g = threadIdx.x; g < npw; g += 256) {
    const double2 y = Y[(int64_t)b * ld + g];
    s += y.x * y.x + y.y * y.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  for (int64_t g = threadIdx.x; g < npw; g += 256) {
    const double2 y = Y[(int64_t)b * ld + g], x = X[(int64_t)b * ld + g];
    Y[(int64_t)b * ld + g] = double2{y.x * inv - x.x, y.y * inv - x.y};
  }
}

}  // namespace pw

using namespace pw;

struct pw_mlp {
  float *W = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *scaler = nullptr;
  float *part = nullptr;
  double *stats = nullptr;
  int64_t stats_cap = 0;
  int t = 0;
};

namespace pw {
int mlp_precond_idx(const pw_mlp *net, pw_problem *p, const double *theta, const double *rnorm,
                    const int *idx, const double2 *R, int64_t ld, double2 *T, int nu, int *bad,
                    const double *tn, hipStream_t s) {
  if (nu <= 0) return PW_OK;
  // bad[] arrives holding the bands already routed to TPA; the kernel adds
  // bands with a non-finite network output
  int bx = (int)((p->npw + 255) / 256);
  if (bx > 128) bx = 128;
  hipLaunchKernelGGL(k_mlp_precond, dim3(bx, nu), dim3(256), 0, s, net->W, net->scaler, p->d_kin,
                     theta, R, ld, rnorm, idx, p->npw, p->vavg, tn, T, ld, bad);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

int mlp_fallback(const int *bad, pw_problem *p, const double *tn, const int *idx, const double2 *R,
                 int64_t ld, double2 *T, int nu, hipStream_t s) {
  if (nu <= 0) return PW_OK;
  int bx = (int)((p->npw + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_precond_fallback, dim3(bx, nu), dim3(256), 0, s, bad, p->d_kin, tn, idx, R, ld,
                     T, ld, p->npw);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}
}  // namespace pw

extern "C" {

pw_status pw_mlp_create(const float *params, const float *scaler, pw_mlp **out) {
  PW_CHECK_ARG(out, PW_ERR_INVALID, "pw_mlp_create: null out");
  *out = nullptr;
  pw_mlp *n = new pw_mlp();
  const size_t pb = kNParam * sizeof(float);
  if (hipMalloc(&n->W, pb) != hipSuccess || hipMalloc(&n->grad, pb) != hipSuccess ||
      hipMalloc(&n->m, pb) != hipSuccess || hipMalloc(&n->v, pb) != hipSuccess ||
      hipMalloc(&n->scaler, 8 * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->part, (size_t)kTrainBlocks * pb) != hipSuccess) {
    pw_mlp_destroy(n);
    set_error("pw_mlp_create: device allocation failed");
    return PW_ERR_NOMEM;
  }
  float sc[8] = {0, 0, 0, 0, 1, 1, 1, 1};
  if (scaler) std::memcpy(sc, scaler, sizeof sc);
  std::vector<float> w(kNParam, 0.0f);
  if (params) std::memcpy(w.data(), params, pb);
  PW_HIP(hipMemcpy(n->W, w.data(), pb, hipMemcpyHostToDevice));
  PW_HIP(hipMemcpy(n->scaler, sc, sizeof sc, hipMemcpyHostToDevice));
  PW_HIP(hipMemset(n->m, 0, pb));
  PW_HIP(hipMemset(n->v, 0, pb));
  PW_HIP(hipMemset(n->grad, 0, pb));
  *out = n;
  return PW_OK;
}

pw_status pw_mlp_destroy(pw_mlp *n) {
  if (!n) return PW_OK;
  (void)hipDeviceSynchronize();
  void *b[] = {n->W, n->grad, n->m, n->v, n->scaler, n->part, n->stats};
  for (void *x : b)
    if (x) (void)hipFree(x);
  delete n;
  return PW_OK;
}

int32_t pw_mlp_num_params(void) { return kNParam; }

pw_status pw_mlp_get(pw_mlp *n, float *params, float *scaler, float *grad) {
  PW_CHECK_ARG(n, PW_ERR_INVALID, "pw_mlp_get: null network");
  PW_HIP(hipDeviceSynchronize());
  if (params) PW_HIP(hipMemcpy(params, n->W, kNParam * sizeof(float), hipMemcpyDeviceToHost));
  if (scaler) PW_HIP(hipMemcpy(scaler, n->scaler, 8 * sizeof(float), hipMemcpyDeviceToHost));
  if (grad) PW_HIP(hipMemcpy(grad, n->grad, kNParam * sizeof(float), hipMemcpyDeviceToHost));
  return PW_OK;
}

pw_status pw_mlp_set(pw_mlp *n, const float *params, const float *scaler) {
  PW_CHECK_ARG(n, PW_ERR_INVALID, "pw_mlp_set: null network");
  PW_HIP(hipDeviceSynchronize());
  if (params) PW_HIP(hipMemcpy(n->W, params, kNParam * sizeof(float), hipMemcpyHostToDevice));
  if (scaler) PW_HIP(hipMemcpy(n->scaler, scaler, 8 * sizeof(float), hipMemcpyHostToDevice));
  return PW_OK;
}

pw_status pw_mlp_features(pw_problem *p, const double *theta, const void *x, const void *r,
                          const double *rnorm, int64_t ld, int64_t nbands, void *F, void *stream) {
  PW_CHECK_ARG(p && theta && x && r && rnorm && F && ld >= p->npw && nbands >= 0 &&
                   nbands <= p->max_bands,
               PW_ERR_INVALID, "pw_mlp_features: bad argument");
  if (nbands == 0) return PW_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = band_kinetic(p->d_kin, x, ld, p->npw, (int)nbands, p->d_tn, s);
  if (rc != PW_OK) return rc;
  int bx = (int)((p->npw + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_features, dim3(bx, (unsigned)nbands), dim3(256), 0, s, p->d_kin, p->d_tn, theta,
                     static_cast<const double2 *>(r), ld, rnorm, (const int *)nullptr, p->npw, p->vavg,
                     static_cast<float4 *>(F));
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_fit_scaler(pw_mlp *n, const void *F, int64_t nsamples, void *stream) {
  PW_CHECK_ARG(n && F && nsamples > 0, PW_ERR_INVALID, "pw_mlp_fit_scaler: bad argument");
  hipLaunchKernelGGL(k_fit_scaler, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const float4 *>(F), nsamples, n->scaler);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_forward(pw_mlp *n, const void *F, int64_t nsamples, float *s, void *stream) {
  PW_CHECK_ARG(n && F && s && nsamples >= 0, PW_ERR_INVALID, "pw_mlp_forward: bad argument");
  if (nsamples == 0) return PW_OK;
  int64_t blocks = (nsamples + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     n->W, n->scaler, static_cast<const float4 *>(F), nsamples, s);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_mlp_train_step(pw_mlp *n, const void *F, const void *R, const void *D,
                            const int64_t *band_off, const int32_t *band_of, int64_t nbands,
                            int64_t nsamples, float *s_work, float lr, int32_t update,
                            double *loss_out, void *stream) {
  PW_CHECK_ARG(n && F && R && D && band_off && band_of && s_work && nbands > 0 && nsamples > 0,
               PW_ERR_INVALID, "pw_mlp_train_step: bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (n->stats_cap < nbands) {
    if (n->stats) (void)hipFree(n->stats);
    n->stats = nullptr;
    if (hipMalloc(&n->stats, (size_t)nbands * 5 * sizeof(double)) != hipSuccess) {
      set_error("pw_mlp_train_step: allocation failed");
      return PW_ERR_NOMEM;
    }
    n->stats_cap = nbands;
  }
  PW_CHECK_ARG(pw_mlp_forward(n, F, nsamples, s_work, stream) == PW_OK, PW_ERR_HIP,
               "pw_mlp_train_step: forward failed");
  hipLaunchKernelGGL(k_band_stats, dim3((unsigned)nbands), dim3(256), 0, st, s_work,
                     static_cast<const double2 *>(R), static_cast<const double2 *>(D), band_off, n->stats);
  PW_HIP(hipGetLastError());
  int64_t nchunk = (nsamples + kChunk - 1) / kChunk;
  const int nblk = (int)std::min<int64_t>(kTrainBlocks, nchunk);
  hipLaunchKernelGGL(k_train_bwd, dim3(nblk), dim3(64), 0, st, n->W, n->scaler,
                     static_cast<const float4 *>(F), static_cast<const double2 *>(R),
                     static_cast<const double2 *>(D), s_work, band_of, n->stats, nsamples,
                     1.0 / (double)nbands, n->part);
  PW_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3((kNParam + 255) / 256), dim3(256), 0, st, n->part, nblk, n->grad);
  PW_HIP(hipGetLastError());
  if (update) {
    n->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)n->t), c2 = 1.0f - std::pow(b2, (float)n->t);
    hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, n->W, n->grad, n->m, n->v,
                       lr, b1, b2, 1e-8f, c1, c2);
    PW_HIP(hipGetLastError());
  }
  if (loss_out) {
    std::vector<double> st_h((size_t)nbands * 5);
    PW_HIP(hipMemcpyAsync(st_h.data(), n->stats, st_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    double l = 0;
    for (int64_t b = 0; b < nbands; ++b) l += st_h[5 * b + 4];
    *loss_out = l / (double)nbands;
  }
  return PW_OK;
}

pw_status pw_mlp_targets(pw_problem *p, const void *Xc, const int32_t *cluster, const void *Xit,
                         int64_t ld, int64_t nbands, void *D, void *work, void *stream) {
  PW_CHECK_ARG(p && Xc && cluster && Xit && D && work && ld >= p->npw && nbands > 0, PW_ERR_INVALID,
               "pw_mlp_targets: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double2 *C = static_cast<double2 *>(work);  // nbands x nbands, then split-K partials
  double2 *part = C + nbands * nbands;
  int splits = choose_splits(nbands, nbands, p->npw);
  if (splits > 16) splits = 16;
  int rc = zgemm_cn(nbands, nbands, p->npw, Xc, ld, Xit, ld, C, nbands, splits, part, s);
  if (rc != PW_OK) return rc;
  hipLaunchKernelGGL(k_cluster_mask, dim3(256), dim3(256), 0, s, C, (int)nbands, (int)nbands, cluster);
  PW_HIP(hipGetLastError());
  rc = zgemm_nn(p->npw, nbands, nbands, 1.0, Xc, ld, C, nbands, 0.0, D, ld, s);
  if (rc != PW_OK) return rc;
  hipLaunchKernelGGL(k_target_finish, dim3((unsigned)nbands), dim3(256), 0, s,
                     static_cast<const double2 *>(Xit), static_cast<double2 *>(D), ld, p->npw);
  PW_HIP(hipGetLastError());
  // keep only the part outside span(Xit): the Rayleigh-Ritz step supplies
  // the rest, so it is no part of what a correction has to carry
  rc = zgemm_cn(nbands, nbands, p->npw, Xit, ld, D, ld, C, nbands, splits, part, s);
  if (rc != PW_OK) return rc;
  return zgemm_nn(p->npw, nbands, nbands, -1.0, Xit, ld, C, nbands, 1.0, D, ld, s);
}

}  // extern "C"
