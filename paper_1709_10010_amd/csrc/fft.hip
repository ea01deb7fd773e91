// Local-potential part of H*psi on the FFT grid (CDNA4 / gfx950).
//
// Operation (paper, eq. pauli_ks: V_LOC acts on the FFT mesh; the
// exchange paragraph's grid rule G_max = 2 G_c fixes the mesh):
//   u(r) = sum_G psi(G) e^{+iG.r}          inverse 3D FFT of the sphere
//   w(r) = V(r) u(r)                        pointwise, V real
//   (V psi)(G) = N^-3 sum_r w(r) e^{-iG.r}  forward 3D FFT, kept on the sphere
// The paper puts the non-linear scaling of the method on these FFTs and
// spreads the bands of the V psi products over "task groups"; here the
// bands of a block are the batch dimension of every launch.
//
// Three kernels, each staging its data through LDS exactly once:
//   k_zfft_inv  per (tile of z-sticks, band): gather psi(G) of the tile's
//               sticks into LDS, inverse FFT along z, store the tile to the
//               stick buffer [band][z][stick] (coalesced across sticks).
//   k_plane     per (z-plane, group of bands): scatter the plane's stick
//               values into an LDS plane, inverse FFT along y on the rows
//               that hold sticks, inverse along x, multiply by V / N^3,
//               forward along x, forward along y on the stick rows, store
//               the sticks back.  V's plane is re-read from L2 per band.
//   k_zfft_fwd  per (tile, band): forward FFT along z, gather the sphere,
//               add the kinetic term t(G) psi(G), write H psi.
// Only the grid columns that hold sphere points (the z-sticks) ever travel
// through HBM; the pruned y passes skip rows without sticks.  The G order
// is the caller's: listed by stick (x, then y, then z on the grid) the z
// passes read psi and write H psi in order, any other order costs a
// gather / scatter through the stick map.
//
// FFTs are in-place Stockham passes in LDS: in each radix-R pass every
// thread loads its butterflies' R inputs into registers, applies the
// twiddles and the R-point DFT, all threads barrier, then every thread
// stores its outputs at their autosorted positions.  Radices 2, 3, 4, 5, 8.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace pw {

// ---------------------------------------------------------------- complex ops
template <typename V> __device__ __forceinline__ V c_add(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V c_sub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V c_mul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V c_mulconj(V a, V b) {  // a * conj(b)
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V, typename S> __device__ __forceinline__ V c_scale(V a, S s) { return V{a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __device__ __forceinline__ V c_rot(V a) {
  return INV ? V{-a.y, a.x} : V{a.y, -a.x};
}

// ---------------------------------------------------------------- small DFTs
template <int R, bool INV, typename V> struct Dft;

template <bool INV, typename V> struct Dft<2, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    V a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <bool INV, typename V> struct Dft<4, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    V t0 = c_add(v[0], v[2]), t1 = c_sub(v[0], v[2]);
    V t2 = c_add(v[1], v[3]), t3 = c_rot<INV>(c_sub(v[1], v[3]));
    v[0] = c_add(t0, t2);
    v[2] = c_sub(t0, t2);
    v[1] = c_add(t1, t3);
    v[3] = c_sub(t1, t3);
  }
};

template <bool INV, typename V> struct Dft<3, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using S = decltype(v[0].x);
    const S h = S(0.86602540378443864676372317075294);  // sqrt(3)/2
    V t1 = c_add(v[1], v[2]);
    V t2 = c_sub(v[0], c_scale(t1, S(0.5)));
    V t3 = c_rot<INV>(c_scale(c_sub(v[1], v[2]), h));
    v[0] = c_add(v[0], t1);
    v[1] = c_add(t2, t3);
    v[2] = c_sub(t2, t3);
  }
};

template <bool INV, typename V> struct Dft<5, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using S = decltype(v[0].x);
    const S c1 = S(0.30901699437494742410229341718282);   // cos(2pi/5)
    const S c2 = S(-0.80901699437494742410229341718282);  // cos(4pi/5)
    const S s1 = S(0.95105651629515357211643933337938);   // sin(2pi/5)
    const S s2 = S(0.58778525229247312916870595463907);   // sin(4pi/5)
    V a1 = c_add(v[1], v[4]), b1 = c_sub(v[1], v[4]);
    V a2 = c_add(v[2], v[3]), b2 = c_sub(v[2], v[3]);
    V x0 = v[0];
    V p1 = V{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
    V p2 = V{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
    V q1 = c_rot<INV>(V{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    V q2 = c_rot<INV>(V{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = c_add(x0, c_add(a1, a2));
    v[1] = c_add(p1, q1);
    v[4] = c_sub(p1, q1);
    v[2] = c_add(p2, q2);
    v[3] = c_sub(p2, q2);
  }
};

template <bool INV, typename V> struct Dft<8, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using S = decltype(v[0].x);
    const S r = S(0.70710678118654752440084436210485);
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, V>::run(e);
    Dft<4, INV, V>::run(o);
    // w^k O_k with w = e^{-i pi/4} (forward) or its conjugate
    V w1 = INV ? V{r * (o[1].x - o[1].y), r * (o[1].x + o[1].y)}
               : V{r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
    V w2 = c_rot<INV>(o[2]);
    V w3 = INV ? V{-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)}
               : V{r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
    v[0] = c_add(e[0], o[0]);
    v[4] = c_sub(e[0], o[0]);
    v[1] = c_add(e[1], w1);
    v[5] = c_sub(e[1], w1);
    v[2] = c_add(e[2], w2);
    v[6] = c_sub(e[2], w2);
    v[3] = c_add(e[3], w3);
    v[7] = c_sub(e[3], w3);
  }
};

// ---------------------------------------------------------------- one Stockham pass
constexpr int kCpt = 8;  // complex values per thread and pass (register budget)

// q = a / d for 0 <= a < 2^22, 0 < d < 2^11, with inv = 1.0f / d: the float
// product is within 1/2 of a/d, so the truncated quotient is off by at most
// one and a single correction step makes it exact.  A few VALU instructions
// instead of the generic integer-division sequence.
__device__ __forceinline__ int qdiv(int a, int d, float inv) {
  int q = (int)((float)a * inv);
  const int r = a - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// Lines of length N live in LDS at base(line) + pos * estride.  base(line) is
// line * lstride, or lbase[line] when INDIRECT.  LINE_FAST maps consecutive
// threads to consecutive lines (strided lines), else to consecutive
// butterflies of one line (contiguous lines).  Each thread holds at most
// kCpt complex values: the host guarantees nlines * N <= kCpt * nthr.
template <typename V, int R, bool INV, bool LINE_FAST, bool INDIRECT>
__device__ __forceinline__ void stockham_pass(V *buf, int nlines, int lstride, int estride,
                                              const int *lbase, int N, int Ns, const V *tw,
                                              int tid_in, int nthr) {
  int tid = tid_in;  // opaque: see wave_pass
  asm volatile("" : "+v"(tid));
  constexpr int MAXB = (kCpt + R - 1) / R;
  const int nbf = N / R;
  const int total = nlines * nbf;
  const int twstep = N / (Ns * R);
  const int dsplit = LINE_FAST ? nlines : nbf;
  const float isplit = 1.0f / (float)dsplit;
  const float ins = 1.0f / (float)Ns;
  V v[MAXB][R];
  int bo[MAXB], oo[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = tid + c * nthr;
    if (idx < total) {
      const int q = qdiv(idx, dsplit, isplit);
      const int rem = idx - q * dsplit;
      const int line = LINE_FAST ? rem : q;
      const int j = LINE_FAST ? q : rem;
      const int base = INDIRECT ? lbase[line] : line * lstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = buf[base + (j + r * nbf) * estride];
      int k = 0;
      if (Ns > 1) {
        k = j - qdiv(j, Ns, ins) * Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const V w = tw[k * r * twstep];
          v[c][r] = INV ? c_mulconj(v[c][r], w) : c_mul(v[c][r], w);
        }
      }
      Dft<R, INV, V>::run(v[c]);
      bo[c] = base;
      oo[c] = (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = tid + c * nthr;
    if (idx < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[bo[c] + (oo[c] + r * Ns) * estride] = v[c][r];
    }
  }
  __syncthreads();
}

template <typename V, bool INV, bool LINE_FAST, bool INDIRECT>
__device__ void fft_lines(V *buf, int nlines, int lstride, int estride, const int *lbase,
                          const AxisPlan &pl, const V *tw, int tid, int nthr) {
  int Ns = 1;
  for (int p = 0; p < pl.npass; ++p) {
    const int R = pl.radix[p];
    switch (R) {
      case 2: stockham_pass<V, 2, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl.n, Ns, tw, tid, nthr); break;
      case 3: stockham_pass<V, 3, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl.n, Ns, tw, tid, nthr); break;
      case 4: stockham_pass<V, 4, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl.n, Ns, tw, tid, nthr); break;
      case 5: stockham_pass<V, 5, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl.n, Ns, tw, tid, nthr); break;
      default: stockham_pass<V, 8, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl.n, Ns, tw, tid, nthr); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------- compile-time plans
// For the grid sizes of the workloads the whole pass sequence is known at
// compile time: radix, butterfly count, twiddle stride and the j mod Ns
// divisor become constants, which removes most of the per-butterfly index
// arithmetic of the runtime passes above.
struct CtPlan {
  int n;
  int r[kMaxPasses];
};
constexpr CtPlan ct_plan(int N) {
  CtPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  int m = N, a = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++a;
  }
  while (a > 0) {
    if (a == 4) {
      p.r[p.n++] = 4;
      p.r[p.n++] = 4;
      a = 0;
    } else if (a >= 3) {
      p.r[p.n++] = 8;
      a -= 3;
    } else if (a == 2) {
      p.r[p.n++] = 4;
      a -= 2;
    } else {
      p.r[p.n++] = 2;
      a -= 1;
    }
  }
  while (m % 3 == 0) {
    p.r[p.n++] = 3;
    m /= 3;
  }
  while (m % 5 == 0) {
    p.r[p.n++] = 5;
    m /= 5;
  }
  return p;
}
constexpr int ct_npass(int N) { return ct_plan(N).n; }
constexpr int ct_radix(int N, int P) { return ct_plan(N).r[P]; }

template <typename V, int N, int NS, int R, bool INV, bool LINE_FAST, bool INDIRECT>
__device__ __forceinline__ void ct_pass(V *buf, int nlines, int lstride, int estride,
                                        const int *lbase, const V *tw, int tid_in, int nthr) {
  int tid = tid_in;
  asm volatile("" : "+v"(tid));
  constexpr int MAXB = (kCpt + R - 1) / R;
  constexpr int nbf = N / R;
  constexpr int twstep = N / (NS * R);
  const int total = nlines * nbf;
  const float inl = 1.0f / (float)nlines;
  V v[MAXB][R];
  int bo[MAXB], oo[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = tid + c * nthr;
    if (idx < total) {
      int line, j;
      if (LINE_FAST) {
        j = qdiv(idx, nlines, inl);
        line = idx - j * nlines;
      } else {
        line = idx / nbf;
        j = idx - line * nbf;
      }
      const int base = INDIRECT ? lbase[line] : line * lstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = buf[base + (j + r * nbf) * estride];
      int k = 0;
      if constexpr (NS > 1) {
        k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const V w = tw[k * r * twstep];
          v[c][r] = INV ? c_mulconj(v[c][r], w) : c_mul(v[c][r], w);
        }
      }
      Dft<R, INV, V>::run(v[c]);
      bo[c] = base;
      oo[c] = (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = tid + c * nthr;
    if (idx < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[bo[c] + (oo[c] + r * NS) * estride] = v[c][r];
    }
  }
  __syncthreads();
}

template <typename V, int N, int P, int NS, bool INV, bool LINE_FAST, bool INDIRECT>
__device__ __forceinline__ void ct_fft(V *buf, int nlines, int lstride, int estride, const int *lbase,
                                       const V *tw, int tid, int nthr) {
  if constexpr (P < ct_npass(N)) {
    constexpr int R = ct_radix(N, P);
    ct_pass<V, N, NS, R, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, tw, tid, nthr);
    ct_fft<V, N, P + 1, NS * R, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, tw, tid,
                                                         nthr);
  }
}

// NC > 0: compile-time length NC (must equal pl.n); NC == 0: runtime plan.
template <typename V, bool INV, bool LINE_FAST, bool INDIRECT, int NC>
__device__ __forceinline__ void fft_axis(V *buf, int nlines, int lstride, int estride, const int *lbase,
                                         const AxisPlan &pl, const V *tw, int tid, int nthr) {
  if constexpr (NC > 0)
    ct_fft<V, NC, 0, 1, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, tw, tid, nthr);
  else
    fft_lines<V, INV, LINE_FAST, INDIRECT>(buf, nlines, lstride, estride, lbase, pl, tw, tid, nthr);
}

// ---------------------------------------------------------------- register FFTs
// One thread transforms one line of compile-time length N held in its own
// registers: every index and every twiddle is a compile-time constant, so
// a line costs its butterflies and nothing else, and no barrier is needed
// inside a transform.
namespace rf {
struct CS {
  double c, s;
};
// cos and sin of 0 <= x <= pi/4: Taylor series, terms summed from the smallest
constexpr CS sincos_small(double x) {
  double tc[14] = {}, ts[14] = {};
  const double x2 = x * x;
  double a = 1.0, b = x;
  for (int k = 0; k < 14; ++k) {
    tc[k] = a;
    ts[k] = b;
    a *= -x2 / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
    b *= -x2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
  }
  double c = 0.0, s = 0.0;
  for (int k = 13; k >= 0; --k) {
    c += tc[k];
    s += ts[k];
  }
  return CS{c, s};
}
// e^{-2 pi i m / n}: the angle is reduced in integers to q quarter turns plus
// at most an eighth of a turn, so the series only sees |x| <= pi/4
constexpr CS twiddle(int m, int n) {
  m %= n;
  if (m < 0) m += n;
  const int q = (4 * m) / n, r = 4 * m - q * n;  // angle = (pi/2) (q + r/n)
  constexpr double kHalfPi = 1.57079632679489661923132169163975;
  CS e{0.0, 0.0};
  if (2 * r <= n) {
    e = sincos_small(kHalfPi * r / n);
  } else {
    const CS t = sincos_small(kHalfPi * (n - r) / n);
    e = CS{t.s, t.c};
  }
  for (int i = 0; i < q; ++i) e = CS{-e.s, e.c};
  return CS{e.c, -e.s};
}

// x[r] *= w^(r M) (forward) or its conjugate, r = 1 .. R-1; exact quarter
// turns become swaps and sign changes.  Other twiddles are compile-time
// constants, or with a table (tw[m * TS] = w_N^m, TS > 0) read from it at the
// point of use, which keeps them out of the registers between uses.
template <typename V, int N, int M, bool INV, int R, int TS, int r = 1>
__device__ __forceinline__ void tw_mul(V *x, const V *tw) {
  if constexpr (r < R) {
    constexpr int m = (r * M) % N;
    if constexpr (m != 0) {
      if constexpr ((4 * m) % N == 0) {
        constexpr int q = (4 * m) / N;
        if constexpr (q == 2) {
          x[r] = V{-x[r].x, -x[r].y};
        } else {
          x[r] = c_rot<INV>(x[r]);
          if constexpr (q == 3) x[r] = V{-x[r].x, -x[r].y};
        }
      } else {
        V wv;
        if constexpr (TS > 0) {
          wv = tw[m * TS];
        } else {
          using S = decltype(x[0].x);
          constexpr CS w = twiddle(m, N);
          wv = V{S(w.c), S(w.s)};
        }
        x[r] = INV ? c_mulconj(x[r], wv) : c_mul(x[r], wv);
      }
    }
    tw_mul<V, N, M, INV, R, TS, r + 1>(x, tw);
  }
}

// butterflies J, J+1, ... of one Stockham pass (radix R, NS = product of the
// radices before it), reading a and writing b
template <typename V, int N, int NS, int R, bool INV, int TS, int J>
__device__ __forceinline__ void pass_bf(const V *a, V *b, const V *tw) {
  if constexpr (J < N / R) {
    constexpr int NBF = N / R;
    constexpr int K = J % NS;
    V x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = a[J + r * NBF];
    if constexpr (NS > 1) tw_mul<V, N, K * (N / (NS * R)), INV, R, TS>(x, tw);
    Dft<R, INV, V>::run(x);
#pragma unroll
    for (int r = 0; r < R; ++r) b[(J - K) * R + K + r * NS] = x[r];
    pass_bf<V, N, NS, R, INV, TS, J + 1>(a, b, tw);
  }
}

template <typename V, int N, int P, int NS, bool INV, int TS>
__device__ __forceinline__ void passes(V *a, V *b, const V *tw) {
  if constexpr (P < ct_npass(N)) {
    constexpr int R = ct_radix(N, P);
    pass_bf<V, N, NS, R, INV, TS, 0>(a, b, tw);
    passes<V, N, P + 1, NS * R, INV, TS>(b, a, tw);
  }
}
}  // namespace rf

// v <- DFT_N(v) (unnormalised; forward e^{-2 pi i jk/N}, inverse e^{+...}),
// natural order in and out; twiddles from tw[m * TS] = w_N^m when TS > 0
template <typename V, int N, bool INV, int TS = 0>
__device__ __forceinline__ void reg_fft(V *v, const V *tw = nullptr) {
  V t[N];
  rf::passes<V, N, 0, 1, INV, TS>(v, t, tw);
  if constexpr (ct_npass(N) % 2 == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = t[i];
  }
}

// ---------------------------------------------------------------- wave-local FFTs
// One wavefront transforms lines it owns alone, so the read and write halves
// of a Stockham pass need no workgroup barrier: the wave's LDS operations
// execute in issue order and the compiler is kept from moving memory
// operations across the pass boundary.  Lines are taken in register-sized
// groups (ng * N <= kCpt * 64 values per pass) and each group runs all
// passes before the next group starts.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename V, int R, bool INV, bool LINE_FAST, typename Base>
__device__ __forceinline__ void wave_pass(V *buf, int ng, Base base, int estride, int N, int Ns,
                                          const V *tw, int lane_in) {
  // keep the per-lane index arithmetic inside the pass: hoisted out of the
  // pass loop it would stay live for every radix case at once
  int lane = lane_in;
  asm volatile("" : "+v"(lane));
  constexpr int MAXB = (kCpt + R - 1) / R;
  const int nbf = N / R;
  const int total = ng * nbf;
  const int twstep = N / (Ns * R);
  const int dsplit = LINE_FAST ? ng : nbf;
  const float isplit = 1.0f / (float)dsplit;
  const float ins = 1.0f / (float)Ns;
  V v[MAXB][R];
  int bo[MAXB], oo[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = lane + c * 64;
    if (idx < total) {
      const int q = qdiv(idx, dsplit, isplit);
      const int rem = idx - q * dsplit;
      const int line = LINE_FAST ? rem : q;
      const int j = LINE_FAST ? q : rem;
      const int b0 = base(line);
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = buf[b0 + (j + r * nbf) * estride];
      int k = 0;
      if (Ns > 1) {
        k = j - qdiv(j, Ns, ins) * Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const V w = tw[k * r * twstep];
          v[c][r] = INV ? c_mulconj(v[c][r], w) : c_mul(v[c][r], w);
        }
      }
      Dft<R, INV, V>::run(v[c]);
      bo[c] = b0;
      oo[c] = (j - k) * R + k;
    }
  }
  wave_sync();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int idx = lane + c * 64;
    if (idx < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[bo[c] + (oo[c] + r * Ns) * estride] = v[c][r];
    }
  }
  wave_sync();
}

template <typename V, bool INV, bool LINE_FAST, typename Base>
__device__ __forceinline__ void wave_fft_group(V *buf, int ng, Base base, int estride,
                                               const AxisPlan &pl, const V *tw, int lane) {
  int Ns = 1;
  for (int p = 0; p < pl.npass; ++p) {
    const int R = pl.radix[p];
    switch (R) {
      case 2: wave_pass<V, 2, INV, LINE_FAST>(buf, ng, base, estride, pl.n, Ns, tw, lane); break;
      case 3: wave_pass<V, 3, INV, LINE_FAST>(buf, ng, base, estride, pl.n, Ns, tw, lane); break;
      case 4: wave_pass<V, 4, INV, LINE_FAST>(buf, ng, base, estride, pl.n, Ns, tw, lane); break;
      case 5: wave_pass<V, 5, INV, LINE_FAST>(buf, ng, base, estride, pl.n, Ns, tw, lane); break;
      default: wave_pass<V, 8, INV, LINE_FAST>(buf, ng, base, estride, pl.n, Ns, tw, lane); break;
    }
    Ns *= R;
  }
}

// Block -> (tile, band) with every tile of a band on the same XCD (blocks
// are dealt to the 8 XCDs round-robin), so the band's psi / H psi lines
// are shared through one L2.  The grid is ntile * roundup(nb, 8) blocks.
__device__ __forceinline__ void tile_band(int bid, int ntile, int *tile, int *band) {
  const int xcd = bid & 7;
  const int q = bid >> 3;
  *tile = q % ntile;
  *band = (q / ntile) * 8 + xcd;
}

// ---------------------------------------------------------------- kernels
template <typename T, int NTHR, int NC>
__global__ __launch_bounds__(NTHR) void k_zfft_inv(FFTDev f, const double2 *__restrict__ psi,
                                                   int64_t ld, cpx_t<T> *__restrict__ sticks,
                                                   int nb) {
  using V = cpx_t<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  V *tw = reinterpret_cast<V *>(smem);
  V *buf = tw + f.n2;
  int tile, b;
  tile_band(blockIdx.x, f.ntile, &tile, &b);
  if (b >= nb) return;
  const int tid = threadIdx.x;
  const V *twg = static_cast<const V *>(f.tw2);
  for (int i = tid; i < f.n2; i += NTHR) tw[i] = twg[i];
  const int nel = f.ts * f.n2;
  for (int i = tid; i < nel; i += NTHR) buf[i] = V{0, 0};
  __syncthreads();
  const int e0 = f.tile_ptr[tile], e1 = f.tile_ptr[tile + 1];
  const double2 *src = psi + (int64_t)b * ld;
  for (int e = e0 + tid; e < e1; e += NTHR) {
    const double2 v = src[f.g_linear ? e : f.gidx[e]];
    buf[f.gpos[e]] = V{(T)v.x, (T)v.y};
  }
  __syncthreads();
  fft_axis<V, true, true, false, NC>(buf, f.ts, 1, f.ts, nullptr, f.pz, tw, tid, NTHR);
  V *dst = sticks + (int64_t)b * f.n2 * f.nst_pad + (int64_t)tile * f.ts;
  for (int i = tid; i < nel; i += NTHR) {
    const int z = i / f.ts;
    const int sl = i - z * f.ts;
    dst[(int64_t)z * f.nst_pad + sl] = buf[i];
  }
}

template <typename T, int NTHR, int NC>
__global__ __launch_bounds__(NTHR) void k_plane(FFTDev f, cpx_t<T> *__restrict__ sticks, int nb,
                                                int group) {
  using V = cpx_t<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  V *tw0 = reinterpret_cast<V *>(smem);
  V *tw1 = tw0 + f.n0;
  V *pl = tw1 + f.n1;
  int *lb = reinterpret_cast<int *>(pl + f.n0 * f.n1);
  const int z = blockIdx.x % f.n2;
  const int g = blockIdx.x / f.n2;
  const int tid = threadIdx.x;
  const V *tw0g = static_cast<const V *>(f.tw0);
  const V *tw1g = static_cast<const V *>(f.tw1);
  for (int i = tid; i < f.n0; i += NTHR) tw0[i] = tw0g[i];
  for (int i = tid; i < f.n1; i += NTHR) tw1[i] = tw1g[i];
  for (int i = tid; i < f.nx; i += NTHR) lb[i] = f.xlist[i] * f.n1;
  const int npl = f.n0 * f.n1;
  const T *vp = static_cast<const T *>(f.vplanes) + (int64_t)z * npl;
  for (int bb = 0; bb < group; ++bb) {
    const int b = g * group + bb;
    if (b >= nb) break;
    for (int i = tid; i < npl; i += NTHR) pl[i] = V{0, 0};
    __syncthreads();
    V *col = sticks + (int64_t)b * f.n2 * f.nst_pad + (int64_t)z * f.nst_pad;
    for (int s = tid; s < f.nst; s += NTHR) pl[f.stick_xy[s]] = col[s];
    __syncthreads();
    fft_axis<V, true, false, true, NC>(pl, f.nx, 0, 1, lb, f.py, tw1, tid, NTHR);
    fft_axis<V, true, true, false, NC>(pl, f.n1, 1, f.n1, nullptr, f.px, tw0, tid, NTHR);
    for (int i = tid; i < npl; i += NTHR) pl[i] = c_scale(pl[i], vp[i]);
    __syncthreads();
    fft_axis<V, false, true, false, NC>(pl, f.n1, 1, f.n1, nullptr, f.px, tw0, tid, NTHR);
    fft_axis<V, false, false, true, NC>(pl, f.nx, 0, 1, lb, f.py, tw1, tid, NTHR);
    for (int s = tid; s < f.nst; s += NTHR) col[s] = pl[f.stick_xy[s]];
    __syncthreads();
  }
}

// Plane pass with wave-owned lines: rows (y transforms) and columns (x
// transforms) are dealt to the waves in contiguous ranges; a wave runs the
// inverse x transform, the V(r) product and the forward x transform of its
// columns back to back.  Four workgroup barriers per band-plane.
template <typename T, int NTHR>
__global__ __launch_bounds__(NTHR) void k_plane_w(FFTDev f, cpx_t<T> *__restrict__ sticks, int nb,
                                                  int group) {
  using V = cpx_t<T>;
  constexpr int NW = NTHR / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  V *tw0 = reinterpret_cast<V *>(smem);
  V *tw1 = tw0 + f.n0;
  V *pl = tw1 + f.n1;
  int *lb = reinterpret_cast<int *>(pl + f.n0 * f.n1);
  const int z = blockIdx.x % f.n2;
  const int g = blockIdx.x / f.n2;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const V *tw0g = static_cast<const V *>(f.tw0);
  const V *tw1g = static_cast<const V *>(f.tw1);
  for (int i = tid; i < f.n0; i += NTHR) tw0[i] = tw0g[i];
  for (int i = tid; i < f.n1; i += NTHR) tw1[i] = tw1g[i];
  for (int i = tid; i < f.nx; i += NTHR) lb[i] = f.xlist[i] * f.n1;
  const int npl = f.n0 * f.n1;
  const T *vp = static_cast<const T *>(f.vplanes) + (int64_t)z * npl;
  // this wave's rows (indices into xlist) and columns
  const int rpw = (f.nx + NW - 1) / NW;
  const int r0 = min(f.nx, wv * rpw), r1 = min(f.nx, r0 + rpw);
  const int cpw = (f.n1 + NW - 1) / NW;
  const int c0 = min(f.n1, wv * cpw), c1 = min(f.n1, c0 + cpw);
  const int rg = max(1, (kCpt * 64) / f.n1);  // rows per register group
  const int cg = max(1, (kCpt * 64) / f.n0);  // columns per register group
  for (int bb = 0; bb < group; ++bb) {
    const int b = g * group + bb;
    if (b >= nb) break;
    for (int i = tid; i < npl; i += NTHR) pl[i] = V{0, 0};
    __syncthreads();
    V *col = sticks + (int64_t)b * f.n2 * f.nst_pad + (int64_t)z * f.nst_pad;
    for (int s = tid; s < f.nst; s += NTHR) pl[f.stick_xy[s]] = col[s];
    __syncthreads();
    for (int q = r0; q < r1; q += rg) {
      const int ng = min(rg, r1 - q);
      wave_fft_group<V, true, false>(pl, ng, [&](int l) { return lb[q + l]; }, 1, f.py, tw1, lane);
    }
    __syncthreads();
    for (int q = c0; q < c1; q += cg) {
      const int ng = min(cg, c1 - q);
      auto base = [&](int l) { return q + l; };
      wave_fft_group<V, true, true>(pl, ng, base, f.n1, f.px, tw0, lane);
      const float ing = 1.0f / (float)ng;
      for (int e = lane; e < ng * f.n0; e += 64) {
        const int x = qdiv(e, ng, ing);
        const int o = x * f.n1 + q + (e - x * ng);
        pl[o] = c_scale(pl[o], vp[o]);
      }
      wave_sync();
      wave_fft_group<V, false, true>(pl, ng, base, f.n1, f.px, tw0, lane);
    }
    __syncthreads();
    for (int q = r0; q < r1; q += rg) {
      const int ng = min(rg, r1 - q);
      wave_fft_group<V, false, false>(pl, ng, [&](int l) { return lb[q + l]; }, 1, f.py, tw1, lane);
    }
    __syncthreads();
    for (int s = tid; s < f.nst; s += NTHR) col[s] = pl[f.stick_xy[s]];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- lane-group FFTs
// A line of length N = L M (L = 2, 4 or 8) is shared by L consecutive
// lanes, which run in lockstep: each holds M values and transforms them as
// an M-point line in registers, and log2(L) radix-2 levels join the lanes
// through cross-lane moves (DPP quad permutations: [1,0,3,2] swaps lanes
// differing in bit 0, [2,3,0,1] lanes differing in bit 1; a swizzle with
// xor mask 4 lanes differing in bit 2).
template <int B> __device__ __forceinline__ int lane_xchg(int v) {
  if constexpr (B == 2)  // lanes differing in bit 2: swizzle with xor mask 4 (and 0x1F, or 0)
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
  else
    return __builtin_amdgcn_update_dpp(0, v, B == 0 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int B> __device__ __forceinline__ double lane_xchg(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xchg<B>((int)b);
  const int hi = lane_xchg<B>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int B> __device__ __forceinline__ float lane_xchg(float v) {
  return __int_as_float(lane_xchg<B>(__float_as_int(v)));
}

// One radix-2 level over lanes q and q ^ 2^B for sub-transforms of length
// NB: lanes with bit B set multiply e[k] by w_NB^(lo M + k), lo being bit LO
// of q (LO < 0: lo = 0), before (decimation in time) or after (decimation
// in frequency) the join, where the bit-clear lane takes own + partner's and
// the other partner's - own.  Twiddles come from the table tw[m] = w_N^m;
// the other lanes read its entry 0 (= 1).
template <typename V, int N, int M, int B, int NB, int LO, bool INV>
__device__ __forceinline__ void level_twiddle(V *e, int q, const V *tw) {
  constexpr int ST = N / NB;
  const bool hi = (q >> B) & 1;
  const int lo = LO >= 0 ? (q >> (LO < 0 ? 0 : LO)) & 1 : 0;
  const V *t = tw + (hi ? lo * M * ST : 0);
  const int step = hi ? ST : 0;
#pragma unroll
  for (int k = (LO < 0 ? 1 : 0); k < M; ++k) {
    const V w = t[k * step];
    e[k] = INV ? c_mulconj(e[k], w) : c_mul(e[k], w);
  }
}
template <typename V, int M, int B>
__device__ __forceinline__ void level_join(V *e, int q) {
  using S = decltype(e[0].x);
  const S sg = ((q >> B) & 1) ? S(-1) : S(1);  // partner's + sg * own
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const V o{lane_xchg<B>(e[k].x), lane_xchg<B>(e[k].y)};
    e[k] = V{fma(sg, e[k].x, o.x), fma(sg, e[k].y, o.y)};
  }
}

// rev reverses the log2(L) bits of a lane index
template <int L> __device__ __forceinline__ int rev_lane(int q) {
  if constexpr (L == 8) return ((q & 1) << 2) | (q & 2) | (q >> 2);
  return L == 4 ? ((q & 1) << 1) | (q >> 1) : q;
}

// The last level of eight lanes: lanes with bit 0 set multiply e[k] by
// w_N^((2 b1 + b2) M + k), b1 and b2 the lane's bits 1 and 2 (after the
// first two levels the lane holds entry (2 b1 + b2) M + k of the transforms
// of length 4M that this level joins).
template <typename V, int N, int M, bool INV>
__device__ __forceinline__ void level_twiddle8(V *e, int q, const V *tw) {
  const bool hi = q & 1;
  const int lo = 2 * ((q >> 1) & 1) + ((q >> 2) & 1);
  const V *t = tw + (hi ? lo * M : 0);
  const int step = hi ? 1 : 0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const V w = t[k * step];
    e[k] = INV ? c_mulconj(e[k], w) : c_mul(e[k], w);
  }
}

// decimation in time: lane q holds x[L j + q] and ends with
// X[rev(q) M + k].  With four lanes, lanes q and q ^ 2 hold the even and
// odd halves of one stride-2 subsequence, so bit 1 is joined first.
template <typename V, int L, int N, bool INV>
__device__ __forceinline__ void group_fft_dit(V *e, int q, const V *tw) {
  constexpr int M = N / L;
  reg_fft<V, M, INV, 0>(e, tw);
  if constexpr (L == 8) {
    // lanes q and q ^ 4 hold the even and odd halves of a stride-4
    // subsequence, then q and q ^ 2 two stride-4 halves of a stride-2 one;
    // lane q ends with X[rev(q) M + k], rev reversing its three bits
    level_twiddle<V, N, M, 2, 2 * M, -1, INV>(e, q, tw);
    level_join<V, M, 2>(e, q);
    level_twiddle<V, N, M, 1, 4 * M, 2, INV>(e, q, tw);
    level_join<V, M, 1>(e, q);
    level_twiddle8<V, N, M, INV>(e, q, tw);
    level_join<V, M, 0>(e, q);
  } else if constexpr (L == 4) {
    level_twiddle<V, N, M, 1, 2 * M, -1, INV>(e, q, tw);
    level_join<V, M, 1>(e, q);
    level_twiddle<V, N, M, 0, 4 * M, 1, INV>(e, q, tw);
    level_join<V, M, 0>(e, q);
  } else {
    level_twiddle<V, N, M, 0, 2 * M, -1, INV>(e, q, tw);
    level_join<V, M, 0>(e, q);
  }
}
// decimation in frequency: lane q holds x[rev(q) M + j] (the layout the
// decimation-in-time transform leaves) and ends with X[L k + q]
template <typename V, int L, int N, bool INV>
__device__ __forceinline__ void group_fft_dif(V *e, int q, const V *tw) {
  constexpr int M = N / L;
  if constexpr (L == 8) {
    level_join<V, M, 0>(e, q);
    level_twiddle8<V, N, M, INV>(e, q, tw);
    level_join<V, M, 1>(e, q);
    level_twiddle<V, N, M, 1, 4 * M, 2, INV>(e, q, tw);
    level_join<V, M, 2>(e, q);
    level_twiddle<V, N, M, 2, 2 * M, -1, INV>(e, q, tw);
  } else if constexpr (L == 4) {
    level_join<V, M, 0>(e, q);
    level_twiddle<V, N, M, 0, 4 * M, 1, INV>(e, q, tw);
    level_join<V, M, 1>(e, q);
    level_twiddle<V, N, M, 1, 2 * M, -1, INV>(e, q, tw);
  } else {
    level_join<V, M, 0>(e, q);
    level_twiddle<V, N, M, 0, 2 * M, -1, INV>(e, q, tw);
  }
  reg_fft<V, M, INV, 0>(e, tw);
}

// Exchange of halves (M = N / 4 even).  The four lanes of a line are
// l + 16 q (q = 0..3), so the two lane levels pair lanes 16 apart (rows of a
// wave, v_permlane16_swap) and 32 apart (halves of a wave,
// v_permlane32_swap).  One such move swaps a register x of one lane with a
// register y of its partner: afterwards the lane with the bit clear holds
// (x, x of the partner) and the partner (y of the first lane, y).  Applied to
// the element pairs (e[k], e[k + M/2]) it leaves in each lane the two inputs
// of M/2 radix-2 butterflies, so a level costs each lane M/2 twiddle
// products and half the exchange traffic of a join over all M values.
template <int B> __device__ __forceinline__ void row_swap(unsigned &x, unsigned &y) {
  if constexpr (B == 0) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}
template <int B> __device__ __forceinline__ void row_swap(double &x, double &y) {
  const unsigned long long a = __double_as_longlong(x), b = __double_as_longlong(y);
  unsigned al = (unsigned)a, ah = (unsigned)(a >> 32), bl = (unsigned)b, bh = (unsigned)(b >> 32);
  row_swap<B>(al, bl);
  row_swap<B>(ah, bh);
  x = __longlong_as_double((long long)(((unsigned long long)ah << 32) | al));
  y = __longlong_as_double((long long)(((unsigned long long)bh << 32) | bl));
}
template <int B> __device__ __forceinline__ void row_swap(float &x, float &y) {
  unsigned a = __float_as_uint(x), b = __float_as_uint(y);
  row_swap<B>(a, b);
  x = __uint_as_float(a);
  y = __uint_as_float(b);
}
template <int B, typename V> __device__ __forceinline__ void row_swap_c(V &x, V &y) {
  row_swap<B>(x.x, y.x);
  row_swap<B>(x.y, y.y);
}

// One lane level by exchange of halves over lane bit 4 + B, twiddles
// t[ST k] (conjugated for INV), k < M/2.  Decimation in time: swap, then
// (X, Y) <- (X + t Y, X - t Y); decimation in frequency: (X, Y) <-
// (X + Y, (X - Y) t), then swap.
template <typename V, int M, int B, int ST, bool INV, bool DIT>
__device__ __forceinline__ void level_halves(V *e, const V *t) {
  constexpr int H = M / 2;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    V x = e[k], y = e[k + H];
    const V w = t[ST * k];
    if constexpr (DIT) {
      row_swap_c<B>(x, y);
      const V u = INV ? c_mulconj(y, w) : c_mul(y, w);
      e[k] = c_add(x, u);
      e[k + H] = c_sub(x, u);
    } else {
      const V d = c_sub(x, y);
      x = c_add(x, y);
      y = INV ? c_mulconj(d, w) : c_mul(d, w);
      row_swap_c<B>(x, y);
      e[k] = x;
      e[k + H] = y;
    }
  }
}

// Lane q of a line holds, between the two transforms, X[c_q + k] in e[k] and
// X[c_q + 2M + k] in e[k + M/2] (k < M/2), c_q = (q >> 1) M/2 + (q & 1) M.
template <int M> __device__ __forceinline__ int halves_base(int q) { return (q >> 1) * (M / 2) + (q & 1) * M; }
template <int M> constexpr int halves_off(int k) { return k < M / 2 ? k : k + 3 * (M / 2); }

// decimation in time: lane q holds x[4 j + q], ends in the layout above
template <typename V, int N, bool INV>
__device__ __forceinline__ void group_fft_dit_h(V *e, int q, const V *tw) {
  constexpr int M = N / 4;
  reg_fft<V, M, INV, 0>(e, tw);
  level_halves<V, M, 1, 2, INV, true>(e, tw + (q >> 1) * M);
  level_halves<V, M, 0, 1, INV, true>(e, tw + halves_base<M>(q));
}
// decimation in frequency: from the layout above to X[4 k + q]
template <typename V, int N, bool INV>
__device__ __forceinline__ void group_fft_dif_h(V *e, int q, const V *tw) {
  constexpr int M = N / 4;
  level_halves<V, M, 0, 1, INV, false>(e, tw + halves_base<M>(q));
  level_halves<V, M, 1, 2, INV, false>(e, tw + (q >> 1) * M);
  reg_fft<V, M, INV, 0>(e, tw);
}

// hides the values from the optimiser: twiddle reads and lane-dependent
// twiddle addresses derived from them stay inside the loop body that uses
// them instead of being hoisted and held in registers across the loop
__device__ __forceinline__ void opaque(int &a, int &b) { asm volatile("" : "+v"(a), "+v"(b)); }


// Plane pass with register FFTs.  LDS holds the twiddle table w_N^m, only
// the nx columns that carry sticks, compact [slot][y] with slot stride
// LS = N | 1 (odd, so that lanes reading down different columns are free of
// bank conflicts), one column kept zero for the x without sticks, and the
// x -> slot table.
// Per band-plane: clear, scatter the sticks, inverse y transform of each
// column, then per row the inverse x transform, the V(r) product and the
// forward x transform back to back, forward y transform of each column,
// gather.  Every line is held by a group of L lanes: L consecutive lanes
// joined by quad permutations, or with XH (L = 4, N / 4 even) lanes
// l + 16 q joined by exchange of halves.  Cubic grids of compile-time size
// N (a multiple of L) only.  Workgroups of four waves
// and a register budget of three (FP64) or four (FP32) waves per SIMD let
// two or more workgroups share a CU and hide each other's latencies.
template <typename T, int N, int L, int NTHR, bool XH>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4)))
void k_plane_r(FFTDev f, cpx_t<T> *__restrict__ sticks, int nb, int group) {
  using V = cpx_t<T>;
  static_assert(N % L == 0 && NTHR % (4 * L) == 0, "lane-group plane pass: whole lane groups");
  static_assert(!XH || (L == 4 && (N / 4) % 2 == 0 && NTHR % 64 == 0), "exchange of halves: L = 4, N / 4 even");
  constexpr int M = N / L, LS = N | 1, NL = NTHR / L;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = f.nx;
  const int nel = (nx + 1) * LS;
  V *tw = reinterpret_cast<V *>(smem);
  V *pl = tw + N;
  int *xs = reinterpret_cast<int *>(pl + nel);
  const int z = blockIdx.x % N;
  const int g = blockIdx.x / N;
  const int tid = threadIdx.x;
  const int line = XH ? (tid >> 6) * 16 + (tid & 15) : tid / L;
  const int q = XH ? (tid >> 4) & 3 : tid % L;
  // first x of the lane's run between the transforms (XH: c_q, else rev(q) M)
  const int xq = XH ? halves_base<M>(q) : rev_lane<L>(q) * M;
  for (int i = tid; i < N; i += NTHR) {
    xs[i] = f.xslot[i];
    tw[i] = static_cast<const V *>(f.tw0)[i];
  }
  const T *vp = static_cast<const T *>(f.vplanes) + (int64_t)z * N * N;
  for (int bb = 0; bb < group; ++bb) {
    const int b = g * group + bb;
    if (b >= nb) break;
    for (int i = tid; i < nel; i += NTHR) pl[i] = V{0, 0};
    __syncthreads();
    V *col = sticks + (int64_t)b * N * f.nst_pad + (int64_t)z * f.nst_pad;
    for (int s = tid; s < f.nst; s += NTHR) pl[f.stick_cpos[s]] = col[s];
    __syncthreads();
    for (int c = line; c < nx; c += NL) {
      V e[M];
      V *p = pl + c * LS;
      int zero = 0, qo = q;
      opaque(zero, qo);
#pragma unroll
      for (int j = 0; j < M; ++j) e[j] = p[L * j + q];
      if constexpr (XH)
        group_fft_dit_h<V, N, true>(e, qo, tw + zero);
      else
        group_fft_dit<V, L, N, true>(e, qo, tw + zero);
#pragma unroll
      for (int k = 0; k < M; ++k) p[xq + (XH ? halves_off<M>(k) : k)] = e[k];
    }
    __syncthreads();
    for (int y = line; y < N; y += NL) {
      V e[M];
      int zero = 0, qo = q;
      opaque(zero, qo);
#pragma unroll
      for (int j = 0; j < M; ++j) e[j] = pl[xs[L * j + q] * LS + y];
      if constexpr (XH)
        group_fft_dit_h<V, N, true>(e, qo, tw + zero);
      else
        group_fft_dit<V, L, N, true>(e, qo, tw + zero);
      // V and the output slots are read only now (their offsets are opaque
      // past the transform), not held in registers across it
      int vo = xq * N + y, xo = q;
      opaque(vo, xo);
      const T *vr = vp + vo;
#pragma unroll
      for (int k = 0; k < M; ++k) e[k] = c_scale(e[k], vr[(XH ? halves_off<M>(k) : k) * N]);
      if constexpr (XH)
        group_fft_dif_h<V, N, false>(e, qo, tw + zero);
      else
        group_fft_dif<V, L, N, false>(e, qo, tw + zero);
      opaque(xo, zero);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int sl = xs[L * k + xo];
        if (sl < nx) pl[sl * LS + y] = e[k];
      }
    }
    __syncthreads();
    for (int c = line; c < nx; c += NL) {
      V e[M];
      V *p = pl + c * LS;
      int zero = 0, qo = q;
      opaque(zero, qo);
#pragma unroll
      for (int j = 0; j < M; ++j) e[j] = p[xq + (XH ? halves_off<M>(j) : j)];
      if constexpr (XH)
        group_fft_dif_h<V, N, false>(e, qo, tw + zero);
      else
        group_fft_dif<V, L, N, false>(e, qo, tw + zero);
#pragma unroll
      for (int k = 0; k < M; ++k) p[L * k + q] = e[k];
    }
    __syncthreads();
    for (int s = tid; s < f.nst; s += NTHR) col[s] = pl[f.stick_cpos[s]];
    __syncthreads();
  }
}

// Plane pass with register FFTs and direct stick I/O, pipelined over the
// bands of the group.  Same line layout as k_plane_r with exchange of halves
// (four lanes l + 16 q per line, N / 4 even), but the stick values never
// pass through an LDS scatter or gather: the inverse y transform of a column
// reads its sticks straight from the stick buffer (the (slot, y) -> stick
// table sits in LDS; positions without a stick read zero) and the forward y
// transform writes its outputs straight back.  A column is owned by the same
// lane group in both y transforms, so the forward transform of band b and
// the inverse transform of band b + 1 share one phase: the group reads the
// column of band b into registers before it writes the column of band b + 1
// over it, and the LDS operations of one wave execute in issue order.  Per
// band: two barriers (after the y phase, after the row phase) instead of
// six.  LDS: twiddles, the compact plane with one zero column, x -> slot,
// and the (slot, y) table.
template <typename T, int N, int NTHR>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4)))
void k_plane_p(FFTDev f, cpx_t<T> *__restrict__ sticks, int nb, int group) {
  using V = cpx_t<T>;
  constexpr int L = 4, M = N / L, LS = N | 1, NL = NTHR / L;
  static_assert(N % 4 == 0 && M % 2 == 0 && NTHR % 64 == 0, "exchange of halves: N / 4 even, whole waves");
  // rows left over after one pass of NL lines that fit one wave as groups of
  // eight lanes (N = 72 with 256 threads) take the eight-lane transform
  constexpr bool TAIL8 = N > NL && N < 2 * NL && N % 8 == 0 && 8 * (N - NL) <= 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = f.nx;
  V *tw = reinterpret_cast<V *>(smem);
  V *pl = tw + N;
  int *xs = reinterpret_cast<int *>(pl + (nx + 1) * LS);
  int16_t *cy = reinterpret_cast<int16_t *>(xs + N);
  const int z = blockIdx.x % N;
  const int g = blockIdx.x / N;
  const int tid = threadIdx.x;
  const int line = (tid >> 6) * 16 + (tid & 15);
  const int q = (tid >> 4) & 3;
  const int xq = halves_base<M>(q);
  const int b0 = g * group;
  const int b1 = min(b0 + group, nb);
  for (int i = tid; i < N; i += NTHR) {
    xs[i] = f.xslot[i];
    tw[i] = static_cast<const V *>(f.tw0)[i];
    pl[nx * LS + i] = V{0, 0};
  }
  for (int i = tid; i < nx * N; i += NTHR) cy[i] = f.stick_cy[i];
  __syncthreads();
  const T *vp = static_cast<const T *>(f.vplanes) + (int64_t)z * N * N;
  const int64_t bstride = (int64_t)N * f.nst_pad;
  V *colz = sticks + (int64_t)z * f.nst_pad;

  // inverse y transform of column c of band b: sticks -> LDS column
  auto col_inv = [&](int b, int c) {
    const V *src = colz + (int64_t)b * bstride;
    const int16_t *cyc = cy + c * N;
    V e[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int s = cyc[L * j + q];
      e[j] = s >= 0 ? src[s] : V{0, 0};
    }
    int zero = 0, qo = q;
    opaque(zero, qo);
    group_fft_dit_h<V, N, true>(e, qo, tw + zero);
    V *p = pl + c * LS;
#pragma unroll
    for (int k = 0; k < M; ++k) p[xq + halves_off<M>(k)] = e[k];
  };

  if (b0 < b1)
    for (int c = line; c < nx; c += NL) col_inv(b0, c);
  __syncthreads();
  for (int b = b0; b < b1; ++b) {
    for (int y = line; y < (TAIL8 ? NL : N); y += NL) {
      V e[M];
      int zero = 0, qo = q;
      opaque(zero, qo);
#pragma unroll
      for (int j = 0; j < M; ++j) e[j] = pl[xs[L * j + q] * LS + y];
      group_fft_dit_h<V, N, true>(e, qo, tw + zero);
      int vo = xq * N + y, xo = q;
      opaque(vo, xo);
      const T *vr = vp + vo;
#pragma unroll
      for (int k = 0; k < M; ++k) e[k] = c_scale(e[k], vr[halves_off<M>(k) * N]);
      group_fft_dif_h<V, N, false>(e, qo, tw + zero);
      opaque(xo, zero);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int sl = xs[L * k + xo];
        if (sl < nx) pl[sl * LS + y] = e[k];
      }
    }
    if constexpr (TAIL8) {
      // the rows past the first NL: eight lanes (tid & 7) of the first wave
      // per row, each with N / 8 values, instead of four lanes with N / 4
      if (tid < 8 * (N - NL)) {
        constexpr int M8 = N / 8;
        const int y = NL + (tid >> 3), q8 = tid & 7;
        V e[M8];
        int zero = 0, qo = q8;
        opaque(zero, qo);
#pragma unroll
        for (int j = 0; j < M8; ++j) e[j] = pl[xs[8 * j + q8] * LS + y];
        group_fft_dit<V, 8, N, true>(e, qo, tw + zero);
        int vo = rev_lane<8>(q8) * M8 * N + y, xo = q8;
        opaque(vo, xo);
        const T *vr = vp + vo;
#pragma unroll
        for (int k = 0; k < M8; ++k) e[k] = c_scale(e[k], vr[k * N]);
        group_fft_dif<V, 8, N, false>(e, qo, tw + zero);
        opaque(xo, zero);
#pragma unroll
        for (int k = 0; k < M8; ++k) {
          const int sl = xs[8 * k + xo];
          if (sl < nx) pl[sl * LS + y] = e[k];
        }
      }
    }
    __syncthreads();
    const bool next = b + 1 < b1;
    V *dst = colz + (int64_t)b * bstride;
    for (int c = line; c < nx; c += NL) {
      {
        V e[M];
        const V *p = pl + c * LS;
        int zero = 0, qo = q;
        opaque(zero, qo);
#pragma unroll
        for (int j = 0; j < M; ++j) e[j] = p[xq + halves_off<M>(j)];
        group_fft_dif_h<V, N, false>(e, qo, tw + zero);
        const int16_t *cyc = cy + c * N;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const int s = cyc[L * k + q];
          if (s >= 0) dst[s] = e[k];
        }
      }
      // every lane of the group has read the column of band b before any
      // lane writes band b + 1 over it
      wave_sync();
      if (next) col_inv(b + 1, c);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- full-grid transforms
// One pass of a 3D transform of a complex FP64 grid [N0][N1][N2] (N2
// fastest) along one axis, scaled by `scale` on the way out.  AXIS 2: a
// workgroup takes T consecutive z-lines.  AXIS 0 / 1: a workgroup takes the
// N lines along the axis at one y (AXIS 0) or one x (AXIS 1) and T
// consecutive z, so that its global loads and stores run along z.  The host
// keeps T * N within kCpt values per thread.  blockIdx.y picks one of a
// batch of grids `stride` elements apart.
template <int AXIS, bool INV, int NTHR>
__global__ __launch_bounds__(NTHR) void k_grid_axis(FFTDev f, double2 *__restrict__ g0, int64_t stride, int T,
                                                    double scale) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2 *__restrict__ g = g0 + (int64_t)blockIdx.y * stride;
  const AxisPlan &pl = AXIS == 0 ? f.px : (AXIS == 1 ? f.py : f.pz);
  const int N = pl.n;
  double2 *tw = reinterpret_cast<double2 *>(smem);
  double2 *buf = tw + N;
  const double2 *twg = static_cast<const double2 *>(AXIS == 0 ? f.tw0 : (AXIS == 1 ? f.tw1 : f.tw2));
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTHR) tw[i] = twg[i];
  const int n1 = f.n1, n2 = f.n2;
  if constexpr (AXIS == 2) {
    const int64_t l0 = (int64_t)blockIdx.x * T;
    const int nl = (int)min<int64_t>(T, (int64_t)f.n0 * n1 - l0);
    double2 *src = g + l0 * n2;
    for (int i = tid; i < nl * n2; i += NTHR) buf[i] = src[i];
    __syncthreads();
    fft_axis<double2, INV, false, false, 0>(buf, nl, n2, 1, nullptr, pl, tw, tid, NTHR);
    for (int i = tid; i < nl * n2; i += NTHR) src[i] = c_scale(buf[i], scale);
  } else {
    const int nzt = (n2 + T - 1) / T;
    const int o = blockIdx.x / nzt;
    const int z0 = (blockIdx.x - o * nzt) * T;
    const int nl = min(T, n2 - z0);
    const float inl = 1.0f / (float)nl;
    // element (a, t): position a along the axis, t in the z tile
    auto at = [&](int a, int t) -> int64_t {
      return AXIS == 0 ? ((int64_t)a * n1 + o) * n2 + z0 + t : ((int64_t)o * n1 + a) * n2 + z0 + t;
    };
    for (int i = tid; i < N * nl; i += NTHR) {
      const int a = qdiv(i, nl, inl);
      buf[i] = g[at(a, i - a * nl)];
    }
    __syncthreads();
    fft_axis<double2, INV, true, false, 0>(buf, nl, 1, nl, nullptr, pl, tw, tid, NTHR);
    for (int i = tid; i < N * nl; i += NTHR) {
      const int a = qdiv(i, nl, inl);
      g[at(a, i - a * nl)] = c_scale(buf[i], scale);
    }
  }
}

// Band density on one z-plane: per band of the workgroup's group, scatter
// the plane's sticks into an LDS plane [x][y], inverse y transform of the x
// rows that hold sticks, inverse x transform of every y column, then add
// w_b |u_b(r)|^2 into the workgroup's own partial plane part[g][z][x][y]
// (each element is owned by one thread across all bands, so no atomics and
// a fixed order of summation).
template <int NTHR>
__global__ __launch_bounds__(NTHR) void k_rho_plane(FFTDev f, const double2 *__restrict__ sticks, int nb,
                                                    int group, const double *__restrict__ w,
                                                    double *__restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2 *tw0 = reinterpret_cast<double2 *>(smem);
  double2 *tw1 = tw0 + f.n0;
  double2 *pl = tw1 + f.n1;
  int *lb = reinterpret_cast<int *>(pl + f.n0 * f.n1);
  const int z = blockIdx.x % f.n2;
  const int g = blockIdx.x / f.n2;
  const int tid = threadIdx.x;
  const double2 *tw0g = static_cast<const double2 *>(f.tw0);
  const double2 *tw1g = static_cast<const double2 *>(f.tw1);
  for (int i = tid; i < f.n0; i += NTHR) tw0[i] = tw0g[i];
  for (int i = tid; i < f.n1; i += NTHR) tw1[i] = tw1g[i];
  for (int i = tid; i < f.nx; i += NTHR) lb[i] = f.xlist[i] * f.n1;
  const int npl = f.n0 * f.n1;
  double *acc = part + ((int64_t)g * f.n2 + z) * npl;
  for (int bb = 0; bb < group; ++bb) {
    const int b = g * group + bb;
    if (b >= nb) break;
    for (int i = tid; i < npl; i += NTHR) pl[i] = double2{0, 0};
    __syncthreads();
    const double2 *col = sticks + (int64_t)b * f.n2 * f.nst_pad + (int64_t)z * f.nst_pad;
    for (int s = tid; s < f.nst; s += NTHR) pl[f.stick_xy[s]] = col[s];
    __syncthreads();
    fft_axis<double2, true, false, true, 0>(pl, f.nx, 0, 1, lb, f.py, tw1, tid, NTHR);
    fft_axis<double2, true, true, false, 0>(pl, f.n1, 1, f.n1, nullptr, f.px, tw0, tid, NTHR);
    const double wb = w[b];
    for (int i = tid; i < npl; i += NTHR) acc[i] += wb * (pl[i].x * pl[i].x + pl[i].y * pl[i].y);
    __syncthreads();
  }
}

template <typename T, int NTHR, int NC>
__global__ __launch_bounds__(NTHR) void k_zfft_fwd(FFTDev f, const cpx_t<T> *__restrict__ sticks,
                                                   const double2 *__restrict__ psi, int64_t ld,
                                                   double2 *__restrict__ hpsi, int64_t ldh, int nb,
                                                   int kinetic) {
  using V = cpx_t<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  V *tw = reinterpret_cast<V *>(smem);
  V *buf = tw + f.n2;
  int tile, b;
  tile_band(blockIdx.x, f.ntile, &tile, &b);
  if (b >= nb) return;
  const int tid = threadIdx.x;
  const V *twg = static_cast<const V *>(f.tw2);
  for (int i = tid; i < f.n2; i += NTHR) tw[i] = twg[i];
  const int nel = f.ts * f.n2;
  const V *srcs = sticks + (int64_t)b * f.n2 * f.nst_pad + (int64_t)tile * f.ts;
  for (int i = tid; i < nel; i += NTHR) {
    const int z = i / f.ts;
    const int sl = i - z * f.ts;
    buf[i] = srcs[(int64_t)z * f.nst_pad + sl];
  }
  __syncthreads();
  fft_axis<V, false, true, false, NC>(buf, f.ts, 1, f.ts, nullptr, f.pz, tw, tid, NTHR);
  const int e0 = f.tile_ptr[tile], e1 = f.tile_ptr[tile + 1];
  const double2 *src = psi + (int64_t)b * ld;
  double2 *dst = hpsi + (int64_t)b * ldh;
  for (int e = e0 + tid; e < e1; e += NTHR) {
    const int gi = f.g_linear ? e : f.gidx[e];
    const V v = buf[f.gpos[e]];
    double2 o = double2{(double)v.x, (double)v.y};
    if (kinetic) {
      const double2 p = src[gi];
      const double t = f.kin[gi];
      o.x += t * p.x;
      o.y += t * p.y;
    }
    dst[gi] = o;
  }
}

__global__ void k_kinetic_only(const double *__restrict__ kin, const double2 *__restrict__ psi,
                               int64_t ld, double2 *__restrict__ hpsi, int64_t ldh, int64_t npw,
                               int kinetic) {
  const int b = blockIdx.y;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < npw;
       g += (int64_t)gridDim.x * blockDim.x) {
    double2 o = double2{0.0, 0.0};
    if (kinetic) {
      const double2 p = psi[(int64_t)b * ld + g];
      o = double2{kin[g] * p.x, kin[g] * p.y};
    }
    hpsi[(int64_t)b * ldh + g] = o;
  }
}

// ---------------------------------------------------------------- host side
bool make_axis_plan(int n, AxisPlan *out) {
  AxisPlan p;
  p.n = n;
  int m = n, a = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++a;
  }
  auto push = [&](int r) {
    if (p.npass >= kMaxPasses) return false;
    p.radix[p.npass++] = r;
    return true;
  };
  while (a > 0) {
    bool ok;
    if (a == 4) {
      ok = push(4) && push(4);
      a = 0;
    } else if (a >= 3) {
      ok = push(8);
      a -= 3;
    } else if (a == 2) {
      ok = push(4);
      a -= 2;
    } else {
      ok = push(2);
      a -= 1;
    }
    if (!ok) return false;
  }
  while (m % 3 == 0) {
    if (!push(3)) return false;
    m /= 3;
  }
  while (m % 5 == 0) {
    if (!push(5)) return false;
    m /= 5;
  }
  if (m != 1) return false;
  *out = p;
  return true;
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static inline int nb_pad8(int nb) { return (nb + 7) / 8 * 8; }

// cubic grids of the workloads run compile-time-planned kernels
#define PW_CT_SIZES(X) X(24) X(36) X(40) X(45) X(48) X(50) X(54) X(60) X(64) X(72) X(81) X(90)
// the register plane pass needs an even length (a line is shared by a lane pair)
#define PW_CT_EVEN_SIZES(X) X(24) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(90)

static int ct_size(const FFTDev &f, int prec) {
  static const bool off = env_switch("PW_FFT_GENERIC", 0) != 0;
  if (off || f.n0 != f.n1 || f.n1 != f.n2) return 0;
  if (f.ts != (prec == PW_FP64 ? 16 : 32)) return 0;
  switch (f.n0) {
#define PW_CASE(n) case n: return n;
    PW_CT_SIZES(PW_CASE)
#undef PW_CASE
    default: return 0;
  }
}

template <typename T, int NT, int NC>
static int zinv_n(const FFTDev &f, const void *psi, int64_t ld, void *sticks, int nb, hipStream_t s) {
  using V = cpx_t<T>;
  const size_t lds = sizeof(V) * (size_t)f.n2 * (1 + f.ts);
  const int blocks = f.ntile * nb_pad8(nb);
  auto k = k_zfft_inv<T, NT, NC>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<const double2 *>(psi), ld,
                     static_cast<V *>(sticks), nb);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}
template <typename T, int NC>
static int zinv_c(const FFTDev &f, const void *psi, int64_t ld, void *sticks, int nb, hipStream_t s) {
  return f.ts * f.n2 <= kCpt * 256 ? zinv_n<T, 256, NC>(f, psi, ld, sticks, nb, s)
                                   : zinv_n<T, 512, NC>(f, psi, ld, sticks, nb, s);
}
template <typename T>
static int zinv_t(const FFTDev &f, const void *psi, int64_t ld, void *sticks, int nb, hipStream_t s) {
  switch (ct_size(f, sizeof(T) == 8 ? PW_FP64 : PW_MIXED_FP32)) {
#define PW_CASE(n) case n: return zinv_c<T, n>(f, psi, ld, sticks, nb, s);
    PW_CT_SIZES(PW_CASE)
#undef PW_CASE
    default: return zinv_c<T, 0>(f, psi, ld, sticks, nb, s);
  }
}

// Plane kernels: PW_PLANE_REGISTER (register FFTs where the grid has an
// even compile-time size, else the LDS Stockham pass), PW_PLANE_WAVE
// (wave-local lines), PW_PLANE_LDS (LDS Stockham passes).  A problem
// starts with PW_PLANE_IMPL from the environment, else PW_PLANE_REGISTER.
int plane_kernel_default() {
  static const int v = [] {
    const int x = env_switch("PW_PLANE_IMPL", PW_PLANE_REGISTER);
    return (x < PW_PLANE_REGISTER || x > PW_PLANE_LDS) ? PW_PLANE_REGISTER : x;
  }();
  return v;
}

// lanes per line: four where N allows (register pressure), else two.  With
// four lanes and N / 4 even the lane levels exchange halves; PW_PLANE_HALVES=0
// keeps the quad-permutation joins.
static bool plane_halves() {
  static const int v = env_switch("PW_PLANE_HALVES", 1);
  return v != 0;
}
#ifndef PW_PLANE_R_THREADS
#define PW_PLANE_R_THREADS 256
#endif
// the pipelined direct-I/O form of the exchange-of-halves kernel;
// PW_PLANE_PIPE=0 keeps the scatter / gather form
static bool plane_pipe() {
  static const int v = env_switch("PW_PLANE_PIPE", 1);
  return v != 0;
}
template <typename T, int N>
static int plane_r(const FFTDev &f, void *sticks, int nb, int group, int blocks, hipStream_t s) {
  using V = cpx_t<T>;
  constexpr int L = (N % 4 == 0) ? 4 : 2;
  constexpr int NT = PW_PLANE_R_THREADS;
  constexpr bool xh_ok = L == 4 && (N / 4) % 2 == 0;
  if constexpr (xh_ok) {
    if (plane_halves() && plane_pipe() && f.stick_cy) {
      const size_t lds = sizeof(V) * ((size_t)(f.nx + 1) * (N | 1) + N) + sizeof(int) * N +
                         sizeof(int16_t) * (size_t)f.nx * N;
      auto k = k_plane_p<T, N, NT>;
      if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
      hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<V *>(sticks), nb, group);
      return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
    }
  }
  const size_t lds = sizeof(V) * ((size_t)(f.nx + 1) * (N | 1) + N) + sizeof(int) * N;
  auto k = (xh_ok && plane_halves()) ? k_plane_r<T, N, L, NT, xh_ok> : k_plane_r<T, N, L, NT, false>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<V *>(sticks), nb, group);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

template <typename T, int NT>
static int plane_w_n(const FFTDev &f, void *sticks, int nb, int group, size_t lds, int blocks,
                     hipStream_t s) {
  using V = cpx_t<T>;
  auto k = k_plane_w<T, NT>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<V *>(sticks), nb, group);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

template <typename T, int NT, int NC>
static int plane_n(const FFTDev &f, void *sticks, int nb, int group, size_t lds, int blocks,
                   hipStream_t s) {
  using V = cpx_t<T>;
  auto k = k_plane<T, NT, NC>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<V *>(sticks), nb, group);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}
template <typename T, int NC>
static int plane_c(const FFTDev &f, void *sticks, int nb, int group, size_t lds, int blocks,
                   hipStream_t s) {
  const int npl = f.n0 * f.n1;
  if (npl <= kCpt * 256) return plane_n<T, 256, NC>(f, sticks, nb, group, lds, blocks, s);
  if (npl <= kCpt * 512) return plane_n<T, 512, NC>(f, sticks, nb, group, lds, blocks, s);
  return plane_n<T, 1024, NC>(f, sticks, nb, group, lds, blocks, s);
}

bool plane_register_ok(const FFTDev &f, int prec) {
  switch (ct_size(f, prec)) {
#define PW_CASE(n) case n: return true;
    PW_CT_EVEN_SIZES(PW_CASE)
#undef PW_CASE
    default: return false;
  }
}

int plane_default_group(const FFTDev &f, int prec, int kernel) {
  return (kernel == PW_PLANE_REGISTER && plane_register_ok(f, prec)) ? 2 : 8;
}

template <typename T>
static int plane_t(const FFTDev &f, void *sticks, int nb, int group, int kernel, hipStream_t s) {
  using V = cpx_t<T>;
  const int npl = f.n0 * f.n1;
  const size_t lds = sizeof(V) * (size_t)(f.n0 + f.n1 + npl) + sizeof(int) * (size_t)f.nx;
  const int groups = (nb + group - 1) / group;
  const int blocks = f.n2 * groups;
  if (kernel == PW_PLANE_WAVE) {
    if (npl <= 2048) return plane_w_n<T, 256>(f, sticks, nb, group, lds, blocks, s);
    if (npl <= 4096) return plane_w_n<T, 512>(f, sticks, nb, group, lds, blocks, s);
    return plane_w_n<T, 1024>(f, sticks, nb, group, lds, blocks, s);
  }
  if (kernel == PW_PLANE_REGISTER) {
    switch (ct_size(f, sizeof(T) == 8 ? PW_FP64 : PW_MIXED_FP32)) {
#define PW_CASE(n) case n: return plane_r<T, n>(f, sticks, nb, group, blocks, s);
      PW_CT_EVEN_SIZES(PW_CASE)
#undef PW_CASE
      default: break;
    }
  }
  switch (ct_size(f, sizeof(T) == 8 ? PW_FP64 : PW_MIXED_FP32)) {
#define PW_CASE(n) case n: return plane_c<T, n>(f, sticks, nb, group, lds, blocks, s);
    PW_CT_SIZES(PW_CASE)
#undef PW_CASE
    default: return plane_c<T, 0>(f, sticks, nb, group, lds, blocks, s);
  }
}

template <typename T, int NT, int NC>
static int zfwd_n(const FFTDev &f, const void *sticks, const void *psi, int64_t ld, void *hpsi,
                  int64_t ldh, int nb, bool kinetic, hipStream_t s) {
  using V = cpx_t<T>;
  const size_t lds = sizeof(V) * (size_t)f.n2 * (1 + f.ts);
  const int blocks = f.ntile * nb_pad8(nb);
  auto k = k_zfft_fwd<T, NT, NC>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(NT), lds, s, f, static_cast<const V *>(sticks),
                     static_cast<const double2 *>(psi), ld, static_cast<double2 *>(hpsi), ldh, nb,
                     kinetic ? 1 : 0);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}
template <typename T, int NC>
static int zfwd_c(const FFTDev &f, const void *sticks, const void *psi, int64_t ld, void *hpsi,
                  int64_t ldh, int nb, bool kinetic, hipStream_t s) {
  return f.ts * f.n2 <= kCpt * 256
             ? zfwd_n<T, 256, NC>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s)
             : zfwd_n<T, 512, NC>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s);
}
template <typename T>
static int zfwd_t(const FFTDev &f, const void *sticks, const void *psi, int64_t ld, void *hpsi,
                  int64_t ldh, int nb, bool kinetic, hipStream_t s) {
  switch (ct_size(f, sizeof(T) == 8 ? PW_FP64 : PW_MIXED_FP32)) {
#define PW_CASE(n) case n: return zfwd_c<T, n>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s);
    PW_CT_SIZES(PW_CASE)
#undef PW_CASE
    default: return zfwd_c<T, 0>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s);
  }
}

int launch_zfft_inv(const FFTDev &f, int prec, const void *psi, int64_t ld, void *sticks, int nb,
                    hipStream_t s) {
  if (nb <= 0) return PW_OK;
  return prec == PW_FP64 ? zinv_t<double>(f, psi, ld, sticks, nb, s)
                         : zinv_t<float>(f, psi, ld, sticks, nb, s);
}

int launch_plane(const FFTDev &f, int prec, void *sticks, int nb, int group, int kernel,
                 hipStream_t s) {
  if (nb <= 0) return PW_OK;
  return prec == PW_FP64 ? plane_t<double>(f, sticks, nb, group, kernel, s)
                         : plane_t<float>(f, sticks, nb, group, kernel, s);
}

int launch_zfft_fwd(const FFTDev &f, int prec, const void *sticks, const void *psi, int64_t ld,
                    void *hpsi, int64_t ldh, int nb, bool kinetic, hipStream_t s) {
  if (nb <= 0) return PW_OK;
  return prec == PW_FP64 ? zfwd_t<double>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s)
                         : zfwd_t<float>(f, sticks, psi, ld, hpsi, ldh, nb, kinetic, s);
}

// Full-grid 3D transforms of nbatch grids [N0][N1][N2] (FP64 complex),
// `stride` elements apart: inverse unnormalised, forward with N^-3 (split as
// 1/N per axis).
int launch_grid_fft(const FFTDev &f, double2 *g, int nbatch, int64_t stride, bool inverse, hipStream_t s) {
  if (nbatch <= 0) return PW_OK;
  constexpr int NT = 256;
  const int n[3] = {f.n0, f.n1, f.n2};
  for (int ax = 2; ax >= 0; --ax) {
    const int N = n[ax];
    const int T = std::max(1, std::min(16, kCpt * NT / N));
    const double scale = inverse ? 1.0 : 1.0 / (double)N;
    const size_t lds = sizeof(double2) * (size_t)N * (1 + T);
    int64_t blocks;
    if (ax == 2)
      blocks = ((int64_t)f.n0 * f.n1 + T - 1) / T;
    else
      blocks = (int64_t)(ax == 0 ? f.n1 : f.n0) * ((f.n2 + T - 1) / T);
    auto pick = [&](auto k) -> int {
      if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
      hipLaunchKernelGGL(k, dim3((unsigned)blocks, (unsigned)nbatch), dim3(NT), lds, s, f, g, stride, T, scale);
      return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
    };
    int rc;
    if (ax == 2)
      rc = inverse ? pick(k_grid_axis<2, true, NT>) : pick(k_grid_axis<2, false, NT>);
    else if (ax == 1)
      rc = inverse ? pick(k_grid_axis<1, true, NT>) : pick(k_grid_axis<1, false, NT>);
    else
      rc = inverse ? pick(k_grid_axis<0, true, NT>) : pick(k_grid_axis<0, false, NT>);
    if (rc != PW_OK) return rc;
  }
  return PW_OK;
}

// Band densities of nb bands whose z transforms sit in the stick buffer:
// part[g][z][x][y] += sum over the bands b of group g of w[b] |u_b|^2.
template <int NT>
static int rho_plane_n(const FFTDev &f, const void *sticks, int nb, int group, const double *w, double *part,
                       hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(f.n0 + f.n1 + f.n0 * f.n1) + sizeof(int) * (size_t)f.nx;
  const int groups = (nb + group - 1) / group;
  auto k = k_rho_plane<NT>;
  if (allow_lds(k, lds) != hipSuccess) return PW_ERR_HIP;
  hipLaunchKernelGGL(k, dim3((unsigned)(f.n2 * groups)), dim3(NT), lds, s, f,
                     static_cast<const double2 *>(sticks), nb, group, w, part);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}
int launch_rho_plane(const FFTDev &f, const void *sticks, int nb, int group, const double *w, double *part,
                     hipStream_t s) {
  if (nb <= 0) return PW_OK;
  // the LDS transforms hold at most kCpt values per thread of a plane
  const int npl = f.n0 * f.n1;
  if (npl <= kCpt * 256) return rho_plane_n<256>(f, sticks, nb, group, w, part, s);
  if (npl <= kCpt * 512) return rho_plane_n<512>(f, sticks, nb, group, w, part, s);
  if (npl <= kCpt * 1024) return rho_plane_n<1024>(f, sticks, nb, group, w, part, s);
  return PW_ERR_SHAPE;
}

int launch_kinetic_only(const double *kin, const void *psi, int64_t ld, void *hpsi, int64_t ldh,
                        int64_t npw, int nb, bool kinetic, hipStream_t s) {
  if (nb <= 0) return PW_OK;
  int bx = (int)((npw + 255) / 256);
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_kinetic_only, dim3(bx, nb), dim3(256), 0, s, kin,
                     static_cast<const double2 *>(psi), ld, static_cast<double2 *>(hpsi), ldh, npw,
                     kinetic ? 1 : 0);
  return hipGetLastError() == hipSuccess ? PW_OK : PW_ERR_HIP;
}

}  // namespace pw
