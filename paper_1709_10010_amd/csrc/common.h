// Internal declarations shared by the HIP sources of libpwhip.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pw_api.h"

namespace pw {

// ----------------------------------------------------------------- errors
void set_error(const std::string &msg);

#define PW_CHECK_ARG(cond, code, msg)            \
  do {                                           \
    if (!(cond)) {                               \
      ::pw::set_error(msg);                      \
      return (code);                             \
    }                                            \
  } while (0)

#define PW_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::pw::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
      return PW_ERR_HIP;                                                    \
    }                                                                       \
  } while (0)

// ----------------------------------------------------------------- complex
template <typename T> struct cpx;
template <> struct cpx<double> { using type = double2; };
template <> struct cpx<float> { using type = float2; };
template <typename T> using cpx_t = typename cpx<T>::type;

// ----------------------------------------------------------------- FFT plans
constexpr int kMaxPasses = 8;
struct AxisPlan {
  int n = 0;
  int npass = 0;
  int radix[kMaxPasses] = {0};
};
bool make_axis_plan(int n, AxisPlan *out);

// Stick/plane layout of one problem's sphere on its grid.
struct StickMap {
  int nst = 0;        // number of z-sticks (distinct (h mod N0, k mod N1))
  int ts = 16;        // sticks per z-pass tile
  int ntile = 0;
  int nst_pad = 0;    // ntile * ts
  int nx = 0;         // distinct x rows holding sticks
  std::vector<int32_t> gidx;     // [npw] caller G index, grouped by tile
  bool g_linear = false;         // gidx[e] == e: the caller lists G by stick, then z
  std::vector<int32_t> gpos;     // [npw] z * ts + (stick - tile*ts)
  std::vector<int32_t> tile_ptr; // [ntile+1]
  std::vector<int32_t> stick_xy; // [nst] x * N1 + y
  std::vector<int32_t> xlist;    // [nx] rows holding sticks
  // compact plane layout of the register plane pass: x -> slot (0..nx-1,
  // nx for an x without sticks, a column kept zero) and each stick's
  // position slot * ls + y, with slot stride ls = N1 | 1
  int ls = 0;
  std::vector<int32_t> xslot;      // [N0]
  std::vector<int32_t> stick_cpos; // [nst]
};

// Device-side view passed to the FFT launchers.
struct FFTDev {
  int n0, n1, n2;
  int nst, ts, ntile, nst_pad, nx;
  AxisPlan px, py, pz;
  const int32_t *gidx, *gpos, *tile_ptr, *stick_xy, *xlist;
  int g_linear;  // gidx is the identity (the z passes then read and write G in order)
  const int32_t *xslot, *stick_cpos;  // compact plane layout (see StickMap)
  const void *tw0, *tw1, *tw2;  // twiddle tables in the FFT precision
  const void *vplanes;          // [N2][N0][N1] V / (N0 N1 N2) in the FFT precision
  const double *kin;            // [npw]
};

}  // namespace pw

// ----------------------------------------------------------------- profiling
namespace pw {
struct Prof {
  bool on = false;
  struct Pend {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pend> pending;
  std::vector<hipEvent_t> pool;
  double ms[PW_NSTAGES] = {0};
  int64_t cnt[PW_NSTAGES] = {0};
  hipEvent_t get();
  void begin(int stage, hipStream_t s, Pend *out);
  void end(const Pend &p, hipStream_t s);
  int drain();
  void release();
};
// RAII bracket: records the start event now and the stop event at scope end.
struct ProfScope {
  Prof *p;
  hipStream_t s;
  Prof::Pend e;
  ProfScope(Prof *pp, int stage, hipStream_t st) : p(pp && pp->on ? pp : nullptr), s(st) {
    if (p) p->begin(stage, s, &e);
  }
  ~ProfScope() {
    if (p) p->end(e, s);
  }
};
}  // namespace pw

// ----------------------------------------------------------------- handles
struct pw_problem {
  pw::Prof prof;
  int device = 0;
  int precision = PW_FP64;
  double A[9], B[9], kpt[3], ecut;
  int nr[3];
  int64_t npw = 0, nproj = 0, max_bands = 0;
  int natom = 0;
  double vavg = 0;          // mean of V_LOC over the grid (a feature of the learned preconditioner)
  int64_t band_chunk = 0;   // bands per FFT sweep (stick-buffer height)
  int64_t band_chunk_max = 0;  // sweep height the stick buffer was sized for
  int plane_group = 8;      // bands per plane-pass workgroup
  int plane_kernel = 0;     // PW_PLANE_REGISTER / _WAVE / _LDS
  int ksplit = 0;           // split-K factor for projections (0 = auto)
  pw::StickMap map;
  pw::FFTDev fft{};
  // device buffers owned by the handle
  int32_t *d_gidx = nullptr, *d_gpos = nullptr, *d_tile_ptr = nullptr;
  int32_t *d_stick_xy = nullptr, *d_xlist = nullptr;
  int32_t *d_xslot = nullptr, *d_stick_cpos = nullptr;
  double *d_kin = nullptr;
  void *d_tw = nullptr;        // three twiddle tables back to back
  void *d_vplanes = nullptr;
  void *d_beta = nullptr;      // complex128 [nproj][ldb]
  void *d_beta_lp = nullptr;   // reduced-precision copy (mixed forms)
  int64_t ldb = 0;
  double *d_dij = nullptr;     // concatenated blocks
  int32_t *d_pj_atom = nullptr;  // [nproj] atom of each projector
  int32_t *d_proj_off = nullptr; // [natom+1]
  int32_t *d_dij_off = nullptr;  // [natom] offset of the atom's block in d_dij
  void *d_sticks = nullptr;    // [band_chunk][N2][nst_pad] complex (FFT precision)
  void *d_P = nullptr;         // [max_bands][nproj] complex128
  void *d_Q = nullptr;         // [max_bands][nproj] complex128
  void *d_part = nullptr;      // split-K partial sums
  size_t part_bytes = 0;
  double *d_tn = nullptr;      // [max_bands] band kinetic energies (preconditioner)
};

namespace pw {
// FFT launchers (fft.hip)
int launch_zfft_inv(const FFTDev &f, int prec, const void *psi, int64_t ld, void *sticks,
                    int nb, hipStream_t s);
int launch_plane(const FFTDev &f, int prec, void *sticks, int nb, int group, int kernel,
                 hipStream_t s);
// plane kernel a new problem starts with, and whether the register plane
// kernel has an instance for the grid (fft.hip)
int plane_kernel_default();
bool plane_register_ok(const FFTDev &f, int prec);
int launch_zfft_fwd(const FFTDev &f, int prec, const void *sticks, const void *psi, int64_t ld,
                    void *hpsi, int64_t ldh, int nb, bool kinetic, hipStream_t s);
int launch_kinetic_only(const double *kin, const void *psi, int64_t ld, void *hpsi, int64_t ldh,
                        int64_t npw, int nb, bool kinetic, hipStream_t s);

// Complex GEMMs (gemm.hip).  Column-major complex128 matrices.
// C[MxN] = A^H B,  A: K x M (lda), B: K x N (ldb); split-K over `splits`
// partial buffers summed in a fixed order.  part must hold splits*M*N complex.
int zgemm_cn(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
             int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s);
// C[MxN] = alpha A B + beta C,  A: M x K (lda), B: K x N (ldb).
int zgemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
             const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s);
int choose_splits(int64_t M, int64_t N, int64_t K);
// Same shapes in a precision form: A in the form's storage (complex128,
// float2 or bf16 pairs), B and C complex128, accumulation FP64 / FP32 / FP32.
int zgemm_cn_p(int prec, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
               int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s);
int zgemm_nn_p(int prec, int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
               const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s);
int convert_beta(const void *src, void *dst, int64_t n, int prec, hipStream_t s);

// Nonlocal D application (nonlocal.hip): Q[n][j] = sum_j' D_a(j,j') P[n][j'].
int launch_apply_d(const double *dij, const int32_t *pj_atom, const int32_t *proj_off,
                   const int32_t *dij_off, const void *P, void *Q, int64_t nproj, int nb,
                   hipStream_t s);
// Diagonal preconditioner (nonlocal.hip): t = K r, K per PW_PRECOND_TPA / _NONE.
int launch_tpa(const double *kin, const void *x, const void *r, void *t, int64_t ld, int64_t npw,
               int nb, int kind, double *tn_work, hipStream_t s);
// Bands per plane-pass workgroup that suits a plane kernel on the grid (fft.hip).
int plane_default_group(const FFTDev &f, int prec, int kernel);
// tn[n] = <x_n|t|x_n> / <x_n|x_n> for nb bands (nonlocal.hip).
int band_kinetic(const double *kin, const void *x, int64_t ld, int64_t npw, int nb, double *tn,
                 hipStream_t s);
}  // namespace pw
