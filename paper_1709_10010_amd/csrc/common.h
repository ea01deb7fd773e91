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

// Integer value of an environment switch (dflt when unset or empty).  The
// library reads each switch once per process, into a function-local static
// whose initialisation C++ makes thread-safe.
int env_switch(const char *name, int dflt);

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

// ----------------------------------------------------------------- workspace
// Hands out 256-byte aligned pieces of a caller's workspace in order.  With
// a null base it only counts: the same sequence of take() calls then gives
// the workspace size a later call with the real base needs.
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += (n > 0 ? n : 1) * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~(size_t)255; }
};

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
  // stick index of each (slot, y) of the compact plane, -1 where there is
  // none: [nx][N1], kept when every index fits 16 bits (else empty)
  std::vector<int16_t> stick_cy;
  std::vector<int32_t> gfull;     // [npw] full-grid index (x N1 + y) N2 + z of each G, caller's order
};

// Device-side view passed to the FFT launchers.
struct FFTDev {
  int n0, n1, n2;
  int nst, ts, ntile, nst_pad, nx;
  AxisPlan px, py, pz;
  const int32_t *gidx, *gpos, *tile_ptr, *stick_xy, *xlist;
  int g_linear;  // gidx is the identity (the z passes then read and write G in order)
  const int32_t *xslot, *stick_cpos;  // compact plane layout (see StickMap)
  const int16_t *stick_cy;            // [nx][N1] stick of (slot, y) or -1; null if unavailable
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
  // small device tables owned by the handle (maps, twiddles, kinetic
  // energies, D blocks and their offsets)
  int32_t *d_gidx = nullptr, *d_gpos = nullptr, *d_tile_ptr = nullptr;
  int32_t *d_stick_xy = nullptr, *d_xlist = nullptr;
  int32_t *d_xslot = nullptr, *d_stick_cpos = nullptr;
  int16_t *d_stick_cy = nullptr;
  int32_t *d_gfull = nullptr;
  double *d_kin = nullptr;
  void *d_tw = nullptr;        // three twiddle tables back to back
  double *d_dij = nullptr;     // concatenated blocks
  int32_t *d_pj_atom = nullptr;  // [nproj] atom of each projector
  int32_t *d_proj_off = nullptr; // [natom+1]
  int32_t *d_dij_off = nullptr;  // [natom] offset of the atom's block in d_dij
  // the caller's workspace (pw_workspace_size bytes), bound to the handle
  // for its lifetime; everything below points into it
  void *ws = nullptr;
  size_t ws_bytes = 0;
  void *d_vplanes = nullptr;   // [N2][N0][N1] V / N^3 in the FFT precision
  void *d_beta = nullptr;      // complex128 [nproj][ldb]
  void *d_beta_lp = nullptr;   // reduced-precision copy (mixed forms)
  int64_t ldb = 0;
  void *d_sticks = nullptr;    // [band_chunk][N2][nst_pad] complex (FFT precision)
  void *d_P = nullptr;         // [max_bands][nproj] complex128
  void *d_Q = nullptr;         // [max_bands][nproj] complex128
  void *d_psi_lp = nullptr;    // BF16 form: psi rounded to bf16 pairs [max_bands][ldb]
  void *d_q_lp = nullptr;      // BF16 form: D P rounded to bf16 pairs [max_bands][nproj]
  void *d_part = nullptr;      // split-K partial sums
  size_t part_bytes = 0;
  double *d_tn = nullptr;      // [max_bands] band kinetic energies (preconditioner)
  double *d_rnorm = nullptr;   // [max_bands] residual norms (pw_precond with the MLP kind)
  int *d_idx = nullptr;        // [max_bands] band indices 0 .. n-1 (same)
  int *d_bad = nullptr;        // [max_bands] per-band fallback flags (same)
  // overlap S = 1 + sum q |beta><beta| when the caller gives augmentation
  // (overlap.hip): S^{-1/2} = 1 + K diag(sfac) K^H
  bool gen = false;
  double *d_qij = nullptr;     // concatenated q blocks (the layout of d_dij)
  double2 *d_K = nullptr;      // [nproj][ldb]
  double *d_sfac = nullptr;    // [nproj]
  double2 *d_ov_qb = nullptr;  // set-up scratch: Q_b [nproj][ldb]
  double2 *d_ov_mat = nullptr; // set-up scratch: 5 nproj^2 complex
  void *d_ov_eig = nullptr;    // set-up scratch: eigensolver workspace
  int *d_ov_flag = nullptr;
  // exact exchange attached by pw_ace_set: H psi gains -alpha zeta zeta^H psi
  // (caller-owned buffers, bound until pw_ace_clear or destroy)
  const double2 *ace_zeta = nullptr;  // [nocc][ldz]
  int64_t ace_ldz = 0, ace_nocc = 0;
  double ace_alpha = 0.0;
  double2 *ace_proj = nullptr;        // [max_bands][nocc] scratch of the H psi term
  // or the exchange operator itself (pw_vx_attach): H psi gains
  // alpha V_x psi by pair densities, nocc pair transforms per band, over the
  // caller's occupied states with host weights and the caller's scratch
  const double2 *exx_occ = nullptr;  // [nocc][exx_ldo]
  int64_t exx_ldo = 0, exx_nocc = 0;
  double exx_alpha = 0.0;
  std::vector<double> exx_w;
  void *exx_work = nullptr;
  // the SCF loop whose workspace holds the attached buffers (null when the
  // caller attached them): told when the problem goes first
  pw_scf *ace_owner = nullptr;
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
// full-grid 3D transform of a complex FP64 grid [N0][N1][N2] in place
// (inverse unnormalised, forward with N^-3), and the band-density plane pass
// (part[group][z][x][y] += w_b |u_b|^2 for the bands in the stick buffer);
// nbatch grids `stride` elements apart
int launch_grid_fft(const FFTDev &f, double2 *g, int nbatch, int64_t stride, bool inverse, hipStream_t s);
int launch_rho_plane(const FFTDev &f, const void *sticks, int nb, int group, const double *w, double *part,
                     hipStream_t s);

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
// float2 or bf16 pairs), B complex128 (bf16 pairs in the BF16 form, made by
// bf16_round), C complex128, accumulation FP64 / FP32 / FP32.
int zgemm_cn_p(int prec, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda, const void *B,
               int64_t ldb, void *C, int64_t ldc, int splits, void *part, hipStream_t s);
int zgemm_nn_p(int prec, int64_t M, int64_t N, int64_t K, double alpha, const void *A, int64_t lda,
               const void *B, int64_t ldb, double beta, void *C, int64_t ldc, hipStream_t s);
int convert_beta(const void *src, void *dst, int64_t n, int prec, hipStream_t s);
// dst[c][r] = src[c][r] rounded to bf16 pairs (nearest even), r < rows, c < cols
int bf16_round(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t rows, int64_t cols, hipStream_t s);

// Nonlocal D application (nonlocal.hip): Q[n][j] = sum_j' D_a(j,j') P[n][j'].
int launch_apply_d(const double *dij, const int32_t *pj_atom, const int32_t *proj_off,
                   const int32_t *dij_off, const void *P, void *Q, int64_t nproj, int nb,
                   hipStream_t s);
// Diagonal preconditioner (nonlocal.hip): t = K r, K per PW_PRECOND_TPA / _NONE.
int launch_tpa(const double *kin, const void *x, const void *r, void *t, int64_t ld, int64_t npw,
               int nb, int kind, double *tn_work, hipStream_t s);
// Bands per plane-pass workgroup that suits a plane kernel on the grid (fft.hip).
int plane_default_group(const FFTDev &f, int prec, int kernel);
// Hermitian eigensolver behind pw_eigh (linalg.hip) on a workspace of
// eigh_ws_bytes(m): the padded matrix, the pair unitaries and the
// eigenvectors (3 mp^2 complex, mp = m rounded up to kEighPad), the
// eigenvalues, the sweep accumulators and the sort permutation.  Every
// region is written before it is read, so earlier contents do not matter.
constexpr int kEighPad = 32;
constexpr int kEighMaxSweeps = 40;
constexpr size_t eigh_ws_bytes(int m) {
  return 3 * (size_t)((m + kEighPad - 1) / kEighPad * kEighPad) * ((m + kEighPad - 1) / kEighPad * kEighPad) *
             sizeof(double2) +
         ((size_t)((m + kEighPad - 1) / kEighPad * kEighPad) + 2 * kEighMaxSweeps + 2) * sizeof(double) +
         (size_t)((m + kEighPad - 1) / kEighPad * kEighPad) * sizeof(int);
}
int eigh_impl(const void *A, int64_t lda, int m, double *w, void *Z, int64_t ldz, void *work, hipStream_t s);
// 2-norms of n columns (linalg.hip).
int col_norms(const double2 *T, int64_t ld, int64_t npw, int n, double *nrm, hipStream_t s);
// Learned preconditioner of the bands idx[0..nu) (mlp.hip): T_i = s K_TPA R_idx[i];
// bad[i] is set for a band whose scales are not finite, and mlp_fallback
// then writes TPA for every flagged band.
int mlp_precond_idx(const pw_mlp *net, pw_problem *p, const double *theta, const double *rnorm,
                    const int *idx, const double2 *R, int64_t ld, double2 *T, int nu, int *bad,
                    const double *tn, hipStream_t s);
int mlp_fallback(const int *bad, pw_problem *p, const double *tn, const int *idx, const double2 *R,
                 int64_t ld, double2 *T, int nu, hipStream_t s);
// Overlap transform (overlap.hip): workspace regions, set-up from the
// concatenated q blocks and the atoms' projector offsets, and
// y = S^{-1/2} x for nb bands.
void carve_overlap(pw_problem *p, Carve &c);
int overlap_setup(pw_problem *p, const std::vector<double> &qblocks, const std::vector<int32_t> &poff,
                  hipStream_t s);
int sinvhalf(pw_problem *p, const void *x, int64_t ldx, void *y, int64_t ldy, int64_t nb, hipStream_t s);
// Exact-exchange term of H psi (exx.hip): hpsi -= alpha zeta (zeta^H psi).
int ace_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi, int64_t ld_hpsi, int64_t nbands,
             hipStream_t s);
// Build ACE from nocc occupied states (weights w, host) and attach alpha
// V_ace (exx.hip); e_xx (may be null) receives sum_i w_i <psi_i|V_x psi_i>.
// work: ace_build_bytes(p, nocc) bytes, 256-byte aligned.
int ace_build(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w, double alpha,
              void *zeta, int64_t ldz, void *proj, void *work, double *e_xx, hipStream_t s);
size_t ace_build_bytes(const pw_problem *p, int64_t nocc);
// The exchange operator applied directly (exx.hip): hpsi += alpha V_x psi.
int exx_direct_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi, int64_t ld_hpsi, int64_t nbands,
                    hipStream_t s);
// Copy nocc occupied states into occ (ldo) and attach alpha V_x, applied
// directly, to the problem; e_xx as for ace_build.  work: ace_build_bytes(p,
// nocc) bytes (its head is the direct operator's scratch afterwards).
int exx_direct_build(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                     double alpha, void *occ, int64_t ldo, void *work, double *e_xx, hipStream_t s);
// an SCF loop's attached problem is being destroyed before the loop
void scf_forget_problem(pw_scf *s, const pw_problem *p);
// Davidson state accessors for the batch scheduler (davidson.hip).
pw_problem *dav_problem(const pw_davidson *d);
int dav_nbands(const pw_davidson *d);
int dav_max_subspace(const pw_davidson *d);
bool dav_converged(const pw_davidson *d);
bool dav_inited(const pw_davidson *d);
// tn[n] = <x_n|t|x_n> / <x_n|x_n> for nb bands (nonlocal.hip).
int band_kinetic(const double *kin, const void *x, int64_t ld, int64_t npw, int nb, double *tn,
                 hipStream_t s);
}  // namespace pw
