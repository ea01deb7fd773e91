// Block Davidson driver (host side of the C ABI; all arithmetic in kernels).
//
// One iteration, in the order of the block Davidson method (Davidson 1975,
// which the paper cites for its Davidson-like solver; subspace
// diagonalisation as in PWscf's iterative diagonalisation):
//   1. Hermitian eigensolve of the subspace matrix H_s = V^H H V (FP64);
//   2. Ritz vectors X = V Y, HX = W Y (W = H V kept alongside V);
//   3. residuals R = HX - X theta and their norms -> host (the one sync);
//   4. if not converged: preconditioned corrections for the unconverged
//      bands (soft locking), restart V = X, W = HX, H_s = diag(theta) when
//      the space is full, classical Gram-Schmidt + Cholesky-QR against
//      the space, a second round for the columns the first leaves short of
//      orthonormal (rank-revealing fallback through an eigendecomposition
//      when Cholesky breaks down), H on the new vectors, and the bordered
//      subspace matrix.
// Everything runs in FP64 on the GPU; the problem's precision form only
// changes how H is applied.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "common.h"

namespace pw {
int eig_herm(double2 *A, int64_t lda, int m, double *w, double2 *Z, int64_t ldz, void *rot_ws,
             double *acc_ws, double *h_acc, int *sweeps, hipStream_t s, double off_abs, int nwant);
int eig_select(const double *w, int m, int nsel, double *wsel, int *idx, const double2 *Z, int64_t ldz,
               double2 *Y, int64_t ldy, hipStream_t s, const double2 *A, int64_t lda, double2 *H,
               int64_t ldh);
int cholesky(const double2 *S, int64_t lds, int n, double2 *L, int64_t ldl, double rel, int *flag,
             hipStream_t s);
int trinv_h(const double2 *L, int64_t ldl, int n, double2 *X, int64_t ldx, double2 *B, int64_t ldb,
            hipStream_t s);
int residual(const double2 *X, const double2 *HX, const double *theta, double2 *R, int64_t ld,
             int64_t npw, int nb, double *rho, double *xn2, hipStream_t s);
int hermitize(double2 *H, int64_t ldh, int m0, int m1, hipStream_t s);
int copy_mat(const double2 *src, int64_t lds, double2 *dst, int64_t ldd, int m, int n, hipStream_t s);
int scaled_cols(const double2 *U, int64_t ldu, const double *lam, const int *keep, int n, int nk,
                double2 *B, int64_t ldb, hipStream_t s);
int precond_idx(const double *kin, const double *tn, const int *idx, const double2 *R, int64_t ldr,
                double2 *T, int64_t ldt, int64_t npw, int nu, int kind, hipStream_t s);
int col_norms2(const double2 *T, int64_t ld, int64_t npw, int n, double *nrm2, hipStream_t s);
int gather_cols(const double2 *Z, int64_t ldz, const int *idx, int64_t m, int nsel, double2 *Y, int64_t ldy,
                hipStream_t s);
}  // namespace pw

using namespace pw;

struct pw_davidson {
  pw_problem *p = nullptr;
  int nb = 0, mmax = 0, lde = 0;
  double tol = 0;
  int64_t ld = 0, npw = 0;
  int m = 0, iter = 0;
  int64_t n_hpsi = 0;
  bool inited = false, converged = false;
  // the last step found every correction numerically inside the space
  bool stalled = false;
  double2 *V = nullptr, *W = nullptr, *R = nullptr, *T = nullptr;
  // the Ritz vectors: the first nb columns of V (the rotation puts them
  // there, and nothing writes them until the next step's rotation)
  double2 *X = nullptr;
  double2 *Vt = nullptr, *Wt = nullptr;  // rotation targets (swapped with V, W each step)
  double *w_sorted = nullptr;
  int *idx_all = nullptr;
  double2 *Hs = nullptr, *Ae = nullptr, *Ze = nullptr, *Y = nullptr, *C = nullptr;
  double2 *S = nullptr, *L = nullptr, *Xi = nullptr, *Bi = nullptr;
  double *w_all = nullptr, *theta = nullptr, *rho = nullptr, *tn = nullptr, *lam = nullptr;
  double *xn2 = nullptr;  // squared norms of the Ritz vectors
  int *idx_sel = nullptr, *dU = nullptr, *keep = nullptr, *flag = nullptr, *sweeps = nullptr;
  int *bad = nullptr;
  void *rot_ws = nullptr;
  double *acc_ws = nullptr;
  void *part = nullptr;
  size_t part_bytes = 0;
  // the caller's workspace (pw_davidson_workspace_size bytes); every device
  // buffer above points into it
  void *ws = nullptr;
  double2 *U1 = nullptr, *U2 = nullptr;  // [nb][ld] each: S^{-1/2} x and H S^{-1/2} x (augmented problems)
  // pinned host mirrors
  double *h_theta = nullptr, *h_rho = nullptr, *h_lam = nullptr, *h_xn2 = nullptr;
  double *h_acc = nullptr;  // eigensolver's off-diagonal and total mass, read once per sweep
  int *h_U = nullptr, *h_flag = nullptr, *h_keep = nullptr;
  // orthonormalisation: column norms^2 before it, the Cholesky diagonal
  double *cnorm = nullptr, *h_cnorm = nullptr;
  double2 *h_ldiag = nullptr;
  // learned-preconditioner fallback: residual of the previous step and the
  // number of consecutive non-decreasing steps, per band; bands that stall
  // for two steps use TPA for the rest of the solve
  std::vector<double> prev_rho;
  std::vector<int> stall;
  std::vector<uint8_t> tpa_only;
  int *h_bad = nullptr;
  double off_target = 0.0;  // eigensolver stop level (Frobenius norm of the off-diagonal part)
  // the space's loss of orthonormality as the Ritz vectors see it,
  // max_n | |x_n|^2 - 1 |, measured every step; raised within a step by the
  // columns taken with one orthonormalisation round
  double ortho_err = 0.0;
  // the most a column taken with one round may carry: a tenth of the
  // tolerance over the largest |Ritz value| (the residual floor that loss of
  // orthonormality sets), at most 1e-9; 0 (two rounds for all) at init
  double skip_err = 0.0;
  // locked prefix: bands 0 .. nl-1 have converged (all of them), their
  // vectors stay fixed in V and W, and Rayleigh-Ritz runs on the rest
  int nl = 0;
};

namespace {

// the device buffers live in the caller's workspace; only the small pinned
// host mirrors belong to the handle
void free_dav(pw_davidson *d) {
  if (!d) return;
  void *host[] = {d->h_theta, d->h_rho, d->h_xn2, d->h_lam, d->h_U, d->h_flag, d->h_keep, d->h_bad, d->h_cnorm,
                  d->h_ldiag, d->h_acc};
  for (void *b : host)
    if (b) (void)hipHostFree(b);
  delete d;
}

// Workspace layout of a Davidson state: counted by pw_davidson_workspace_size
// with a null base, placed by pw_davidson_create with the caller's.
void carve_dav(pw_davidson *d, Carve &c) {
  const size_t blk = (size_t)d->ld, nb = d->nb, lde = d->lde;
  d->V = c.take<double2>(lde * blk);
  d->W = c.take<double2>(lde * blk);
  d->Vt = c.take<double2>(lde * blk);
  d->Wt = c.take<double2>(lde * blk);
  d->R = c.take<double2>(nb * blk);
  d->T = c.take<double2>(nb * blk);
  d->Hs = c.take<double2>(lde * lde);
  d->Ae = c.take<double2>(lde * lde);
  d->Ze = c.take<double2>(lde * lde);
  d->rot_ws = c.take<double2>(lde * lde);
  d->Y = c.take<double2>(lde * nb);
  d->C = c.take<double2>(lde * nb);
  d->S = c.take<double2>(nb * nb);
  d->L = c.take<double2>(nb * nb);
  d->Xi = c.take<double2>(nb * nb);
  d->Bi = c.take<double2>(nb * nb);
  d->w_sorted = c.take<double>(lde);
  d->idx_all = c.take<int>(lde);
  d->w_all = c.take<double>(lde);
  d->lam = c.take<double>(lde);
  d->theta = c.take<double>(nb);
  d->rho = c.take<double>(nb);
  d->xn2 = c.take<double>(nb);
  d->tn = c.take<double>(nb);
  d->cnorm = c.take<double>(nb);
  d->idx_sel = c.take<int>(nb);
  d->dU = c.take<int>(nb);
  d->keep = c.take<int>(nb);
  d->bad = c.take<int>(nb);
  d->flag = c.take<int>(1);
  d->sweeps = c.take<int>(1);
  d->acc_ws = c.take<double>(128);
  d->part_bytes = (size_t)32 * lde * nb * sizeof(double2);
  d->part = c.take<char>(d->part_bytes);
  if (d->p->gen) {
    d->U1 = c.take<double2>(nb * blk);
    d->U2 = c.take<double2>(nb * blk);
  }
}

// The operator the state iterates with on n columns: H, or for an augmented
// problem S^{-1/2} H S^{-1/2} (n <= nb).
int dav_apply(pw_davidson *d, const double2 *src, double2 *dst, int n, hipStream_t s) {
  pw_problem *p = d->p;
  if (!p->gen) return pw_hpsi(p, src, d->ld, dst, d->ld, n, PW_TERM_ALL, s);
  int rc = sinvhalf(p, src, d->ld, d->U1, d->ld, n, s);
  if (rc == PW_OK) rc = pw_hpsi(p, d->U1, d->ld, d->U2, d->ld, n, PW_TERM_ALL, s);
  if (rc == PW_OK) rc = sinvhalf(p, d->U2, d->ld, dst, d->ld, n, s);
  return rc;
}

// sizes of a Davidson state from its arguments (shared by the size query and create)
int dav_shape(pw_problem *p, int64_t nbands, int64_t *max_subspace, double tol, const char *who) {
  auto msg = [&](const char *m) { return std::string(who) + ": " + m; };
  PW_CHECK_ARG(nbands >= 1 && nbands <= p->max_bands && nbands <= p->npw, PW_ERR_INVALID,
               msg("nbands must be in 1 .. min(max_bands, npw)"));
  if (*max_subspace == 0) *max_subspace = 3 * nbands;
  PW_CHECK_ARG(*max_subspace >= 2 * nbands && *max_subspace <= p->npw && *max_subspace <= 8192, PW_ERR_INVALID,
               msg("max_subspace must be in 2*nbands .. min(npw, 8192)"));
  PW_CHECK_ARG(tol > 0 && std::isfinite(tol), PW_ERR_INVALID, msg("tol must be > 0"));
  return PW_OK;
}

void dav_dims(pw_davidson *d, pw_problem *p, int64_t nbands, int64_t max_subspace) {
  d->p = p;
  d->nb = (int)nbands;
  d->mmax = (int)max_subspace;
  d->lde = (d->mmax + 31) / 32 * 32;  // room for the block eigensolver's padding
  d->npw = p->npw;
  d->ld = (p->npw + 63) / 64 * 64;
}

template <typename T>
bool halloc(T **p, size_t n) {
  return hipHostMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault) == hipSuccess;
}

int cn(pw_davidson *d, int64_t M, int64_t N, const double2 *A, const double2 *B, double2 *Cm,
       int64_t ldc, hipStream_t s) {
  ProfScope ps(&d->p->prof, PW_STAGE_SUBGEMM, s);
  int splits = choose_splits(M, N, d->npw);
  while (splits > 1 && (size_t)splits * M * N * 16 > d->part_bytes) --splits;
  return zgemm_cn(M, N, d->npw, A, d->ld, B, d->ld, Cm, ldc, splits, d->part, s);
}

int nn(pw_davidson *d, int64_t N, int64_t K, double alpha, const double2 *A, const double2 *B,
       int64_t ldb, double beta, double2 *Cm, hipStream_t s) {
  ProfScope ps(&d->p->prof, PW_STAGE_UPDGEMM, s);
  return zgemm_nn(d->npw, N, K, alpha, A, d->ld, B, ldb, beta, Cm, d->ld, s);
}

#define DV_RC(x)              \
  do {                        \
    const int rc_ = (x);      \
    if (rc_ != PW_OK) {       \
      if (set_error_if_empty) \
        set_error(where);     \
      return rc_;             \
    }                         \
  } while (0)

// PW_DAV_ORTHO_SKIP=0 runs the second orthonormalisation round on every column.
static bool ortho_skip() {
  static const int v = env_switch("PW_DAV_ORTHO_SKIP", 1);
  return v != 0;
}

// Gram-Schmidt passes against V in the first orthonormalisation round
// (PW_DAV_GS_FIRST, 1 or 2; default 1).
static int gs_first() {
  static const int v = env_switch("PW_DAV_GS_FIRST", 1) == 2 ? 2 : 1;
  return v;
}

// A column whose squared norm after the projection against the space (and
// the block's earlier columns) is at most kDrop0 of its squared norm before
// it lies numerically in the space: what is left of it is rounding and the
// space's own loss of orthogonality, and normalising that would put a
// direction already in the space into it a second time, so it is dropped.
// The second round starts from orthonormal columns; one that loses half of
// its squared norm there had such a direction amplified by the first round
// and is dropped too.
constexpr double kDrop0 = 1e-16;
constexpr double kDrop1 = 0.5;
constexpr double kEps = 2.220446049250313e-16;

// Cholesky-QR of the n columns at *src into *out (the compaction below may
// swap the two buffers; on return the result is in *out).  Columns that kept
// too little through the projection are dropped first; a block dependent in
// itself goes to the rank-revealing path.  In round 0 the result is ordered
// head first: the *nh columns a second round would change by less than
// d->skip_err (they are taken as they are), then the rest.
int cholqr(pw_davidson *d, int round, double2 **src, double2 **out, int *n, int *nh, hipStream_t s) {
  const bool set_error_if_empty = true;
  const char *where = "pw_davidson: orthonormalisation failed";
  *nh = 0;
  while (*n > 0) {
    const int nc = *n;
    DV_RC(cn(d, nc, nc, *src, *src, d->S, nc, s));
    {
      ProfScope ps(&d->p->prof, PW_STAGE_CHOL, s);
      DV_RC(cholesky(d->S, nc, nc, d->L, nc, 1e-12, d->flag, s));
    }
    PW_HIP(hipMemcpyAsync(d->h_flag, d->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PW_HIP(hipMemcpy2DAsync(d->h_ldiag, sizeof(double2), d->L, (size_t)(nc + 1) * sizeof(double2),
                            sizeof(double2), nc, hipMemcpyDeviceToHost, s));
    PW_HIP(hipStreamSynchronize(s));
    if (*d->h_flag != 0) {
      // rank-revealing path: S = U diag(lam) U^H, keep the directions with
      // lam above 1e-12 of the largest and above the drop level; they mix
      // the columns, so all of them take the second round
      {
        ProfScope ps(&d->p->prof, PW_STAGE_EIG, s);
        DV_RC(copy_mat(d->S, nc, d->Ae, d->lde, nc, nc, s));
        DV_RC(eig_herm(d->Ae, d->lde, nc, d->lam, d->Ze, d->lde, d->rot_ws, d->acc_ws, d->h_acc, d->sweeps, s,
                       0.0, 0));
      }
      PW_HIP(hipMemcpyAsync(d->h_lam, d->lam, nc * sizeof(double), hipMemcpyDeviceToHost, s));
      PW_HIP(hipStreamSynchronize(s));
      double lmax = 0, cmax = 0;
      for (int i = 0; i < nc; ++i) {
        lmax = std::max(lmax, d->h_lam[i]);
        cmax = std::max(cmax, d->h_cnorm[i]);
      }
      const double floor = std::max(1e-12 * lmax, round == 0 ? kDrop0 * cmax : kDrop1);
      int nk = 0;
      for (int i = 0; i < nc; ++i)
        if (std::isfinite(d->h_lam[i]) && d->h_lam[i] > floor) d->h_keep[nk++] = i;
      PW_HIP(hipMemcpyAsync(d->keep, d->h_keep, nk * sizeof(int), hipMemcpyHostToDevice, s));
      if (nk > 0) {
        DV_RC(scaled_cols(d->Ze, d->lde, d->lam, d->keep, nc, nk, d->Bi, nc, s));
        DV_RC(nn(d, nk, nc, 1.0, *src, d->Bi, nc, 0.0, *out, s));
      }
      *n = nk;
      return PW_OK;
    }
    // L_jj^2 is what column j kept of its squared norm through the
    // projection and against the columns before it
    int ng = 0;
    for (int j = 0; j < nc; ++j) {
      const double l = d->h_ldiag[j].x;
      const double ref = round == 0 ? kDrop0 * d->h_cnorm[j] : kDrop1;
      if (std::isfinite(l) && l * l > ref) d->h_keep[ng++] = j;
    }
    if (ng < nc) {
      // compact the block to the columns that stay and factor again
      if (ng > 0) {
        PW_HIP(hipMemcpyAsync(d->keep, d->h_keep, ng * sizeof(int), hipMemcpyHostToDevice, s));
        DV_RC(gather_cols(*src, d->ld, d->keep, d->npw, ng, *out, d->ld, s));
        std::swap(*src, *out);
        for (int i = 0; i < ng; ++i) d->h_cnorm[i] = d->h_cnorm[d->h_keep[i]];
      }
      *n = ng;
      continue;
    }
    {
      ProfScope ps(&d->p->prof, PW_STAGE_CHOL, s);
      DV_RC(trinv_h(d->L, nc, nc, d->Xi, nc, d->Bi, nc, s));
    }
    // The normalisation amplifies what the first pass left in column j by
    // a_j = |t_j| / L_jj: the rounding of the projection (Cholesky-QR then
    // loses about eps a_j^2 of orthogonality) and the space's own loss of
    // orthonormality (the pass leaves that much of each V component, so the
    // column carries about ortho_err a_j).  A column with a_j < 1/kKeep
    // whose sum stays below skip_err would change by less than that in a
    // second round: it is taken as it is.  The head / tail order comes from
    // permuting the columns of L^-H, so the one product writes it.
    const double2 *B = d->Bi;
    if (round == 0 && ortho_skip()) {
      constexpr double kKeep2 = 1e-4;  // kKeep = 1e-2
      std::vector<char> one((size_t)nc);
      int h = 0;
      double worst = 0.0;
      for (int j = 0; j < nc; ++j) {
        const double l = d->h_ldiag[j].x, a2 = d->h_cnorm[j] / (l * l);
        const double err = d->ortho_err * std::sqrt(a2) + kEps * a2;
        one[j] = a2 < 1.0 / kKeep2 && err <= d->skip_err;
        if (one[j]) {
          d->h_keep[h++] = j;
          worst = std::max(worst, err);
        }
      }
      int t = h;
      for (int j = 0; j < nc; ++j)
        if (!one[j]) d->h_keep[t++] = j;
      if (h > 0 && h < nc) {
        PW_HIP(hipMemcpyAsync(d->keep, d->h_keep, nc * sizeof(int), hipMemcpyHostToDevice, s));
        DV_RC(gather_cols(d->Bi, nc, d->keep, nc, nc, d->Xi, nc, s));
        B = d->Xi;
      }
      *nh = h;
      if (h > 0) d->ortho_err = std::max(d->ortho_err, worst);
    }
    DV_RC(nn(d, nc, nc, 1.0, *src, B, nc, 0.0, *out, s));
    return PW_OK;
  }
  return PW_OK;
}

// Orthonormalise n columns at T against V[0:m] into dst (right after V[0:m]);
// *n_out columns kept.  Round 0: one Gram-Schmidt pass against V and
// Cholesky-QR.  Round 1, for the columns round 0 could not settle: one pass
// against V and the settled columns, Cholesky-QR.  The normalisation between
// the two passes amplifies what the first left; the second takes that to the
// rounding level ("twice is enough").
int ortho_block(pw_davidson *d, int m, double2 *T, int n, double2 *dst, int *n_out, hipStream_t s) {
  const bool set_error_if_empty = true;
  const char *where = "pw_davidson: orthonormalisation failed";
  *n_out = 0;
  if (n <= 0) return PW_OK;
  // squared column norms before any projection: the reference of the drop
  // test and of the one-round test
  DV_RC(col_norms2(T, d->ld, d->npw, n, d->cnorm, s));
  PW_HIP(hipMemcpyAsync(d->h_cnorm, d->cnorm, n * sizeof(double), hipMemcpyDeviceToHost, s));
  double2 *src = T, *out = dst;
  if (m > 0) {
    for (int c = 0; c < gs_first(); ++c) {
      DV_RC(cn(d, m, n, d->V, src, d->C, d->lde, s));
      DV_RC(nn(d, n, m, -1.0, d->V, d->C, d->lde, 1.0, src, s));
    }
  }
  int nh = 0;
  DV_RC(cholqr(d, 0, &src, &out, &n, &nh, s));
  if (n == 0) return PW_OK;
  if (out != dst) PW_HIP(hipMemcpyAsync(dst, out, (size_t)n * d->ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
  const int nt = n - nh;
  if (nt > 0) {
    double2 *tail = dst + (size_t)nh * d->ld;
    const int mv = m + nh;  // V[0:m] and the head are contiguous
    if (mv > 0) {
      DV_RC(cn(d, mv, nt, d->V, tail, d->C, d->lde, s));
      DV_RC(nn(d, nt, mv, -1.0, d->V, d->C, d->lde, 1.0, tail, s));
    }
    double2 *src1 = tail, *out1 = T;
    int n1 = nt, nh1 = 0;
    DV_RC(cholqr(d, 1, &src1, &out1, &n1, &nh1, s));
    if (n1 > 0 && out1 != tail)
      PW_HIP(hipMemcpyAsync(tail, out1, (size_t)n1 * d->ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
    n = nh + n1;
  }
  *n_out = n;
  return PW_OK;
}

}  // namespace

// Eigensolver stop level relative to the smallest open residual
// (PW_DAV_OFF_FACTOR).
static double off_factor() {
  static const double v = [] {
    const char *e = std::getenv("PW_DAV_OFF_FACTOR");
    return (e && *e) ? std::max(1e-6, std::atof(e)) : 3.0;
  }();
  return v;
}

// The eigensolver's stop test counts every off-diagonal pair.  With
// PW_EIG_WANTED=1 it counts only the pairs that touch the nb - nl lowest
// diagonal entries, leaving the rest among the upper directions carried in
// H_s.  That is about 7 % cheaper at the medium workload, but with the
// loose stop level the carried upper block can hide an eigenvalue below the
// wanted ones: on 3 of the 64 ragged cells the solve then stalls (the FP64
// refinement of cell 55) or diverges (cell 59 with the learned
// preconditioner), so it is off by default.
static bool eig_wanted() {
  static const int v = env_switch("PW_EIG_WANTED", 0);
  return v != 0;
}

// Active-space cap of the restart (step 5); PW_DAV_ACT_MUL=0 turns it off.
struct RestartCap {
  int mul = 3, min = 64, keep = 3;
};
static const RestartCap &restart_cap() {
  static const RestartCap c = [] {
    RestartCap r;
    r.mul = std::max(0, env_switch("PW_DAV_ACT_MUL", r.mul));
    r.min = std::max(0, env_switch("PW_DAV_ACT_MIN", r.min));
    r.keep = std::max(0, env_switch("PW_DAV_ACT_KEEP", r.keep));
    return r;
  }();
  return c;
}

namespace pw {
// Shape of a Davidson state for the batch scheduler (batch.hip): its
// problem, bands, subspace bound, and whether its last step converged.
pw_problem *dav_problem(const pw_davidson *d) { return d->p; }
int dav_nbands(const pw_davidson *d) { return d->nb; }
int dav_max_subspace(const pw_davidson *d) { return d->mmax; }
bool dav_converged(const pw_davidson *d) { return d->inited && d->converged; }
bool dav_inited(const pw_davidson *d) { return d->inited; }
}  // namespace pw

extern "C" {

pw_status pw_davidson_workspace_size(pw_problem *p, int64_t nbands, int64_t max_subspace, size_t *bytes) {
  PW_CHECK_ARG(p && bytes, PW_ERR_INVALID, "pw_davidson_workspace_size: null argument");
  *bytes = 0;
  const int rc = dav_shape(p, nbands, &max_subspace, 1.0, "pw_davidson_workspace_size");
  if (rc != PW_OK) return rc;
  pw_davidson d;
  dav_dims(&d, p, nbands, max_subspace);
  Carve c(nullptr);
  carve_dav(&d, c);
  *bytes = c.size();
  return PW_OK;
}

pw_status pw_davidson_create(pw_problem *p, int64_t nbands, int64_t max_subspace, double tol,
                             void *workspace, size_t ws_bytes, void *stream, pw_davidson **out) {
  PW_CHECK_ARG(p && out, PW_ERR_INVALID, "pw_davidson_create: null argument");
  *out = nullptr;
  int rc = dav_shape(p, nbands, &max_subspace, tol, "pw_davidson_create");
  if (rc != PW_OK) return rc;
  pw_davidson *d = new pw_davidson();
  dav_dims(d, p, nbands, max_subspace);
  d->tol = tol;
  {
    Carve count(nullptr);
    carve_dav(d, count);
    if (!workspace || ws_bytes < count.size() || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
      free_dav(d);
      set_error("pw_davidson_create: workspace must be 256-byte aligned device memory of at least "
                "pw_davidson_workspace_size() = " + std::to_string(count.size()) + " bytes");
      return PW_ERR_INVALID;
    }
    Carve c(workspace);
    carve_dav(d, c);
    d->ws = workspace;
  }
  const size_t nb = d->nb, lde = d->lde;
  const bool ok = halloc(&d->h_theta, nb) && halloc(&d->h_rho, nb) && halloc(&d->h_xn2, nb) &&
                  halloc(&d->h_lam, lde) &&
                  halloc(&d->h_U, nb) && halloc(&d->h_flag, 1) && halloc(&d->h_keep, nb) &&
                  halloc(&d->h_bad, nb) && halloc(&d->h_cnorm, nb) && halloc(&d->h_ldiag, nb) &&
                  halloc(&d->h_acc, 2);
  if (!ok) {
    free_dav(d);
    set_error("pw_davidson_create: pinned host allocation failed");
    return PW_ERR_NOMEM;
  }
  if (hipMemsetAsync(d->Hs, 0, lde * lde * sizeof(double2), static_cast<hipStream_t>(stream)) != hipSuccess) {
    free_dav(d);
    set_error("pw_davidson_create: workspace initialisation failed");
    return PW_ERR_HIP;
  }
  *out = d;
  return PW_OK;
}

pw_status pw_davidson_destroy(pw_davidson *d) {
  if (d) {
    (void)hipDeviceSynchronize();
    free_dav(d);
  }
  return PW_OK;
}

pw_status pw_davidson_init(pw_davidson *d, const void *psi0, int64_t ld, void *stream) {
  PW_CHECK_ARG(d && psi0, PW_ERR_INVALID, "pw_davidson_init: null argument");
  PW_CHECK_ARG(ld >= d->npw, PW_ERR_INVALID, "pw_davidson_init: ld < npw");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool set_error_if_empty = true;
  const char *where = "pw_davidson_init: launch failed";
  PW_HIP(hipMemsetAsync(d->T, 0, (size_t)d->nb * d->ld * sizeof(double2), s));
  PW_HIP(hipMemcpy2DAsync(d->T, d->ld * sizeof(double2), psi0, ld * sizeof(double2),
                          d->npw * sizeof(double2), d->nb, hipMemcpyDeviceToDevice, s));
  int nk = 0;
  d->ortho_err = 0.0;
  d->skip_err = 0.0;
  DV_RC(ortho_block(d, 0, d->T, d->nb, d->V, &nk, s));
  PW_CHECK_ARG(nk == d->nb, PW_ERR_NUMERIC, "pw_davidson_init: start block is rank deficient");
  DV_RC(dav_apply(d, d->V, d->W, d->nb, s));
  DV_RC(cn(d, d->nb, d->nb, d->V, d->W, d->Hs, d->lde, s));
  DV_RC(hermitize(d->Hs, d->lde, 0, d->nb, s));
  d->X = d->V;
  d->m = d->nb;
  d->iter = 0;
  d->n_hpsi = d->nb;
  d->prev_rho.assign(d->nb, INFINITY);
  d->off_target = 0.0;
  d->nl = 0;
  d->stall.assign(d->nb, 0);
  d->tpa_only.assign(d->nb, 0);
  d->inited = true;
  d->converged = false;
  d->stalled = false;
  return PW_OK;
}

pw_status pw_davidson_step(pw_davidson *d, int32_t precond_kind, const pw_mlp *net, void *stream,
                           int32_t *converged) {
  PW_CHECK_ARG(d && d->inited, PW_ERR_INVALID, "pw_davidson_step: state not initialised");
  PW_CHECK_ARG(precond_kind >= PW_PRECOND_NONE && precond_kind <= PW_PRECOND_MLP, PW_ERR_INVALID,
               "pw_davidson_step: unknown preconditioner");
  PW_CHECK_ARG(precond_kind != PW_PRECOND_MLP || net, PW_ERR_INVALID,
               "pw_davidson_step: the MLP preconditioner needs a network");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool set_error_if_empty = true;
  const char *where = "pw_davidson_step: launch failed";
  const int nb = d->nb;
  d->stalled = false;
  // 1. Rayleigh-Ritz: Z^H H_s Z = diag(w) + E, eigenpairs sorted ascending.
  //    The eigensolver transforms H_s in place and stops once the
  //    off-diagonal part E is below off_target (tied to the residuals of
  //    the previous step) and Z^H H_s Z, E included, becomes the next H_s,
  //    so nothing is dropped and the next step continues the diagonalisation.
  //    The residual test below sees E: R_n has an in-subspace part of norm
  //    |E e_n|, so convergence still means every Ritz pair is accurate.
  //    Only the active block (indices nl .. m-1) takes part: the locked
  //    prefix is fixed, and its couplings to the active part, of the order
  //    of its residuals (below the tolerance), are left out.
  const int nl = d->nl, ma = d->m - nl;
  const double used_target = d->off_target;
  const size_t hoff = (size_t)nl * d->lde + nl;
  {
    ProfScope ps(&d->p->prof, PW_STAGE_EIG, s);
    DV_RC(copy_mat(d->Hs + hoff, d->lde, d->Ae, d->lde, ma, ma, s));
    DV_RC(eig_herm(d->Ae, d->lde, ma, d->w_all, d->Ze, d->lde, d->rot_ws, d->acc_ws, d->h_acc, d->sweeps,
                   s, d->off_target, eig_wanted() ? nb - nl : 0));
    DV_RC(eig_select(d->w_all, ma, ma, d->w_sorted, d->idx_all, d->Ze, d->lde, d->Ae, d->lde, s,
                     d->Ae, d->lde, d->Hs + hoff, d->lde));
  }
  // 2. rotate the active space into the Ritz basis (V <- V Z, W <- W Z): the
  //    first nb columns are the Ritz vectors, the active H_s becomes diag(w),
  //    and the next bordered H_s is nearly diagonal, so its Jacobi solve is
  //    short.  The locked columns are carried over unchanged.  The Ritz
  //    vectors are rotated first; the upper columns only once step 5 has
  //    decided how many of them the space keeps.
  const size_t lcol = (size_t)nl * d->ld;
  const int nw = nb - nl;
  DV_RC(nn(d, nw, ma, 1.0, d->V + lcol, d->Ae, d->lde, 0.0, d->Vt + lcol, s));
  DV_RC(nn(d, nw, ma, 1.0, d->W + lcol, d->Ae, d->lde, 0.0, d->Wt + lcol, s));
  if (nl > 0) {
    PW_HIP(hipMemcpyAsync(d->Vt, d->V, lcol * sizeof(double2), hipMemcpyDeviceToDevice, s));
    PW_HIP(hipMemcpyAsync(d->Wt, d->W, lcol * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  if (nb > nl)
    PW_HIP(hipMemcpyAsync(d->theta + nl, d->w_sorted, (nb - nl) * sizeof(double), hipMemcpyDeviceToDevice, s));
  // 3. residuals
  {
    ProfScope ps(&d->p->prof, PW_STAGE_VEC, s);
    DV_RC(residual(d->Vt, d->Wt, d->theta, d->R, d->ld, d->npw, nb, d->rho, d->xn2, s));
  }
  PW_HIP(hipMemcpyAsync(d->h_theta, d->theta, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  PW_HIP(hipMemcpyAsync(d->h_rho, d->rho, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  PW_HIP(hipMemcpyAsync(d->h_xn2, d->xn2, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  d->iter++;
  d->ortho_err = 0.0;
  double th_max = 0.1;
  for (int n = 0; n < nb; ++n) {
    d->ortho_err = std::max(d->ortho_err, std::fabs(d->h_xn2[n] - 1.0));
    th_max = std::max(th_max, std::fabs(d->h_theta[n]));
  }
  d->skip_err = std::min(1e-9, 0.1 * d->tol / th_max);
  for (int n = 0; n < nb; ++n)
    if (!std::isfinite(d->h_theta[n]) || !std::isfinite(d->h_rho[n])) {
      set_error("pw_davidson_step: non-finite Ritz value or residual");
      return PW_ERR_NOT_FINITE;
    }
  int nu = 0;
  double rho_min = INFINITY;
  for (int n = 0; n < nb; ++n) {
    if (d->h_rho[n] >= d->tol) {
      d->h_U[nu++] = n;
      rho_min = std::min(rho_min, d->h_rho[n]);
    }
    d->stall[n] = (d->h_rho[n] >= d->prev_rho[n]) ? d->stall[n] + 1 : 0;
    if (d->stall[n] >= 2) d->tpa_only[n] = 1;
    d->prev_rho[n] = d->h_rho[n];
  }
  d->converged = (nu == 0);
  // next step's eigensolver target: off_factor (3) times the smallest
  // residual still to converge, never below that times the tolerance.  The
  // off-diagonal rest is carried in H_s and counted in every residual, so a
  // band converges only once its column of it is below the tolerance.
  d->off_target = off_factor() * std::max(d->tol, nu ? rho_min : d->tol);
  // lock the converged prefix.  An active Ritz value below the largest
  // locked one means the locked bands are not the lowest after all: the
  // locking is dropped and H_s rebuilt over the whole space.
  bool lock_drop = false;
  if (!d->converged) {
    if (nl > 0 && nl < nb && d->h_theta[nl] < d->h_theta[nl - 1] - d->tol) {
      d->nl = 0;
      lock_drop = true;
    } else {
      int l = nl;
      while (l < nb && d->h_rho[l] < d->tol) ++l;
      d->nl = l;
    }
  }
  // 5. restart with the Ritz vectors when the space is full (they are the
  //    first nb columns of the rotated V, with H_s = diag(theta) there)
  //    The active part is also capped at act_mul times the bands still to
  //    converge (at least act_min): late in a solve nearly all of it is
  //    upper Ritz vectors, which carry almost all of the next subspace
  //    matrix's off-diagonal mass and none of the wanted pairs.  That
  //    restart keeps act_keep times as many upper Ritz vectors as bands
  //    left to converge.  A converged solve keeps the whole space.
  int keep = d->m;
  if (!d->converged) {
    if (d->m + nu > d->mmax) {
      keep = nb;
    } else {
      const int nact = nb - d->nl;
      const RestartCap &rc = restart_cap();
      if (rc.mul > 0 && d->m - d->nl + nu > std::max(rc.min, rc.mul * nact))
        keep = std::min(d->m, nb + rc.keep * nact);
    }
  }
  // the upper columns that stay: nb .. keep-1
  if (keep > nb) {
    const size_t ucol = (size_t)nb * d->ld;
    const double2 *Zu = d->Ae + (size_t)nw * d->lde;
    DV_RC(nn(d, keep - nb, ma, 1.0, d->V + lcol, Zu, d->lde, 0.0, d->Vt + ucol, s));
    DV_RC(nn(d, keep - nb, ma, 1.0, d->W + lcol, Zu, d->lde, 0.0, d->Wt + ucol, s));
  }
  std::swap(d->V, d->Vt);
  std::swap(d->W, d->Wt);
  d->X = d->V;
  d->m = keep;
  if (lock_drop) {
    DV_RC(cn(d, d->m, d->m, d->V, d->W, d->Hs, d->lde, s));
    DV_RC(hermitize(d->Hs, d->lde, 0, d->m, s));
    d->off_target = 0.0;
  }
  if (converged) *converged = d->converged ? 1 : 0;
  if (d->converged) return PW_OK;
  PW_HIP(hipMemcpyAsync(d->dU, d->h_U, nu * sizeof(int), hipMemcpyHostToDevice, s));
  // 4. preconditioned corrections for the unconverged bands
  auto corrections = [&]() -> int {
    ProfScope ps(&d->p->prof, PW_STAGE_PRECOND, s);
    DV_RC(band_kinetic(d->p->d_kin, d->X, d->ld, d->npw, nb, d->tn, s));
    if (precond_kind == PW_PRECOND_MLP) {
      for (int i = 0; i < nu; ++i) d->h_bad[i] = d->tpa_only[d->h_U[i]];
      PW_HIP(hipMemcpyAsync(d->bad, d->h_bad, nu * sizeof(int), hipMemcpyHostToDevice, s));
      DV_RC(mlp_precond_idx(net, d->p, d->theta, d->rho, d->dU, d->R, d->ld, d->T, nu, d->bad, d->tn, s));
      DV_RC(mlp_fallback(d->bad, d->p, d->tn, d->dU, d->R, d->ld, d->T, nu, s));
    } else {
      DV_RC(precond_idx(d->p->d_kin, d->tn, d->dU, d->R, d->ld, d->T, d->ld, d->npw, nu, precond_kind, s));
    }
    return PW_OK;
  };
  DV_RC(corrections());
  // 6. orthonormalise against the space
  int nk = 0;
  DV_RC(ortho_block(d, d->m, d->T, nu, d->V + (size_t)d->m * d->ld, &nk, s));
  if (nk == 0) {
    // Every correction lies numerically in the space, so what the residuals
    // still hold is their part inside it: the off-diagonal rest the
    // eigensolver stopped at, or the couplings to the locked prefix.  Those
    // are resolved first (the next step diagonalises to the rounding level,
    // over the whole space if bands were locked); then the corrections are
    // tried against the Ritz vectors alone.  Past that the residuals are at
    // the rounding level of the Ritz vectors and the solve has stalled.
    if (used_target > 0.0 || nl > 0) {
      if (nl > 0) {
        d->nl = 0;
        DV_RC(cn(d, d->m, d->m, d->V, d->W, d->Hs, d->lde, s));
        DV_RC(hermitize(d->Hs, d->lde, 0, d->m, s));
      }
      d->off_target = 0.0;
      return PW_OK;
    }
    if (d->m > nb) {
      d->m = nb;
      DV_RC(corrections());
      DV_RC(ortho_block(d, d->m, d->T, nu, d->V + (size_t)d->m * d->ld, &nk, s));
    }
    if (nk == 0) {
      d->stalled = true;
      return PW_OK;
    }
  }
  double2 *Vn = d->V + (size_t)d->m * d->ld;
  double2 *Wn = d->W + (size_t)d->m * d->ld;
  // 7. H on the new vectors, bordered subspace matrix
  DV_RC(dav_apply(d, Vn, Wn, nk, s));
  d->n_hpsi += nk;
  DV_RC(cn(d, d->m + nk, nk, d->V, Wn, d->Hs + (size_t)d->m * d->lde, d->lde, s));
  DV_RC(hermitize(d->Hs, d->lde, d->m, d->m + nk, s));
  d->m += nk;
  return PW_OK;
}

pw_status pw_davidson_set_problem(pw_davidson *d, pw_problem *p, void *stream) {
  PW_CHECK_ARG(d && p, PW_ERR_INVALID, "pw_davidson_set_problem: null argument");
  PW_CHECK_ARG(p->npw == d->npw && p->max_bands >= d->nb, PW_ERR_INVALID,
               "pw_davidson_set_problem: problem must share npw and allow nbands bands");
  PW_CHECK_ARG(p->gen == d->p->gen, PW_ERR_INVALID,
               "pw_davidson_set_problem: both problems must have augmentation, or neither");
  d->p = p;
  if (!d->inited) return PW_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool set_error_if_empty = true;
  const char *where = "pw_davidson_set_problem: launch failed";
  for (int c0 = 0; c0 < d->m; c0 += d->nb) {
    const int nc = std::min(d->nb, d->m - c0);
    DV_RC(dav_apply(d, d->V + (size_t)c0 * d->ld, d->W + (size_t)c0 * d->ld, nc, s));
  }
  d->n_hpsi += d->m;
  DV_RC(cn(d, d->m, d->m, d->V, d->W, d->Hs, d->lde, s));
  DV_RC(hermitize(d->Hs, d->lde, 0, d->m, s));
  // a new operator: every band is checked again, nothing stays locked
  d->nl = 0;
  d->off_target = 0.0;
  return PW_OK;
}

pw_status pw_davidson_set_tol(pw_davidson *d, double tol) {
  PW_CHECK_ARG(d && tol > 0 && std::isfinite(tol), PW_ERR_INVALID, "pw_davidson_set_tol: bad argument");
  d->tol = tol;
  return PW_OK;
}

pw_status pw_davidson_run(pw_davidson *d, int32_t max_iter, int32_t precond_kind, const pw_mlp *net,
                          void *stream, int32_t *converged) {
  PW_CHECK_ARG(d && max_iter >= 1, PW_ERR_INVALID, "pw_davidson_run: bad argument");
  int32_t c = 0;
  for (int it = 0; it < max_iter; ++it) {
    const int rc = pw_davidson_step(d, precond_kind, net, stream, &c);
    if (rc != PW_OK) return rc;
    if (c || d->stalled) break;
  }
  if (converged) *converged = c;
  return c ? PW_OK : PW_NOT_CONVERGED;
}

pw_status pw_davidson_query(pw_davidson *d, double *theta, double *resid, int32_t *iterations,
                            int64_t *n_hpsi, void *stream) {
  PW_CHECK_ARG(d, PW_ERR_INVALID, "pw_davidson_query: null state");
  PW_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  if (theta) std::copy(d->h_theta, d->h_theta + d->nb, theta);
  if (resid) std::copy(d->h_rho, d->h_rho + d->nb, resid);
  if (iterations) *iterations = d->iter;
  if (n_hpsi) *n_hpsi = d->n_hpsi;
  return PW_OK;
}

pw_status pw_davidson_snapshot(pw_davidson *d, void *x, void *r, double *theta, double *rho,
                               int64_t ld, void *stream) {
  PW_CHECK_ARG(d && ld >= d->npw, PW_ERR_INVALID, "pw_davidson_snapshot: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t row = d->npw * sizeof(double2), lds = ld * sizeof(double2), ldd = d->ld * sizeof(double2);
  if (x) PW_HIP(hipMemcpy2DAsync(x, lds, d->X, ldd, row, d->nb, hipMemcpyDeviceToDevice, s));
  if (r) PW_HIP(hipMemcpy2DAsync(r, lds, d->R, ldd, row, d->nb, hipMemcpyDeviceToDevice, s));
  if (theta) PW_HIP(hipMemcpyAsync(theta, d->theta, d->nb * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (rho) PW_HIP(hipMemcpyAsync(rho, d->rho, d->nb * sizeof(double), hipMemcpyDeviceToDevice, s));
  return PW_OK;
}

pw_status pw_davidson_vectors(pw_davidson *d, void *x, int64_t ld, void *stream) {
  PW_CHECK_ARG(d && x && ld >= d->npw, PW_ERR_INVALID, "pw_davidson_vectors: bad argument");
  if (d->p->gen) {
    // x = S^{-1/2} y: the S-orthonormal eigenvectors of the pencil
    const int rc = sinvhalf(d->p, d->X, d->ld, x, ld, d->nb, static_cast<hipStream_t>(stream));
    if (rc != PW_OK) set_error("pw_davidson_vectors: launch failed");
    return rc;
  }
  PW_HIP(hipMemcpy2DAsync(x, ld * sizeof(double2), d->X, d->ld * sizeof(double2),
                          d->npw * sizeof(double2), d->nb, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)));
  return PW_OK;
}

}  // extern "C"
