/*
 * pw_api.h -- C ABI of the MI355X plane-wave H*psi / block-Davidson library
 * (libpwhip.so, gfx950).
 *
 * The operator is the scalar, norm-conserving reduction (one spin
 * component, S = 1, no augmentation) of the Kohn-Sham equation the paper
 * writes in its fully relativistic PAW section (eq. pauli_ks):
 *
 *   H = p^2/2 + V_LOC(r) + sum_I sum_mn D_I,mn |beta_m^I><beta_n^I|
 *
 * in Hartree atomic units, acting on bands expanded in plane waves
 * c_{k,n}(G) (section "New parallelization levels": the largest array).
 * The local term is applied on an FFT grid (the exchange paragraph's grid
 * rule: G up to 2 G_c), the nonlocal term through the scalar products
 * p_ij = <beta_j|psi_i> (same section), and the lowest bands are found by
 * a Davidson-like iteration with subspace diagonalisation (the paper cites
 * Davidson 1975 and names subspace diagonalisation as PWscf's dominant
 * dense linear-algebra step).
 *
 * Conventions shared by every entry point
 *   - Every function returns pw_status; 0 is success.  Negative values are
 *     errors; PW_NOT_CONVERGED (1) is a non-fatal outcome.  No C++
 *     exception crosses this boundary.  pw_last_error() returns a
 *     thread-local message for the last non-OK status of the calling thread.
 *   - Argument checks run on the host, synchronously, before any launch.
 *   - Complex numbers are interleaved (re, im) doubles (complex128), the
 *     layout of C99 double _Complex and of torch.complex128.
 *   - Band blocks are band-major: element G of band n sits at
 *     ptr[n * ld + G], ld >= npw.  Padding columns G >= npw are neither read
 *     nor written.
 *   - "device" pointers are HIP device memory on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every
 *     pointer it passes, workspaces included, and never loses memory to
 *     the library: the paper's own library interface runs its routines
 *     inside resources the caller hands to an init routine (section
 *     "Modular parallelism").  A problem or Davidson handle keeps every
 *     large buffer (the reordered V_LOC, the copies of beta, the stick
 *     buffer, projections, split-K partials, the Davidson space and its
 *     subspace matrices) in a workspace the caller allocates from the size
 *     query and binds at create; it stays bound until destroy and must not
 *     be touched meanwhile.  The handle itself owns only small tables
 *     (stick maps, twiddles, kinetic energies, D blocks, a few pinned host
 *     words), released by the matching destroy call.  A handle is used by
 *     one stream at a time: two calls on one handle from different streams
 *     race on its workspace.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on that stream; calls return
 *     without waiting for it unless stated.  Buffers must stay valid until
 *     the stream has reached the end of the call's work.
 *   - Units: Hartree and bohr.  A cutoff given in Rydberg as ecutwfc is
 *     ecut = ecutwfc / 2 here.
 */
#ifndef PW_API_H
#define PW_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pw_status;
#define PW_OK 0
#define PW_NOT_CONVERGED 1
#define PW_ERR_INVALID (-1)     /* bad argument (null, negative, inconsistent) */
#define PW_ERR_SHAPE (-2)       /* sphere / grid / size does not fit */
#define PW_ERR_NOMEM (-3)       /* device allocation failed */
#define PW_ERR_HIP (-4)         /* HIP runtime error */
#define PW_ERR_NOT_FINITE (-5)  /* non-finite eigenvalue or residual seen */
#define PW_ERR_NUMERIC (-6)     /* breakdown (e.g. rank-deficient start block) */

/* precision forms of H*psi (inputs and outputs stay complex128) */
#define PW_FP64 0        /* FFT complex128, projector GEMMs FP64 MFMA */
#define PW_MIXED_FP32 1  /* FFT complex64, projector GEMMs FP32 MFMA, FP32 accumulate */
#define PW_MIXED_BF16 2  /* FFT complex64, projector GEMMs BF16 in / FP32 accumulate */

/* terms of H applied by pw_hpsi (bit mask) */
#define PW_TERM_KINETIC 1
#define PW_TERM_LOCAL 2
#define PW_TERM_NONLOCAL 4
#define PW_TERM_EXX 8      /* the exact-exchange term attached by pw_ace_set (none otherwise) */
#define PW_TERM_ALL 15

/* preconditioners */
#define PW_PRECOND_NONE 0
#define PW_PRECOND_TPA 1
#define PW_PRECOND_MLP 2

typedef struct pw_problem pw_problem;
typedef struct pw_davidson pw_davidson;
typedef struct pw_mlp pw_mlp;

/*
 * One plane-wave problem: one cell at one k-point.
 */
typedef struct {
  double cell[9];      /* bohr; row-major 3x3, rows are a1, a2, a3 */
  double kpt[3];       /* k in crystal coordinates (fractions of b1, b2, b3) */
  double ecut;         /* Ha; the sphere is |k+G|^2/2 < ecut */
  int32_t nr[3];       /* FFT grid N0, N1, N2; each 2^a 3^b 5^c, 2..128 */
  int32_t precision;   /* PW_FP64 / PW_MIXED_FP32 / PW_MIXED_BF16 */
  int64_t npw;         /* number of plane waves (> 0) */
  const int32_t *miller; /* host [npw][3] Miller triples (h,k,l), any order;
                            each |h_i| < N_i/2, else PW_ERR_SHAPE; no duplicates */
  const double *vloc;  /* device [N0][N1][N2] real V_LOC(r_j), Ha, N2 fastest;
                          r_j = (j0/N0) a1 + (j1/N1) a2 + (j2/N2) a3 */
  int64_t nproj;       /* number of projectors (>= 0) */
  int32_t natom;       /* number of atoms = D blocks (>= 0) */
  const int32_t *proj_offset; /* host [natom+1], 0 = off[0] <= ... <= off[natom] = nproj;
                                 projectors off[a]..off[a+1]-1 belong to atom a */
  const double *dij;   /* host, per-atom real symmetric blocks, row-major,
                          concatenated in atom order (sum of n_a^2 doubles), Ha */
  const void *beta;    /* device complex128 [nproj][ld_beta]: beta_j(k+G), already
                          carrying the structure factor and normalisation */
  int64_t ld_beta;     /* >= npw */
  const double *qij;   /* host, augmentation of the overlap in the layout of dij, or NULL
                          for S = 1 (norm-conserving): S = 1 + sum_I sum_mn q_I,mn
                          |beta_m^I><beta_n^I| (the -eps S of eq. pauli_ks); S must be
                          positive definite and the projectors linearly independent on
                          the sphere, else pw_problem_create returns PW_ERR_NUMERIC */
} pw_problem_desc;

/* Message for the calling thread's last non-OK status ("" if none). */
const char *pw_last_error(void);

/* Library version string. */
const char *pw_version(void);

/*
 * Plane-wave sphere {G : |k+G|^2/2 < ecut} (host only, no GPU needed).
 * Writes at most `cap` Miller triples to miller_out (host [cap][3]) in the
 * reproducible order the paper asks for in its large-record file-format
 * section: ascending kinetic energy, ties broken by (h, k, l) ascending.
 * *npw_out receives the full count; with miller_out == NULL or cap too
 * small only the count is produced (returns PW_OK).
 */
pw_status pw_gsphere(const double cell[9], const double kpt[3], double ecut,
                     int32_t *miller_out, int64_t cap, int64_t *npw_out);

/*
 * Device workspace a problem needs (bytes, into *bytes): the reordered and
 * scaled V_LOC, the padded complex128 copy of beta (and its FP32 / BF16
 * copy in the mixed forms), the stick buffer of one FFT sweep, the
 * projections P and D P for max_bands bands, split-K partial sums, and a
 * few per-band words.  Runs every check pw_problem_create runs on desc and
 * max_bands (same errors), on the host only; desc->vloc and desc->beta are
 * not read.  The size depends on PW_STICK_TILE and PW_BAND_CHUNK when set.
 */
pw_status pw_workspace_size(const pw_problem_desc *desc, int64_t max_bands, size_t *bytes);

/*
 * Build a problem handle.  Host arrays of desc are copied; V_LOC and beta
 * (device) are copied into the workspace, so the caller's V_LOC and beta
 * may be freed after the stream has passed this call.  max_bands bounds
 * nbands of later pw_hpsi calls.  workspace: device memory, 256-byte
 * aligned, of at least pw_workspace_size(desc, max_bands) bytes
 * (ws_bytes), owned by the caller and bound to the handle until
 * pw_problem_destroy; a null, misaligned or smaller workspace is
 * PW_ERR_INVALID before any device work.  Allocates only the small tables
 * (stick maps, twiddles, kinetic energies, D blocks); pw_hpsi then
 * allocates nothing.  Synchronises `stream`.
 * Errors: PW_ERR_INVALID, PW_ERR_SHAPE (sphere does not fit the grid, grid
 * size not 2^a 3^b 5^c or outside 2..128, plane too large for LDS),
 * PW_ERR_NOMEM, PW_ERR_HIP.
 */
pw_status pw_problem_create(const pw_problem_desc *desc, int64_t max_bands, void *workspace,
                            size_t ws_bytes, void *stream, pw_problem **out);
pw_status pw_problem_destroy(pw_problem *p);

/* Realised sizes of a handle: npw, number of z-sticks, nproj. */
pw_status pw_problem_info(const pw_problem *p, int64_t *npw, int64_t *nsticks,
                          int64_t *nproj);

/*
 * hpsi[n] = H psi[n] for n < nbands (terms selected by `terms`, a mask of
 * PW_TERM_*; PW_TERM_ALL for the full operator, with the exact-exchange
 * term when pw_ace_set attached one):
 *   kinetic   t(G) psi(G), t = |k+G|^2 / 2
 *   local     sum_G' V~(G - G') psi(G'),  V~(q) = N^-3 sum_j V(r_j) e^{-i q.r_j}
 *             (applied as scatter -> inverse 3D FFT -> x V(r) -> forward 3D FFT -> gather)
 *   nonlocal  sum_ij beta_i(G) D_ij <beta_j | psi>
 * psi, hpsi: device complex128, band-major, ld_psi / ld_hpsi >= npw; they
 * must not overlap.  0 <= nbands <= max_bands.  No allocation, no host sync.
 */
pw_status pw_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi,
                  int64_t ld_hpsi, int64_t nbands, int32_t terms, void *stream);

/*
 * spsi[n] = S psi[n] = psi[n] + sum_ij beta_i q_ij <beta_j|psi[n]> for
 * n < nbands (a copy of psi when the problem has no augmentation), FP64
 * whatever the precision form.  psi, spsi: device complex128 band-major,
 * distinct blocks, ld >= npw; 0 <= nbands <= max_bands.  No allocation, no
 * host sync; uses the problem's workspace (projections).
 */
pw_status pw_spsi(pw_problem *p, const void *psi, int64_t ld_psi, void *spsi, int64_t ld_spsi,
                  int64_t nbands, void *stream);

/*
 * P[n][j] = <beta_j | psi_n> (device complex128 [nbands][nproj]), the
 * paper's p_ij scalar products, in the handle's precision form.
 */
pw_status pw_projections(pw_problem *p, const void *psi, int64_t ld_psi,
                         void *proj_out, int64_t nbands, void *stream);

/*
 * Diagonal preconditioner: t[n](G) = K_n(G) r[n](G).
 *   PW_PRECOND_TPA : Teter-Payne-Allan (1989) K(x) = (27+18x+12x^2+8x^3) /
 *                    (27+18x+12x^2+8x^3+16x^4), x = t(G)/T_n, T_n the band
 *                    kinetic energy <x_n|t|x_n>/<x_n|x_n> of the iterate x.
 *   PW_PRECOND_NONE: K = 1.
 *   PW_PRECOND_MLP : K = s(G, n) K_TPA(G, n), s from the network `net` (see
 *                    pw_mlp_*): a learned per-G scale on top of TPA, with
 *                    per-band fallback to TPA when any s of the band is not
 *                    finite.  The features are those of pw_mlp_features,
 *                    with |r_n| computed here.  (Inside pw_davidson_step a
 *                    band also falls back once its residual has not
 *                    decreased for two consecutive steps; a single call has
 *                    no such history.)
 * theta: device double [nbands] Ritz values (MLP only; may be NULL otherwise);
 * x, r, t: device complex128 band-major with leading dimension ld; t must
 * not overlap x or r.  Uses the problem's workspace (per-band words).
 */
pw_status pw_precond(pw_problem *p, int32_t kind, const double *theta,
                     const void *x, const void *r, void *t, int64_t ld,
                     int64_t nbands, const pw_mlp *net, void *stream);

/*
 * Device workspace of a Davidson state (bytes): the space V, W = H V and
 * their rotation targets [max_subspace][ld], the Ritz vectors X, H X, the
 * residuals and corrections [nbands][ld] (ld = npw rounded up to 64), the
 * subspace matrices and eigensolver work [lde][lde] (lde = max_subspace
 * rounded up to 32), split-K partials and per-band words.  Same argument
 * checks as pw_davidson_create (tol excepted); host only.
 */
pw_status pw_davidson_workspace_size(pw_problem *p, int64_t nbands, int64_t max_subspace,
                                     size_t *bytes);

/*
 * Block-Davidson state for the lowest nbands eigenpairs of one problem.
 * max_subspace (>= 2*nbands; 0 = 3*nbands) bounds the search space; tol is
 * the residual 2-norm target in Ha (|H x - theta x| < tol for every band).
 * All subspace work (H_s = V^H H V, Cholesky orthonormalisation, the
 * Hermitian eigensolve, Ritz vectors, residual norms) runs in FP64 on the
 * GPU whatever the problem's precision form.  With augmentation (S != 1)
 * the solve is of the pencil H x = theta S x: the state iterates y =
 * S^{1/2} x with the operator S^{-1/2} H S^{-1/2} (S^{-1/2} is exact, from
 * the projector span), so its space is S-orthonormal in x; residual norms
 * are |S^{-1/2}(H x - theta S x)|, and pw_davidson_vectors returns the
 * S-orthonormal x (snapshots stay in y).  workspace: device memory,
 * 256-byte aligned, of at least pw_davidson_workspace_size bytes, owned by
 * the caller and bound to the state until pw_davidson_destroy (null,
 * misaligned or too small: PW_ERR_INVALID before any device work).  The
 * state allocates only a few pinned host words.
 */
pw_status pw_davidson_create(pw_problem *p, int64_t nbands, int64_t max_subspace, double tol,
                             void *workspace, size_t ws_bytes, void *stream, pw_davidson **out);
pw_status pw_davidson_destroy(pw_davidson *d);

/* Load and orthonormalise the start block (device complex128 [nbands][ld]),
 * apply H, build the first subspace matrix.  PW_ERR_NUMERIC if rank deficient. */
pw_status pw_davidson_init(pw_davidson *d, const void *psi0, int64_t ld, void *stream);

/*
 * One Davidson iteration: Rayleigh-Ritz in the current space, Ritz vectors,
 * residuals and their norms; if not converged, preconditioned corrections
 * for the unconverged bands, restart when the space is full or its active
 * part (the columns past the converged prefix) exceeds max(64, 3 x the bands
 * left to converge) -- that restart keeps the lowest Ritz vectors plus three
 * upper ones per band left (PW_DAV_ACT_MUL / _MIN / _KEEP override; MUL=0
 * disables it) --, classical Gram-Schmidt + Cholesky-QR (a second round
 * for the columns the first leaves further from orthonormal than a tenth of
 * the tolerance over the largest |Ritz value|), H on the new
 * vectors and the bordered subspace matrix.  A correction that keeps at most
 * 1e-8 of its norm through the projection lies numerically in the space and
 * is dropped; when every correction is dropped the space restarts from the
 * Ritz vectors and tries once more, and if nothing is added then either, the
 * solve has stalled at its rounding floor: the step returns PW_OK with
 * *converged = 0 and pw_davidson_run stops there.  Synchronises the stream to
 * read back the residual norms, the Cholesky checks and the eigensolver's
 * convergence per sweep; sets *converged.  Returns PW_ERR_NOT_FINITE on a
 * non-finite norm.
 */
pw_status pw_davidson_step(pw_davidson *d, int32_t precond_kind, const pw_mlp *net,
                           void *stream, int32_t *converged);

/* Switch a solve to another problem on the same sphere (same npw and G
 * order, max_bands >= nbands), typically the FP64 form of a mixed-precision
 * problem: W = H V and H_s = V^H W are recomputed for the current space, so
 * the following steps converge on the new operator ("refinement"). */
pw_status pw_davidson_set_problem(pw_davidson *d, pw_problem *p, void *stream);

/* Change the residual target of a solve (Ha, > 0). */
pw_status pw_davidson_set_tol(pw_davidson *d, double tol);

/* Up to max_iter calls of pw_davidson_step (fewer if a step stalls); PW_OK
 * when converged, else PW_NOT_CONVERGED (positive) with the state left after
 * the last step. */
pw_status pw_davidson_run(pw_davidson *d, int32_t max_iter, int32_t precond_kind,
                          const pw_mlp *net, void *stream, int32_t *converged);

/* Host copies of the current Ritz values / residual norms ([nbands] each,
 * either may be NULL), the iteration count and the number of bands H has
 * been applied to.  Synchronises the stream. */
pw_status pw_davidson_query(pw_davidson *d, double *theta, double *resid,
                            int32_t *iterations, int64_t *n_hpsi, void *stream);

/* Device copies of the last step's Ritz vectors x, residuals r (complex128
 * [nbands][ld], either may be NULL), Ritz values and residual norms (double
 * [nbands], either may be NULL).  Stream-ordered, no sync. */
pw_status pw_davidson_snapshot(pw_davidson *d, void *x, void *r, double *theta, double *rho,
                               int64_t ld, void *stream);

/* Copy the current Ritz vectors to x (device complex128 [nbands][ld]). */
pw_status pw_davidson_vectors(pw_davidson *d, void *x, int64_t ld, void *stream);

/*
 * Hermitian eigensolver of the subspace step (cyclic two-sided Jacobi, FP64):
 * eigenvalues ascending in w (device double [m]) and the matching
 * orthonormal eigenvectors as the columns of Z (device complex128, column-
 * major, ldz >= m).  A (device complex128, column-major, lda >= m) is read,
 * not modified.  work: device scratch of pw_eigh_workspace(m) bytes.
 */
pw_status pw_eigh_workspace(int32_t m, size_t *bytes);
pw_status pw_eigh(const void *A, int64_t lda, int32_t m, double *w, void *Z, int64_t ldz, void *work,
                  size_t work_bytes, void *stream);
/*
 * pw_eigh for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same eigensolver with its workspace in a static device array of the
 * library (12.6 MB per GPU, held until the process ends) instead of a
 * caller buffer.  Same arguments and results as pw_eigh without work and
 * work_bytes.  m at most 512 (PW_ERR_INVALID above, before any device
 * work).  Allocates nothing.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two host threads)
 * race on it and must be serialised by the caller.
 */
pw_status pw_eigh_noalloc(const void *A, int64_t lda, int32_t m, double *w, void *Z, int64_t ldz,
                          void *stream);

/*
 * Batched H*psi over independent problems (cells or k-points with ragged
 * npw, grids and band counts): the paper runs such units side by side as
 * images and k-point pools.  A batch lists, per problem, its input and
 * output band blocks (device complex128, band-major) and band count; the
 * caller keeps every pointer valid for the batch's lifetime.
 *   pw_batch_hpsi     eager sweep (pw_hpsi on every problem, in order)
 *   pw_batch_capture  records the sweep into a HIP graph on `stream` (a
 *                     non-null stream; profiling must be off) and
 *                     instantiates it
 *   pw_batch_launch   replays the graph: one launch per sweep
 */
typedef struct pw_batch pw_batch;
pw_status pw_batch_create(pw_problem *const *probs, int32_t n, const void *const *psi,
                          const int64_t *ld_psi, void *const *hpsi, const int64_t *ld_hpsi,
                          const int64_t *nbands, pw_batch **out);
pw_status pw_batch_destroy(pw_batch *b);
pw_status pw_batch_hpsi(pw_batch *b, void *stream);
pw_status pw_batch_capture(pw_batch *b, void *stream);
pw_status pw_batch_launch(pw_batch *b, void *stream);
/*
 * Side streams for a batch's sweep (distinct non-null hipStream_t as void*,
 * at most 64; nstreams = 0 restores the in-order sweep).  Problems are
 * placed on them longest first by npw * nbands * (log2 N0 + nproj / 64);
 * pw_batch_hpsi, and the graph pw_batch_capture records, then fork from the
 * call's stream to the side streams (an event) and join back (one event per
 * side stream), so the problems of different side streams overlap on the
 * GPU.  Results are those of the in-order sweep, bit for bit.
 */
pw_status pw_batch_set_streams(pw_batch *b, void *const *streams, int32_t nstreams);

/*
 * Batched Davidson: independent solves (cells, k-points) advanced side by
 * side, the paper's images and k-point pools on one GPU.  Each caller
 * stream gets one host worker thread, which issues its solves' kernels on
 * that stream and waits on their host syncs, so the kernels of different
 * solves overlap and one solve's syncs do not stall the others.  The solves
 * are created beforehand (pw_davidson_create, each with its own problem and
 * workspaces) and stay owned by the caller; they must be distinct, must not
 * share a problem, and must live on the current device.  Streams: distinct
 * non-null hipStream_t as void*, 1..64.  A solve is placed on the streams
 * longest first by npw * nbands * (log2 N0 + nproj / 64) + npw * m_max^2 / 8.
 *   pw_batch_davidson_init  pw_davidson_init of every solve (psi0[i] device
 *                           complex128 [nbands_i][ld[i]]), on its stream
 *   pw_batch_davidson_step  one pw_davidson_step of every solve not yet
 *                           converged; *nconverged (may be NULL) counts the
 *                           converged solves afterwards
 *   pw_batch_davidson_run   init and up to max_iter steps of every solve,
 *                           the workers taking solves from one queue,
 *                           longest first; with psi0 == NULL no init: every
 *                           solve continues from its state (e.g. after
 *                           pw_davidson_set_problem and _set_tol for an FP64
 *                           refinement).  converged[i] (host int32 [n], may
 *                           be NULL) per solve.  PW_OK when every solve
 *                           converged, else PW_NOT_CONVERGED.
 * Results per solve are those of the same calls made one solve after
 * another.  Every call returns once its workers have finished and every
 * stream has completed the call's device work (the caller may then use or
 * free the solves' memory from any stream); the first failing solve's
 * status and message are returned.
 */
typedef struct pw_batch_dav pw_batch_dav;
pw_status pw_batch_davidson_create(pw_davidson *const *solvers, int32_t n, void *const *streams,
                                   int32_t nstreams, pw_batch_dav **out);
pw_status pw_batch_davidson_destroy(pw_batch_dav *b);
pw_status pw_batch_davidson_init(pw_batch_dav *b, const void *const *psi0, const int64_t *ld);
pw_status pw_batch_davidson_step(pw_batch_dav *b, int32_t precond_kind, const pw_mlp *net,
                                 int32_t *nconverged);
pw_status pw_batch_davidson_run(pw_batch_dav *b, const void *const *psi0, const int64_t *ld, int32_t max_iter,
                                int32_t precond_kind, const pw_mlp *net, int32_t *converged);

/*
 * Autotuner: times pw_hpsi on nbands scratch bands (reps timed calls per
 * shape) over the plane kernel and the bands per plane workgroup, then the
 * bands per FFT sweep, then the split-K factor of the projection GEMM, keeps
 * the fastest in the handle and returns its time (ms per call, may be NULL).
 * scratch: device memory of at least 2 * nbands * ld * 16 bytes
 * (scratch_bytes; ld = npw rounded up to 64), owned by the caller, for the
 * input and output bands of the timing runs; synchronises the stream.
 * pw_problem_tuning reports the handle's current choices (any output may be
 * NULL); plane_kernel is one of PW_PLANE_*.
 */
#define PW_PLANE_REGISTER 0 /* line FFTs in registers (even compile-time grid sizes) */
#define PW_PLANE_WAVE 1     /* wave-local LDS passes                                 */
#define PW_PLANE_LDS 2      /* workgroup LDS Stockham passes                         */
pw_status pw_problem_autotune(pw_problem *p, int64_t nbands, int32_t reps, void *scratch,
                              size_t scratch_bytes, void *stream, double *best_ms);
pw_status pw_problem_tuning(const pw_problem *p, int32_t *plane_group, int64_t *band_chunk,
                            int32_t *ksplit, int32_t *plane_kernel);
/*
 * Sets the launch choices (e.g. saved from an earlier autotune):
 * plane_group >= 1; 1 <= band_chunk <= the sweep height chosen at create
 * (the stick buffer's size); 0 <= ksplit <= 64 (0: automatic); plane_kernel
 * one of PW_PLANE_* (PW_PLANE_REGISTER falls back to PW_PLANE_LDS on grids
 * without a register instance).  PW_ERR_INVALID leaves the handle unchanged.
 */
pw_status pw_problem_set_tuning(pw_problem *p, int32_t plane_group, int64_t band_chunk, int32_t ksplit,
                                int32_t plane_kernel);

/*
 * Learned diagonal preconditioner (FP32 network 4 -> 64 -> 64 -> 1, SiLU,
 * output z mapped to s = 1/4 + (15/4) sigmoid(z), so 1/4 < s < 4; not part
 * of the paper).  In a Davidson step the
 * correction of band n is T(G) = s(G, n) K_TPA(G, n) R(G), so s = 1 is TPA;
 * training therefore takes K_TPA R as its residual samples.  Parameters are one packed float
 * array of pw_mlp_num_params() values: W1 [64][4], b1 [64], W2 [64][64],
 * b2 [64], W3 [64], b3 [1] (row-major, y = W x + b).  The scaler holds the
 * feature means mu[4] and inverse standard deviations is[4]; features are
 * standardised as (f - mu) * is.  Features of sample (G, n), float4:
 * (t(G)/T_n, theta_n, |r_n(G)| sqrt(npw) / ||r_n||, <V_LOC>), with t(G) the
 * kinetic energy |k+G|^2/2 and T_n = <x_n|t|x_n>/<x_n|x_n> the band's.
 */
int32_t pw_mlp_num_params(void);
/* params / scaler: host arrays (NULL: zeros / identity scaling). */
pw_status pw_mlp_create(const float *params, const float *scaler, pw_mlp **out);
pw_status pw_mlp_destroy(pw_mlp *net);
/* Host copies (any may be NULL); grad is the last train step's gradient. Syncs the device. */
pw_status pw_mlp_get(pw_mlp *net, float *params, float *scaler, float *grad);
pw_status pw_mlp_set(pw_mlp *net, const float *params, const float *scaler);
/* Raw features of nbands bands (nbands <= the problem's max_bands):
 * F[n][G] = (t(G)/T_n, theta_n, |r_n(G)| sqrt(npw)/rnorm_n, <V_loc>) with
 * T_n = <x_n|t|x_n>/<x_n|x_n>.  theta, rnorm device double [nbands]; x, r
 * device complex128 [nbands][ld] (iterates and residuals); F device float4
 * [nbands * npw] (band-major). */
pw_status pw_mlp_features(pw_problem *p, const double *theta, const void *x, const void *r,
                          const double *rnorm, int64_t ld, int64_t nbands, void *F, void *stream);
/* scaler <- mean and 1/std of the raw features F (device float4 [nsamples]). */
pw_status pw_mlp_fit_scaler(pw_mlp *net, const void *F, int64_t nsamples, void *stream);
/* s[i] = network output for raw features F[i] (device float [nsamples]). */
pw_status pw_mlp_forward(pw_mlp *net, const void *F, int64_t nsamples, float *s, void *stream);
/*
 * One training step on a batch of band samples.  F: raw features (float4),
 * R: residual values, D: target corrections (complex128), one entry per
 * sample; band b owns samples band_off[b] .. band_off[b+1]-1 (device int64
 * [nbands+1]); band_of[i] is the band of sample i (device int32).  Loss =
 * mean over bands of 1 - |<d, sR>|^2 / (||d||^2 ||sR||^2); its gradient is
 * left in the network (pw_mlp_get), and with update != 0 one Adam step (lr,
 * 0.9, 0.999, 1e-8) is applied.  s_work: device float [nsamples].  loss_out
 * (host, may be NULL) syncs the stream.
 */
pw_status pw_mlp_train_step(pw_mlp *net, const void *F, const void *R, const void *D,
                            const int64_t *band_off, const int32_t *band_of, int64_t nbands,
                            int64_t nsamples, float *s_work, float lr, int32_t update,
                            double *loss_out, void *stream);
/*
 * Target corrections from converged bands: with Xc the converged vectors
 * (complex128 [nbands][ld]) and cluster[m] the degenerate-cluster id of
 * converged band m (device int32), d_n = y_n/||y_n|| - x_n where
 * y_n = sum_{m in cluster(n)} Xc_m <Xc_m | x_n> and x_n = Xit[n], and
 * D[n] = d_n - sum_m x_m <x_m | d_n>: the part of the move outside the
 * iterate block (Xit is expected to have orthonormal columns, as Ritz
 * vectors do; the formula is applied as written either way).
 * work: device scratch of 17 * nbands^2 complex128.
 */
pw_status pw_mlp_targets(pw_problem *p, const void *Xc, const int32_t *cluster, const void *Xit,
                         int64_t ld, int64_t nbands, void *D, void *work, void *stream);

/*
 * Lanczos recursion on H for many chains in lockstep, and the continued
 * fraction of the resolvent (the paper's dynamic-perturbation section:
 * g_v(w) = <v|(w - L)^{-1} v>, eq. resolvent, from the chain q_0 = 0,
 * q_1 = v, alpha_n = <q_n|L q_n>, beta_{n+1} q_{n+1} = (L - alpha_n) q_n -
 * beta_n q_{n-1}, |q_{n+1}| = 1, eqs. rec1 - rec4, as the continued fraction
 * of the tridiagonal T_M, eqs. tridiagonal and continuedfraction), here
 * with L = H of a problem.  Chain c starts from q_1 = v_c / |v_c|; beta_1 =
 * |v_c| is kept, so g_c(z) = |v_c|^2 / (z - alpha_1 - beta_2^2 / (z - ...)).
 * A chain ends at beta_{n+1} <= 1e-12 |H q_n| (an invariant subspace):
 * beta_{n+1}, q_{n+1} and every later alpha, beta are zero.  One step is one
 * pw_hpsi over the chains plus one kernel per chain; alpha and beta stay on
 * the device, so pw_lanczos_run has no host synchronisation.  Three vectors
 * per chain are kept, as the paper notes.
 *   workspace: device, 256-byte aligned, pw_lanczos_workspace_size bytes
 *              (3 nchains ld complex128, ld = npw rounded up to 64, and the
 *              coefficients), owned by the caller, bound until destroy.
 *   nchains    1 .. the problem's max_bands; max_steps >= 1.
 *   start      v: device complex128 [nchains][ld_v], ld_v >= npw; resets
 *              the chains (steps done = 0).
 *   run        nsteps more steps (steps done + nsteps <= max_steps).
 *   coefficients  device copies: alpha double [nchains][max_steps] (alpha_n
 *              at [c][n-1]), beta double [nchains][max_steps + 1] (beta_1 =
 *              |v_c| at [c][0], beta_{n+1} at [c][n]); entries past the
 *              steps done are zero; *nsteps = steps done (host).
 *   resolvent  g device complex128 [nchains][nz] at the points z (device
 *              complex128 [nz]) from the steps done (at least one).
 * The chain set uses the problem's workspace for H*psi: one stream at a
 * time for both.
 */
typedef struct pw_lanczos pw_lanczos;
pw_status pw_lanczos_workspace_size(pw_problem *p, int64_t nchains, int32_t max_steps, size_t *bytes);
pw_status pw_lanczos_create(pw_problem *p, int64_t nchains, int32_t max_steps, void *workspace,
                            size_t ws_bytes, pw_lanczos **out);
pw_status pw_lanczos_destroy(pw_lanczos *l);
pw_status pw_lanczos_start(pw_lanczos *l, const void *v, int64_t ld_v, void *stream);
pw_status pw_lanczos_run(pw_lanczos *l, int32_t nsteps, void *stream);
pw_status pw_lanczos_coefficients(pw_lanczos *l, double *alpha, double *beta, int32_t *nsteps, void *stream);
pw_status pw_lanczos_resolvent(pw_lanczos *l, const void *z, int32_t nz, void *g, void *stream);

/*
 * Stage timing (instrumentation, off by default).  When enabled, every
 * kernel launch a call makes is bracketed by two HIP events recorded on the
 * call's stream; pw_profile_read synchronises on those events and returns
 * per-stage totals (milliseconds and launch counts, arrays of PW_NSTAGES).
 * reset != 0 clears the totals after reading.
 */
#define PW_STAGE_ZFFT_INV 0   /* gather sphere + inverse z FFT          */
#define PW_STAGE_PLANE 1      /* xy FFTs + V(r) product                 */
#define PW_STAGE_ZFFT_FWD 2   /* forward z FFT + gather + kinetic       */
#define PW_STAGE_KINETIC 3    /* kinetic-only (no local term)           */
#define PW_STAGE_PROJ 4       /* <beta|psi> GEMM (+ split-K reduction)  */
#define PW_STAGE_DMAT 5       /* D p                                    */
#define PW_STAGE_NLUPD 6      /* H psi += beta (D p) GEMM               */
#define PW_STAGE_PRECOND 7    /* preconditioner                         */
#define PW_STAGE_SUBGEMM 8    /* Davidson subspace GEMMs (V^H W ...)    */
#define PW_STAGE_UPDGEMM 9    /* Davidson basis updates (V Y ...)       */
#define PW_STAGE_EIG 10       /* Davidson Hermitian eigensolve          */
#define PW_STAGE_CHOL 11      /* Davidson Cholesky / triangular solves  */
#define PW_STAGE_VEC 12       /* Davidson vector kernels (norms, copies)*/
#define PW_STAGE_EXX 13       /* exact-exchange term of H psi (ACE)     */
#define PW_NSTAGES 16
pw_status pw_profile_enable(pw_problem *p, int32_t on);
pw_status pw_profile_read(pw_problem *p, double *ms_total, int64_t *launches, int32_t reset);

/*
 * Self-consistent field loop around the solver.  The Kohn-Sham potential is
 * the sum of the local ionic, Hartree and exchange-correlation potentials
 * (the paper's relativistic PAW section writes V_LOC that way), and the
 * exact-exchange section describes the outer loop that rebuilds the
 * operator from the bands until it stops changing.  Scalar, spin-unpolarised
 * path in Hartree units:
 *   n(r)   = Omega^-1 sum_k w_k sum_n f_nk |u_nk(r)|^2, u = sum_G psi(G) e^{iG.r}
 *   V_H(G) = 4 pi n(G) / |G|^2 for G != 0, V_H(0) = 0  (Poisson in G space, as
 *            the exact-exchange section solves it for pair densities)
 *   V_x(r) = -(3 n(r) / pi)^{1/3}  (local-density exchange)
 *   f_nk   = 2 / (1 + exp((eps_nk - mu) / sigma)),  sum_k w_k sum_n f_nk = nel
 *   n_in  <- n_in + alpha (n_out - n_in)  (linear mixing), or with kerker_q0 > 0
 *            the Kerker weight alpha G^2 / (G^2 + q0^2) on each Fourier
 *            component of the residual (alpha at G = 0)
 * Grid arrays are device double [N0][N1][N2] (N2 fastest), the layout of
 * pw_problem_desc.vloc.  Only FP64 problems without augmentation.
 */

/* Bytes of device scratch pw_density needs for problem p. */
pw_status pw_density_workspace_size(const pw_problem *p, size_t *bytes);
/* n[r] += Omega^-1 sum_b f[b] |u_b(r)|^2 for the nbands bands psi (device
 * complex128 [nbands][ld], normalised so that sum_G |psi(G)|^2 = 1 for the
 * density to integrate to sum f).  f: host double [nbands] (occupation times
 * k-point weight), read before the call returns.  work: 256-byte aligned
 * device scratch of pw_density_workspace_size bytes.  Uses the problem's
 * stick buffer (one stream at a time per problem).  The sum over bands runs
 * in a fixed order (no atomics): the result is reproducible. */
pw_status pw_density(pw_problem *p, const void *psi, int64_t ld, int64_t nbands, const double *f, double *n,
                     void *work, size_t work_bytes, void *stream);
/* Bytes of device scratch pw_hxc needs on the grid of p. */
pw_status pw_hxc_workspace_size(const pw_problem *p, size_t *bytes);
/* v = vion + V_H[n] + V_x[n] on the grid of p (vion may be NULL: then
 * V_H + V_x); energies (host double [3]) = E_H = (1/2) int V_H n,
 * E_x = int n eps_x, int n v_x.  Synchronises the stream. */
pw_status pw_hxc(pw_problem *p, const double *n, const double *vion, double *v, double *energies, void *work,
                 size_t work_bytes, void *stream);
/* Replace the local potential of an FP64 problem by v (device double
 * [N0][N1][N2], Ha).  A Davidson state on the problem must be told with
 * pw_davidson_set_problem before its next step.  Synchronises the stream. */
pw_status pw_problem_set_vloc(pw_problem *p, const double *v, void *stream);

typedef struct pw_scf pw_scf;
typedef struct pw_scf_desc {
  int32_t nk;                     /* k-points */
  pw_problem *const *probs;       /* [nk] FP64 problems on one grid and cell; their V_loc is replaced */
  pw_davidson *const *davs;       /* [nk] initialised Davidson states, davs[k] on probs[k] */
  pw_batch_dav *batch;            /* optional: a batch over davs (then the solves run on its streams) */
  const double *kweights;         /* host [nk], > 0 */
  const double *vion;             /* device double [N0][N1][N2]: the fixed local potential, Ha; kept by reference */
  double nel;                     /* electrons per cell, below 2 sum_k w_k nbands_k */
  double sigma;                   /* Fermi-Dirac width, Ha, > 0 */
  double alpha;                   /* mixing factor, 0 < alpha <= 1 */
  double kerker_q0;               /* Kerker wave vector, 1/bohr; 0 for plain linear mixing */
  double exx_alpha;               /* hybrid functional: fraction of Fock exchange (0: none); Gamma point only */
  double exx_tol;                 /* outer-loop target on the exchange energy, Ha (> 0 when exx_alpha > 0) */
  int32_t exx_direct;             /* 1: the outer step attaches V_x itself (pw_vx_attach) instead of V_ace,
                                     the uncompressed operator ACE replaces; 0: ACE */
} pw_scf_desc;
/* Device workspace of the loop: densities, potential, the density and
 * Hartree scratch and one band block. */
pw_status pw_scf_workspace_size(const pw_scf_desc *d, size_t *bytes);
/* Checks the descriptor, binds the workspace (256-byte aligned, owned by the
 * caller until pw_scf_destroy), sets V_ion on every problem and refreshes
 * the Davidson states: step 0 solves with V_ion alone.  With exx_alpha > 0
 * the loop detaches any exchange term from the problem and attaches its own
 * (kept in its workspace; pw_scf_destroy detaches it again). */
pw_status pw_scf_create(const pw_scf_desc *d, void *workspace, size_t ws_bytes, void *stream, pw_scf **out);
pw_status pw_scf_destroy(pw_scf *s);
/* One SCF step: every Davidson solve to dav_tol (at most dav_max_iter
 * iterations, TPA preconditioner), occupations and mu, the output density,
 * out[0] = int |n_out - n_in| / nel (-1 at step 0, whose output density
 * becomes the first input density), then -- unless step > 0 and out[0] <
 * tol (*converged = 1) -- the mixed input density, its potential on every
 * problem and the Davidson states refreshed.  With exx_alpha > 0 this is the
 * inner loop of the paper's double loop: when it converges, the step instead
 * rebuilds V_ace from the occupied orbitals (weights f/2 above 1e-8), and
 * unless the exchange energy e_xx = sum_i w_i <psi_i|V_x psi_i> moved by
 * less than exx_tol (then *converged = 1) attaches exx_alpha V_ace, scales
 * the local exchange by 1 - exx_alpha (the first inner loop runs the plain
 * local functional) and continues from the same input density.  out (host
 * double [10]): drho, mu, E_band = sum_k w_k sum_n f eps, E_H, E_x,
 * int v_x n (of the input density this step solved with, local exchange
 * scaled), E = E_band - exx_alpha e_xx - E_H + E_x - int v_x n,
 * F = E - sigma S (S the occupations' entropy), e_xx of the attached
 * operator (0 before the first), the outer steps taken.  Synchronises the
 * stream. */
pw_status pw_scf_step(pw_scf *s, double dav_tol, int32_t dav_max_iter, double tol, double *out,
                      int32_t *converged);
/* Device copies of the input density of the last step solved and its
 * output density (either may be NULL), and of the potential the next solves
 * use.  Stream-ordered. */
pw_status pw_scf_density(pw_scf *s, double *n_in, double *n_out, void *stream);
pw_status pw_scf_potential(pw_scf *s, double *v, void *stream);

/*
 * Exact (Fock) exchange and its adaptively compressed form, ACE (the paper's
 * exact-exchange section, eqs. Vx, Poisson, Vxace).  Spin-unpolarised,
 * Hartree units, Gamma point only (k = 0, else PW_ERR_INVALID):
 *   (V_x phi)(r) = - sum_j w_j psi_j(r) v_j(r),  v_j(G) = 4 pi rho_j(G) / |G|^2
 *   (0 at G = 0),  rho_j = psi_j^* phi,
 * over the nocc occupied states psi_j (device complex128 [nocc][ld_occ]) with
 * weights w (host double [nocc]; 1 for a fully occupied spatial orbital).
 * FP64 problems without augmentation.
 */
/* Bytes of device scratch pw_vx needs (the occupied states on the full grid
 * among them: nocc N0 N1 N2 complex). */
pw_status pw_vx_workspace_size(const pw_problem *p, int64_t nocc, size_t *bytes);
/* out[i] = V_x phi_i for nphi bands (device complex128 [nphi][ld], out distinct
 * from phi), by pair densities and reciprocal-space Poisson solves on the
 * full grid: nocc pair transforms per band. */
pw_status pw_vx(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                const void *phi, int64_t ld_phi, int64_t nphi, void *out, int64_t ld_out, void *work,
                size_t work_bytes, void *stream);
/* Bytes of device scratch pw_ace_set needs. */
pw_status pw_ace_workspace_size(const pw_problem *p, int64_t nocc, size_t *bytes);
/* Build ACE from the occupied states: xi = V_x psi, M = <psi|xi> (negative
 * definite, else PW_ERR_NUMERIC), zeta = -xi L^-H with -M = L L^H, so that
 * V_ace = xi M^-1 xi^H = -zeta zeta^H, exact on the occupied manifold; then
 * attach alpha V_ace to the problem: pw_hpsi with PW_TERM_EXX (part of
 * PW_TERM_ALL) adds -alpha zeta (zeta^H psi).  zeta (device complex128
 * [nocc][ldz], ldz >= npw) and proj (device complex128 of nocc * max_bands
 * values, the scratch of that term) are the caller's and stay bound to the
 * problem until pw_ace_clear, another pw_ace_set or destroy.  A Davidson
 * state on the problem must be refreshed with pw_davidson_set_problem.
 * Synchronises the stream. */
pw_status pw_ace_set(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                     double alpha, void *zeta, int64_t ldz, void *proj, void *work, size_t work_bytes,
                     void *stream);
/* Attach alpha V_x itself, applied directly: pw_hpsi with PW_TERM_EXX adds
 * alpha V_x psi by pair densities, nocc pair transforms per band (the
 * operator ACE stands in for).  psi_occ, the host weights (copied) and work
 * (device, 256-byte aligned, pw_vx_workspace_size bytes) stay bound to the
 * problem until pw_ace_clear, another attach or destroy; each such H psi
 * call synchronises its stream.  Replaces an attached ACE. */
pw_status pw_vx_attach(pw_problem *p, const void *psi_occ, int64_t ld_occ, int64_t nocc, const double *w,
                       double alpha, void *work, size_t work_bytes, void *stream);
/* Detach the exchange term (ACE or direct). */
pw_status pw_ace_clear(pw_problem *p);

#ifdef __cplusplus
}
#endif
#endif /* PW_API_H */
