// Batched H*psi over many independent problems (cells or k-points) and a
// per-problem autotuner.
//
// The paper runs independent units side by side as images and k-point
// pools; on one GPU the same independence lets the H*psi sweeps of many
// ragged problems (different npw, grids, band counts) be recorded once into
// a HIP graph and replayed with a single launch per step.  Nothing inside
// pw_hpsi allocates, synchronises or clears memory with a memset, so the
// recorded graph is the same sequence of kernels an eager sweep enqueues.
//
// The autotuner times pw_hpsi on scratch bands for a few launch choices
// (plane kernel and bands per plane workgroup, bands per FFT sweep, split-K
// of the projection GEMM) and keeps the fastest for the handle.
#include <algorithm>
#include <vector>

#include "common.h"

using namespace pw;

struct pw_batch {
  std::vector<pw_problem *> probs;
  std::vector<const void *> psi;
  std::vector<void *> hpsi;
  std::vector<int64_t> ld_psi, ld_hpsi, nb;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

pw_status pw_batch_create(pw_problem *const *probs, int32_t n, const void *const *psi,
                          const int64_t *ld_psi, void *const *hpsi, const int64_t *ld_hpsi,
                          const int64_t *nbands, pw_batch **out) {
  PW_CHECK_ARG(out && probs && psi && hpsi && ld_psi && ld_hpsi && nbands && n >= 1, PW_ERR_INVALID,
               "pw_batch_create: bad argument");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    PW_CHECK_ARG(probs[i] && psi[i] && hpsi[i], PW_ERR_INVALID, "pw_batch_create: null entry");
    PW_CHECK_ARG(nbands[i] >= 0 && nbands[i] <= probs[i]->max_bands, PW_ERR_INVALID,
                 "pw_batch_create: nbands out of range");
    PW_CHECK_ARG(ld_psi[i] >= probs[i]->npw && ld_hpsi[i] >= probs[i]->npw, PW_ERR_INVALID,
                 "pw_batch_create: ld < npw");
  }
  pw_batch *b = new pw_batch();
  b->probs.assign(probs, probs + n);
  b->psi.assign(psi, psi + n);
  b->hpsi.assign(hpsi, hpsi + n);
  b->ld_psi.assign(ld_psi, ld_psi + n);
  b->ld_hpsi.assign(ld_hpsi, ld_hpsi + n);
  b->nb.assign(nbands, nbands + n);
  *out = b;
  return PW_OK;
}

pw_status pw_batch_destroy(pw_batch *b) {
  if (!b) return PW_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return PW_OK;
}

// Eager sweep: pw_hpsi on every problem of the batch, in order, on `stream`.
pw_status pw_batch_hpsi(pw_batch *b, void *stream) {
  PW_CHECK_ARG(b, PW_ERR_INVALID, "pw_batch_hpsi: null batch");
  for (size_t i = 0; i < b->probs.size(); ++i) {
    const int rc = pw_hpsi(b->probs[i], b->psi[i], b->ld_psi[i], b->hpsi[i], b->ld_hpsi[i], b->nb[i],
                           PW_TERM_ALL, stream);
    if (rc != PW_OK) return rc;
  }
  return PW_OK;
}

// Record the sweep into a graph (stream capture on `stream`, which must be a
// non-null stream) and instantiate it.  Profiling must be off for the batch's
// problems while capturing.
pw_status pw_batch_capture(pw_batch *b, void *stream) {
  PW_CHECK_ARG(b && stream, PW_ERR_INVALID, "pw_batch_capture: needs a batch and a non-null stream");
  for (pw_problem *p : b->probs)
    PW_CHECK_ARG(!p->prof.on, PW_ERR_INVALID, "pw_batch_capture: disable profiling first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  PW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int rc = pw_batch_hpsi(b, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != PW_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("pw_batch_capture: ") + hipGetErrorString(e));
    return PW_ERR_HIP;
  }
  b->graph = g;
  PW_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return PW_OK;
}

// One graph launch = one H*psi sweep over the whole batch.
pw_status pw_batch_launch(pw_batch *b, void *stream) {
  PW_CHECK_ARG(b && b->exec, PW_ERR_INVALID, "pw_batch_launch: capture the batch first");
  PW_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return PW_OK;
}

pw_status pw_problem_autotune(pw_problem *p, int64_t nbands, int32_t reps, void *stream,
                              double *best_ms) {
  PW_CHECK_ARG(p && nbands >= 1 && nbands <= p->max_bands && reps >= 1, PW_ERR_INVALID,
               "pw_problem_autotune: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t ld = (p->npw + 63) / 64 * 64;
  const size_t bytes = (size_t)nbands * ld * sizeof(double2);
  void *x = nullptr, *y = nullptr;
  if (hipMalloc(&x, bytes) != hipSuccess || hipMalloc(&y, bytes) != hipSuccess) {
    if (x) (void)hipFree(x);
    set_error("pw_problem_autotune: scratch allocation failed");
    return PW_ERR_NOMEM;
  }
  PW_HIP(hipMemsetAsync(x, 0, bytes, s));
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  const int64_t chunk0 = p->band_chunk;
  const int groups[] = {1, 2, 4, 8, 16};
  const int64_t chunks[] = {chunk0, 128, 64, 32};
  const int splits[] = {0, 4, 8, 12, 14, 16, 24, 28, 32};
  // the register plane kernel only where it has an instance for the grid
  std::vector<int> kernels{PW_PLANE_LDS};
  if (plane_register_ok(p->fft, p->precision)) kernels.insert(kernels.begin(), PW_PLANE_REGISTER);
  double best = 1e30;
  int bg = p->plane_group, bs = p->ksplit, bk = p->plane_kernel;
  int64_t bc = chunk0;
  auto time_it = [&](double *ms) -> int {
    int rc = pw_hpsi(p, x, ld, y, ld, nbands, PW_TERM_ALL, stream);  // warm-up
    if (rc != PW_OK) return rc;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r)
      if ((rc = pw_hpsi(p, x, ld, y, ld, nbands, PW_TERM_ALL, stream)) != PW_OK) return rc;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return PW_ERR_HIP;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t / reps;
    return PW_OK;
  };
  int rc = PW_OK;
  // coordinate search: plane kernel x plane group, then sweep height, then split-K
  for (int k : kernels) {
    for (int g : groups) {
      if (rc != PW_OK) break;
      p->plane_kernel = k;
      p->plane_group = g;
      double ms;
      if ((rc = time_it(&ms)) != PW_OK) break;
      if (ms < best) {
        best = ms;
        bg = g;
        bk = k;
      }
    }
  }
  p->plane_kernel = bk;
  p->plane_group = bg;
  for (int64_t c : chunks) {
    if (rc != PW_OK || c > chunk0 || c < 1) continue;
    p->band_chunk = c;
    double ms;
    if ((rc = time_it(&ms)) != PW_OK) break;
    if (ms < best) {
      best = ms;
      bc = c;
    }
  }
  p->band_chunk = bc;
  for (int k : splits) {
    if (rc != PW_OK) break;
    p->ksplit = k;
    double ms;
    if ((rc = time_it(&ms)) != PW_OK) break;
    if (ms < best) {
      best = ms;
      bs = k;
    }
  }
  p->ksplit = bs;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(x);
  (void)hipFree(y);
  if (rc != PW_OK) {
    set_error("pw_problem_autotune: timing run failed");
    return rc;
  }
  if (best_ms) *best_ms = best;
  return PW_OK;
}

pw_status pw_problem_set_tuning(pw_problem *p, int32_t plane_group, int64_t band_chunk, int32_t ksplit,
                                int32_t plane_kernel) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_problem_set_tuning: null handle");
  PW_CHECK_ARG(plane_group >= 1 && band_chunk >= 1 && band_chunk <= p->band_chunk_max && ksplit >= 0 &&
                   ksplit <= 64 && plane_kernel >= PW_PLANE_REGISTER && plane_kernel <= PW_PLANE_LDS,
               PW_ERR_INVALID, "pw_problem_set_tuning: choice out of range");
  p->plane_group = plane_group;
  p->band_chunk = band_chunk;
  p->ksplit = ksplit;
  p->plane_kernel = plane_kernel;
  return PW_OK;
}

pw_status pw_problem_tuning(const pw_problem *p, int32_t *plane_group, int64_t *band_chunk,
                            int32_t *ksplit, int32_t *plane_kernel) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_problem_tuning: null handle");
  if (plane_kernel) *plane_kernel = p->plane_kernel;
  if (plane_group) *plane_group = p->plane_group;
  if (band_chunk) *band_chunk = p->band_chunk;
  if (ksplit) *ksplit = p->ksplit;
  return PW_OK;
}

}  // extern "C"
