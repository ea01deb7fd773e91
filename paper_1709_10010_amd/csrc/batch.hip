// Batched H*psi and batched Davidson over many independent problems (cells
// or k-points), and a per-problem autotuner.
//
// The paper runs independent units side by side as images and k-point
// pools; on one GPU the same independence lets the H*psi sweeps of many
// ragged problems (different npw, grids, band counts) be recorded once into
// a HIP graph and replayed with a single launch per step.  Nothing inside
// pw_hpsi allocates, synchronises or clears memory with a memset, so the
// recorded graph is the same sequence of kernels an eager sweep enqueues.
//
// The autotuner times pw_hpsi on the caller's scratch bands for a few launch choices
// (plane kernel and bands per plane workgroup, bands per FFT sweep, split-K
// of the projection GEMM) and keeps the fastest for the handle.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <thread>
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
  // side streams of the sweep (pw_batch_set_streams): problems placed on
  // them longest first, forked from and joined to the call's stream
  std::vector<hipStream_t> side;
  std::vector<std::vector<int>> placed;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

namespace {

// Work of one H*psi sweep of a problem (FFT lines and projector GEMMs), the
// unit the batch balances its streams by.
double hpsi_cost(const pw_problem *p, int64_t nb) {
  return (double)p->npw * (double)nb * (std::log2((double)p->nr[0]) + (double)p->nproj / 64.0);
}

// Longest-processing-time placement of items with the given costs on k bins.
std::vector<std::vector<int>> lpt(const std::vector<double> &cost, int k) {
  std::vector<int> order(cost.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int>> bins(k);
  std::vector<double> load(k, 0.0);
  for (int i : order) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bins[j].push_back(i);
    load[j] += cost[i];
  }
  return bins;
}

void release_streams(pw_batch *b) {
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  b->fork = nullptr;
  b->join.clear();
  b->side.clear();
  b->placed.clear();
}

}  // namespace

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
  release_streams(b);
  delete b;
  return PW_OK;
}

pw_status pw_batch_set_streams(pw_batch *b, void *const *streams, int32_t nstreams) {
  PW_CHECK_ARG(b && nstreams >= 0 && nstreams <= 64 && (nstreams == 0 || streams), PW_ERR_INVALID,
               "pw_batch_set_streams: bad argument");
  for (int k = 0; k < nstreams; ++k)
    PW_CHECK_ARG(streams[k], PW_ERR_INVALID, "pw_batch_set_streams: side streams must be non-null streams");
  release_streams(b);
  if (nstreams == 0) return PW_OK;
  std::vector<double> cost(b->probs.size());
  for (size_t i = 0; i < cost.size(); ++i) cost[i] = hpsi_cost(b->probs[i], b->nb[i]);
  b->placed = lpt(cost, nstreams);
  for (int k = 0; k < nstreams; ++k) b->side.push_back(static_cast<hipStream_t>(streams[k]));
  PW_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  b->join.assign(nstreams, nullptr);
  for (int k = 0; k < nstreams; ++k) PW_HIP(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  return PW_OK;
}

// Sweep: pw_hpsi on every problem of the batch.  Without side streams, in
// order on `stream`; with them, each side stream runs its problems after
// `stream` has reached the call (fork event), and `stream` continues only
// once every side stream is done (join events), so the problems of
// different side streams overlap on the GPU.
pw_status pw_batch_hpsi(pw_batch *b, void *stream) {
  PW_CHECK_ARG(b, PW_ERR_INVALID, "pw_batch_hpsi: null batch");
  if (b->side.empty()) {
    for (size_t i = 0; i < b->probs.size(); ++i) {
      const int rc = pw_hpsi(b->probs[i], b->psi[i], b->ld_psi[i], b->hpsi[i], b->ld_hpsi[i], b->nb[i],
                             PW_TERM_ALL, stream);
      if (rc != PW_OK) return rc;
    }
    return PW_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  PW_HIP(hipEventRecord(b->fork, s));
  for (size_t k = 0; k < b->side.size(); ++k) {
    hipStream_t sk = b->side[k];
    PW_HIP(hipStreamWaitEvent(sk, b->fork, 0));
    for (int i : b->placed[k]) {
      const int rc = pw_hpsi(b->probs[i], b->psi[i], b->ld_psi[i], b->hpsi[i], b->ld_hpsi[i], b->nb[i],
                             PW_TERM_ALL, sk);
      if (rc != PW_OK) return rc;
    }
    PW_HIP(hipEventRecord(b->join[k], sk));
    PW_HIP(hipStreamWaitEvent(s, b->join[k], 0));
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

}  // extern "C"

// ---------------------------------------------------------------- batched Davidson
// Independent solves (cells or k-points) advanced side by side, one host
// worker thread per caller stream: each worker issues its solves' kernels
// on its own stream and waits on its own host syncs, so the kernels of
// different solves overlap on the GPU and one solve's syncs do not stall
// the others.  This is the paper's images and k-point pools on one GPU.
struct pw_batch_dav {
  std::vector<pw_davidson *> dav;
  std::vector<hipStream_t> streams;
  std::vector<int> order;               // solves, most work first
  std::vector<std::vector<int>> owned;  // static placement of init / step
  std::vector<int32_t> conv, iters;
  int device = 0;
};

namespace {

double solve_cost(const pw_davidson *d) {
  const pw_problem *p = dav_problem(d);
  const double mm = dav_max_subspace(d);
  return hpsi_cost(p, dav_nbands(d)) + (double)p->npw * mm * mm / 8.0;
}

// fn(k) on one host thread per stream, with the batch's device current;
// each worker then waits for its stream, so every device operation of the
// call has finished when it returns (a converged Davidson step enqueues its
// last rotation after its last host sync, and the caller may reuse or free
// the solves' memory from another stream).  The first failure's status and
// message come back to the calling thread.
template <typename F>
int run_workers(pw_batch_dav *b, F &&fn) {
  const int nw = (int)b->streams.size();
  std::vector<int> rc(nw, PW_OK);
  std::vector<std::string> msg(nw);
  std::vector<std::thread> th;
  th.reserve(nw);
  for (int k = 0; k < nw; ++k)
    th.emplace_back([&, k] {
      if (hipSetDevice(b->device) != hipSuccess) {
        rc[k] = PW_ERR_HIP;
        msg[k] = "batched Davidson: hipSetDevice failed in a worker";
        return;
      }
      rc[k] = fn(k);
      if (rc[k] < 0) msg[k] = pw_last_error();
      const hipError_t e = hipStreamSynchronize(b->streams[k]);
      if (e != hipSuccess && rc[k] >= 0) {
        rc[k] = PW_ERR_HIP;
        msg[k] = std::string("batched Davidson: stream synchronisation failed: ") + hipGetErrorString(e);
      }
    });
  for (std::thread &t : th) t.join();
  for (int k = 0; k < nw; ++k)
    if (rc[k] < 0) {
      set_error(msg[k]);
      return rc[k];
    }
  return PW_OK;
}

}  // namespace

extern "C" {

pw_status pw_batch_davidson_create(pw_davidson *const *solvers, int32_t n, void *const *streams,
                                   int32_t nstreams, pw_batch_dav **out) {
  PW_CHECK_ARG(out && solvers && streams && n >= 1 && nstreams >= 1 && nstreams <= 64, PW_ERR_INVALID,
               "pw_batch_davidson_create: bad argument");
  *out = nullptr;
  int dev = 0;
  PW_HIP(hipGetDevice(&dev));
  for (int i = 0; i < n; ++i) {
    PW_CHECK_ARG(solvers[i], PW_ERR_INVALID, "pw_batch_davidson_create: null solver");
    PW_CHECK_ARG(dav_problem(solvers[i])->device == dev, PW_ERR_INVALID,
                 "pw_batch_davidson_create: every solve must live on the current device");
    for (int j = 0; j < i; ++j)
      PW_CHECK_ARG(solvers[j] != solvers[i] && dav_problem(solvers[j]) != dav_problem(solvers[i]),
                   PW_ERR_INVALID,
                   "pw_batch_davidson_create: solves must be distinct and must not share a problem");
  }
  for (int k = 0; k < nstreams; ++k)
    PW_CHECK_ARG(streams[k], PW_ERR_INVALID, "pw_batch_davidson_create: streams must be non-null streams");
  pw_batch_dav *b = new pw_batch_dav();
  b->device = dev;
  b->dav.assign(solvers, solvers + n);
  for (int k = 0; k < nstreams; ++k) b->streams.push_back(static_cast<hipStream_t>(streams[k]));
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) cost[i] = solve_cost(solvers[i]);
  b->owned = lpt(cost, nstreams);
  b->order.resize(n);
  for (int i = 0; i < n; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  b->conv.assign(n, 0);
  b->iters.assign(n, 0);
  *out = b;
  return PW_OK;
}

pw_status pw_batch_davidson_destroy(pw_batch_dav *b) {
  delete b;
  return PW_OK;
}

pw_status pw_batch_davidson_init(pw_batch_dav *b, const void *const *psi0, const int64_t *ld) {
  PW_CHECK_ARG(b && psi0 && ld, PW_ERR_INVALID, "pw_batch_davidson_init: bad argument");
  const int rc = run_workers(b, [&](int k) {
    for (int i : b->owned[k]) {
      const int r = pw_davidson_init(b->dav[i], psi0[i], ld[i], b->streams[k]);
      if (r != PW_OK) return r;
      b->conv[i] = 0;
    }
    return (int)PW_OK;
  });
  return rc;
}

pw_status pw_batch_davidson_step(pw_batch_dav *b, int32_t precond_kind, const pw_mlp *net, int32_t *nconverged) {
  PW_CHECK_ARG(b, PW_ERR_INVALID, "pw_batch_davidson_step: null batch");
  for (pw_davidson *d : b->dav)
    PW_CHECK_ARG(dav_inited(d), PW_ERR_INVALID, "pw_batch_davidson_step: initialise every solve first");
  const int rc = run_workers(b, [&](int k) {
    for (int i : b->owned[k]) {
      if (b->conv[i]) continue;
      int32_t c = 0;
      const int r = pw_davidson_step(b->dav[i], precond_kind, net, b->streams[k], &c);
      if (r != PW_OK) return r;
      b->conv[i] = c;
    }
    return (int)PW_OK;
  });
  if (nconverged) {
    int32_t nc = 0;
    for (int32_t c : b->conv) nc += c ? 1 : 0;
    *nconverged = nc;
  }
  return rc;
}

pw_status pw_batch_davidson_run(pw_batch_dav *b, const void *const *psi0, const int64_t *ld, int32_t max_iter,
                                int32_t precond_kind, const pw_mlp *net, int32_t *converged) {
  PW_CHECK_ARG(b && max_iter >= 1 && (!psi0 || ld), PW_ERR_INVALID, "pw_batch_davidson_run: bad argument");
  if (!psi0)
    for (pw_davidson *d : b->dav)
      PW_CHECK_ARG(dav_inited(d), PW_ERR_INVALID, "pw_batch_davidson_run: without start blocks every solve "
                                                  "must have been initialised");
  std::atomic<int> next{0};
  const int n = (int)b->dav.size();
  const int rc = run_workers(b, [&](int k) {
    for (int t = next.fetch_add(1); t < n; t = next.fetch_add(1)) {
      const int i = b->order[t];
      int r = psi0 ? pw_davidson_init(b->dav[i], psi0[i], ld[i], b->streams[k]) : (int)PW_OK;
      if (r != PW_OK) return r;
      int32_t c = 0;
      r = pw_davidson_run(b->dav[i], max_iter, precond_kind, net, b->streams[k], &c);
      if (r < 0) return r;
      b->conv[i] = c;
    }
    return (int)PW_OK;
  });
  if (rc != PW_OK) return rc;
  bool all = true;
  for (int i = 0; i < n; ++i) {
    if (converged) converged[i] = b->conv[i];
    all = all && b->conv[i];
  }
  return all ? PW_OK : PW_NOT_CONVERGED;
}

pw_status pw_problem_autotune(pw_problem *p, int64_t nbands, int32_t reps, void *scratch,
                              size_t scratch_bytes, void *stream, double *best_ms) {
  PW_CHECK_ARG(p && nbands >= 1 && nbands <= p->max_bands && reps >= 1, PW_ERR_INVALID,
               "pw_problem_autotune: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t ld = (p->npw + 63) / 64 * 64;
  const size_t bytes = (size_t)nbands * ld * sizeof(double2);
  PW_CHECK_ARG(scratch && scratch_bytes >= 2 * bytes, PW_ERR_INVALID,
               "pw_problem_autotune: scratch must hold 2 * nbands * ld * 16 bytes (ld = npw rounded up to 64)");
  void *x = scratch;
  void *y = static_cast<char *>(scratch) + bytes;
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
