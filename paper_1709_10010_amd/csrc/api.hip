// Host side of the C ABI: argument checks, sphere and stick maps, handle
// set-up and the launch sequence of H*psi.  No device code lives here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "common.h"

namespace pw {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int env_switch(const char *name, int dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}
static int env_int(const char *name, int dflt) { return env_switch(name, dflt); }

static void inv3(const double *A, double *Ai) {
  const double a = A[0], b = A[1], c = A[2], d = A[3], e = A[4], f = A[5], g = A[6], h = A[7],
               i = A[8];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  Ai[0] = (e * i - f * h) / det;
  Ai[1] = (c * h - b * i) / det;
  Ai[2] = (b * f - c * e) / det;
  Ai[3] = (f * g - d * i) / det;
  Ai[4] = (a * i - c * g) / det;
  Ai[5] = (c * d - a * f) / det;
  Ai[6] = (d * h - e * g) / det;
  Ai[7] = (b * g - a * h) / det;
  Ai[8] = (a * e - b * d) / det;
}

// Rows b_i of B satisfy a_i . b_j = 2 pi delta_ij:  B = 2 pi inv(A)^T.
static void recip(const double *A, double *B) {
  double Ai[9];
  inv3(A, Ai);
  const double tp = 6.283185307179586476925286766559;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) B[r * 3 + c] = tp * Ai[c * 3 + r];
}

// |k + G|^2 / 2 for Miller triple m (crystal coordinates through B).
static double kin_of(const double *B, const double *k, const int32_t *m) {
  double q[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double c = (double)m[i] + k[i];
    for (int x = 0; x < 3; ++x) q[x] += c * B[i * 3 + x];
  }
  return 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
}

static bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

static size_t cplx_bytes(int prec) { return prec == PW_FP64 ? 16 : 8; }

// Build sticks, tiles and the per-G gather/scatter tables.
static int build_stick_map(pw_problem *p, const int32_t *miller, int ts) {
  const int n0 = p->nr[0], n1 = p->nr[1], n2 = p->nr[2];
  const int64_t npw = p->npw;
  std::vector<int32_t> gx(npw), gy(npw), gz(npw);
  std::vector<uint8_t> occ((size_t)n0 * n1 * n2, 0);
  for (int64_t g = 0; g < npw; ++g) {
    const int32_t *m = miller + 3 * g;
    for (int i = 0; i < 3; ++i)
      PW_CHECK_ARG(2 * std::abs((int64_t)m[i]) < p->nr[i], PW_ERR_SHAPE,
                   "pw_problem_create: Miller index outside |h| < N/2 (sphere does not fit the grid)");
    gx[g] = ((m[0] % n0) + n0) % n0;
    gy[g] = ((m[1] % n1) + n1) % n1;
    gz[g] = ((m[2] % n2) + n2) % n2;
    const size_t cell = ((size_t)gx[g] * n1 + gy[g]) * n2 + gz[g];
    PW_CHECK_ARG(!occ[cell], PW_ERR_INVALID, "pw_problem_create: duplicate Miller triple");
    occ[cell] = 1;
  }
  // sticks: distinct (x, y), ordered by x then y
  std::vector<int32_t> stick_of_xy((size_t)n0 * n1, -1);
  for (int64_t g = 0; g < npw; ++g) stick_of_xy[(size_t)gx[g] * n1 + gy[g]] = 0;
  StickMap &sm = p->map;
  sm.stick_xy.clear();
  for (int x = 0; x < n0; ++x)
    for (int y = 0; y < n1; ++y)
      if (stick_of_xy[(size_t)x * n1 + y] == 0) {
        stick_of_xy[(size_t)x * n1 + y] = (int32_t)sm.stick_xy.size();
        sm.stick_xy.push_back(x * n1 + y);
      }
  sm.nst = (int)sm.stick_xy.size();
  sm.ts = ts;
  sm.ntile = (sm.nst + ts - 1) / ts;
  sm.nst_pad = sm.ntile * ts;
  sm.xlist.clear();
  {
    std::vector<uint8_t> hasx(n0, 0);
    for (int s = 0; s < sm.nst; ++s) hasx[sm.stick_xy[s] / n1] = 1;
    for (int x = 0; x < n0; ++x)
      if (hasx[x]) sm.xlist.push_back(x);
  }
  sm.nx = (int)sm.xlist.size();
  sm.ls = n1 | 1;
  sm.xslot.assign(n0, sm.nx);
  for (int i = 0; i < sm.nx; ++i) sm.xslot[sm.xlist[i]] = i;
  sm.stick_cpos.resize(sm.nst);
  for (int s = 0; s < sm.nst; ++s)
    sm.stick_cpos[s] = sm.xslot[sm.stick_xy[s] / n1] * sm.ls + sm.stick_xy[s] % n1;
  sm.gfull.resize(npw);
  for (int64_t g = 0; g < npw; ++g) sm.gfull[g] = (gx[g] * n1 + gy[g]) * n2 + gz[g];
  sm.stick_cy.clear();
  if (sm.nst <= 32767) {
    sm.stick_cy.assign((size_t)sm.nx * n1, -1);
    for (int s = 0; s < sm.nst; ++s)
      sm.stick_cy[(size_t)sm.xslot[sm.stick_xy[s] / n1] * n1 + sm.stick_xy[s] % n1] = (int16_t)s;
  }
  // entries grouped by tile, then stick, then z
  std::vector<int64_t> key(npw);
  std::vector<int32_t> order(npw);
  for (int64_t g = 0; g < npw; ++g) {
    const int32_t s = stick_of_xy[(size_t)gx[g] * n1 + gy[g]];
    key[g] = (int64_t)s * n2 + gz[g];
    order[g] = (int32_t)g;
  }
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  sm.gidx.assign(npw, 0);
  sm.gpos.assign(npw, 0);
  sm.tile_ptr.assign(sm.ntile + 1, 0);
  for (int64_t e = 0; e < npw; ++e) {
    const int32_t g = order[e];
    const int32_t s = (int32_t)(key[g] / n2);
    const int32_t tile = s / ts;
    sm.gidx[e] = g;
    sm.gpos[e] = gz[g] * ts + (s - tile * ts);
    sm.tile_ptr[tile + 1]++;
  }
  for (int t = 0; t < sm.ntile; ++t) sm.tile_ptr[t + 1] += sm.tile_ptr[t];
  sm.g_linear = true;
  for (int64_t e = 0; e < npw && sm.g_linear; ++e) sm.g_linear = sm.gidx[e] == (int32_t)e;
  return PW_OK;
}

template <typename T>
static void make_twiddles(int n, std::vector<unsigned char> &out) {
  const size_t off = out.size();
  out.resize(off + sizeof(T) * 2 * n);
  T *w = reinterpret_cast<T *>(out.data() + off);
  const long double tp = 6.283185307179586476925286766559L;
  for (int k = 0; k < n; ++k) {
    const long double a = tp * (long double)k / (long double)n;
    w[2 * k] = (T)cosl(a);
    w[2 * k + 1] = (T)(-sinl(a));
  }
}

template <typename T>
static int make_vplanes(pw_problem *p, const std::vector<double> &v) {
  const int n0 = p->nr[0], n1 = p->nr[1], n2 = p->nr[2];
  const double inv = 1.0 / ((double)n0 * n1 * n2);
  std::vector<T> vp((size_t)n0 * n1 * n2);
  for (int x = 0; x < n0; ++x)
    for (int y = 0; y < n1; ++y)
      for (int z = 0; z < n2; ++z)
        vp[((size_t)z * n0 + x) * n1 + y] = (T)(v[((size_t)x * n1 + y) * n2 + z] * inv);
  PW_HIP(hipMemcpy(p->d_vplanes, vp.data(), vp.size() * sizeof(T), hipMemcpyHostToDevice));
  return PW_OK;
}

template <typename V>
static int upload(V **dst, const std::vector<V> &src) {
  if (src.empty()) {
    *dst = nullptr;
    return PW_OK;
  }
  PW_HIP(hipMalloc((void **)dst, src.size() * sizeof(V)));
  PW_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return PW_OK;
}

hipEvent_t Prof::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
void Prof::begin(int stage, hipStream_t s, Pend *out) {
  out->stage = stage;
  out->a = get();
  out->b = get();
  if (out->a) (void)hipEventRecord(out->a, s);
}
void Prof::end(const Pend &p, hipStream_t s) {
  if (!p.a || !p.b) return;
  (void)hipEventRecord(p.b, s);
  pending.push_back(p);
}
int Prof::drain() {
  for (const Pend &p : pending) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&t, p.a, p.b) != hipSuccess)
      return PW_ERR_HIP;
    ms[p.stage] += t;
    cnt[p.stage] += 1;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
  return PW_OK;
}
void Prof::release() {
  (void)drain();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

static void free_problem(pw_problem *p) {
  if (!p) return;
  p->prof.release();
  // the workspace regions belong to the caller
  void *bufs[] = {p->d_gidx,  p->d_gpos,       p->d_tile_ptr, p->d_stick_xy, p->d_xlist,
                  p->d_xslot, p->d_stick_cpos, p->d_kin,      p->d_tw,       p->d_dij,
                  p->d_pj_atom, p->d_proj_off, p->d_dij_off, p->d_stick_cy, p->d_gfull};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete p;
}

// Workspace layout of a problem.  pw_workspace_size runs it with a counting
// Carve; pw_problem_create runs the same take() sequence on the caller's
// workspace to place the handle's buffers.
static void carve_problem(pw_problem *p, Carve &c) {
  const size_t cb = cplx_bytes(p->precision);
  const size_t n3 = (size_t)p->nr[0] * p->nr[1] * p->nr[2];
  p->d_vplanes = c.take<char>(n3 * (p->precision == PW_FP64 ? sizeof(double) : sizeof(float)));
  if (p->nproj > 0) {
    p->d_beta = c.take<char>((size_t)p->nproj * p->ldb * 16);
    if (p->precision != PW_FP64)
      p->d_beta_lp = c.take<char>((size_t)p->nproj * p->ldb * (p->precision == PW_MIXED_FP32 ? 8 : 4));
    const size_t pq = (size_t)p->max_bands * p->nproj * 16;
    p->d_P = c.take<char>(pq);
    p->d_Q = c.take<char>(pq);
    p->part_bytes = std::min<size_t>(32 * pq, (size_t)512 << 20);
    p->d_part = c.take<char>(p->part_bytes);
    if (p->precision == PW_MIXED_BF16) {
      p->d_psi_lp = c.take<char>((size_t)p->max_bands * p->ldb * 4);
      p->d_q_lp = c.take<char>((size_t)p->max_bands * p->nproj * 4);
    }
  }
  p->d_sticks = c.take<char>((size_t)p->nr[2] * p->map.nst_pad * cb * p->band_chunk_max);
  if (p->gen) carve_overlap(p, c);
  p->d_tn = c.take<double>(p->max_bands);
  p->d_rnorm = c.take<double>(p->max_bands);
  p->d_idx = c.take<int>(p->max_bands);
  p->d_bad = c.take<int>(p->max_bands);
}

// Argument checks shared by pw_workspace_size and pw_problem_create, then
// the host-side set-up both need: sizes, reciprocal cell, stick map and the
// sweep height the stick buffer is sized for.
static int prepare_problem(const pw_problem_desc *d, int64_t max_bands, pw_problem *p, const char *who) {
  auto msg = [&](const char *m) { return std::string(who) + ": " + m; };
  PW_CHECK_ARG(d->npw > 0 && d->npw < (int64_t)1 << 31, PW_ERR_INVALID, msg("npw must be in 1 .. 2^31-1"));
  PW_CHECK_ARG(d->miller, PW_ERR_INVALID, msg("miller is null"));
  PW_CHECK_ARG(d->nproj >= 0 && d->natom >= 0, PW_ERR_INVALID, msg("nproj / natom must be >= 0"));
  PW_CHECK_ARG(d->nproj == 0 || (d->proj_offset && d->dij && d->ld_beta >= d->npw), PW_ERR_INVALID,
               msg("beta / proj_offset / dij / ld_beta invalid"));
  PW_CHECK_ARG(max_bands >= 1 && max_bands <= (1 << 20), PW_ERR_INVALID, msg("max_bands must be in 1 .. 2^20"));
  PW_CHECK_ARG(d->precision >= PW_FP64 && d->precision <= PW_MIXED_BF16, PW_ERR_INVALID,
               msg("unknown precision"));
  PW_CHECK_ARG(std::isfinite(d->ecut) && d->ecut > 0, PW_ERR_INVALID, msg("ecut must be > 0"));
  for (int i = 0; i < 3; ++i)
    PW_CHECK_ARG(d->nr[i] >= 2 && d->nr[i] <= 128 && smooth235(d->nr[i]), PW_ERR_SHAPE,
                 msg("grid sizes must be 2^a 3^b 5^c in 2..128"));
  const size_t cb = cplx_bytes(d->precision);
  PW_CHECK_ARG((size_t)d->nr[0] * d->nr[1] * cb + (d->nr[0] + d->nr[1]) * cb + 4 * d->nr[0] <= 160 * 1024,
               PW_ERR_SHAPE, msg("N0*N1 plane does not fit in LDS for this precision"));
  PW_CHECK_ARG((int64_t)d->nr[0] * d->nr[1] <= 8 * 1024, PW_ERR_SHAPE, msg("plane larger than 8192 points"));
  if (d->nproj > 0) {
    PW_CHECK_ARG(d->natom >= 1 && d->proj_offset[0] == 0 && d->proj_offset[d->natom] == d->nproj,
                 PW_ERR_INVALID, msg("proj_offset must run 0 .. nproj"));
    for (int a = 0; a < d->natom; ++a)
      PW_CHECK_ARG(d->proj_offset[a + 1] >= d->proj_offset[a], PW_ERR_INVALID,
                   msg("proj_offset must be non-decreasing"));
  }
  p->precision = d->precision;
  std::memcpy(p->A, d->cell, sizeof p->A);
  std::memcpy(p->kpt, d->kpt, sizeof p->kpt);
  p->ecut = d->ecut;
  std::memcpy(p->nr, d->nr, sizeof p->nr);
  p->npw = d->npw;
  p->nproj = d->nproj;
  p->natom = d->natom;
  p->max_bands = max_bands;
  p->gen = d->qij != nullptr && d->nproj > 0;
  p->ldb = (d->npw + 63) / 64 * 64;
  recip(p->A, p->B);
  const int ts = std::max(1, std::min(64, env_int("PW_STICK_TILE", d->precision == PW_FP64 ? 16 : 32)));
  PW_CHECK_ARG(ts * d->nr[2] <= 8 * 512, PW_ERR_SHAPE, msg("stick tile too long"));
  int rc = build_stick_map(p, d->miller, ts);
  if (rc != PW_OK) return rc;
  // stick buffer: band_chunk x N2 x nst_pad, at most 1 GiB unless PW_BAND_CHUNK asks
  const size_t per_band = (size_t)d->nr[2] * p->map.nst_pad * cb;
  int64_t chunk = env_int("PW_BAND_CHUNK", 0);
  if (chunk <= 0) chunk = std::max<int64_t>(1, std::min<int64_t>(max_bands, ((size_t)1 << 30) / per_band));
  chunk = std::min(chunk, max_bands);
  p->band_chunk = chunk;
  p->band_chunk_max = chunk;
  return PW_OK;
}

}  // namespace pw

using namespace pw;

extern "C" {

const char *pw_last_error(void) { return g_err.c_str(); }

const char *pw_version(void) { return "pwhip 0.1 (gfx950)"; }

pw_status pw_gsphere(const double cell[9], const double kpt[3], double ecut, int32_t *miller_out,
                     int64_t cap, int64_t *npw_out) {
  PW_CHECK_ARG(cell && kpt && npw_out, PW_ERR_INVALID, "pw_gsphere: null argument");
  PW_CHECK_ARG(ecut > 0 && std::isfinite(ecut), PW_ERR_INVALID, "pw_gsphere: ecut must be > 0");
  double B[9];
  recip(cell, B);
  const double qmax = std::sqrt(2.0 * ecut);
  int lo[3], hi[3];
  for (int i = 0; i < 3; ++i) {
    const double an = std::sqrt(cell[3 * i] * cell[3 * i] + cell[3 * i + 1] * cell[3 * i + 1] +
                                cell[3 * i + 2] * cell[3 * i + 2]);
    const double span = qmax * an / 6.283185307179586476925286766559;
    lo[i] = (int)std::floor(-kpt[i] - span) - 1;
    hi[i] = (int)std::ceil(-kpt[i] + span) + 1;
  }
  struct E {
    double key;
    int32_t m[3];
  };
  std::vector<E> v;
  for (int h = lo[0]; h <= hi[0]; ++h)
    for (int k = lo[1]; k <= hi[1]; ++k)
      for (int l = lo[2]; l <= hi[2]; ++l) {
        E e;
        e.m[0] = h;
        e.m[1] = k;
        e.m[2] = l;
        const double t = kin_of(B, kpt, e.m);
        if (t < ecut) {
          char buf[40];
          std::snprintf(buf, sizeof buf, "%.11e", t);  // 12 significant digits
          e.key = std::strtod(buf, nullptr);
          v.push_back(e);
        }
      }
  std::sort(v.begin(), v.end(), [](const E &a, const E &b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.m[0] != b.m[0]) return a.m[0] < b.m[0];
    if (a.m[1] != b.m[1]) return a.m[1] < b.m[1];
    return a.m[2] < b.m[2];
  });
  *npw_out = (int64_t)v.size();
  if (miller_out && cap >= (int64_t)v.size())
    for (size_t g = 0; g < v.size(); ++g)
      for (int i = 0; i < 3; ++i) miller_out[3 * g + i] = v[g].m[i];
  return PW_OK;
}

pw_status pw_workspace_size(const pw_problem_desc *d, int64_t max_bands, size_t *bytes) {
  PW_CHECK_ARG(d && bytes, PW_ERR_INVALID, "pw_workspace_size: null argument");
  *bytes = 0;
  pw_problem p;
  const int rc = prepare_problem(d, max_bands, &p, "pw_workspace_size");
  if (rc != PW_OK) return rc;
  Carve c(nullptr);
  carve_problem(&p, c);
  *bytes = c.size();
  return PW_OK;
}

pw_status pw_problem_create(const pw_problem_desc *d, int64_t max_bands, void *workspace,
                            size_t ws_bytes, void *stream, pw_problem **out) {
  PW_CHECK_ARG(d && out, PW_ERR_INVALID, "pw_problem_create: null argument");
  *out = nullptr;
  PW_CHECK_ARG(d->vloc, PW_ERR_INVALID, "pw_problem_create: vloc is null");
  PW_CHECK_ARG(d->nproj == 0 || d->beta, PW_ERR_INVALID, "pw_problem_create: beta is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  pw_problem *p = new pw_problem();
  int rc = PW_OK;
  auto fail = [&](int code) {
    free_problem(p);
    return code;
  };
  if ((rc = prepare_problem(d, max_bands, p, "pw_problem_create")) != PW_OK) return fail(rc);
  {
    Carve count(nullptr);
    carve_problem(p, count);
    if (!workspace || ws_bytes < count.size() || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
      set_error("pw_problem_create: workspace must be 256-byte aligned device memory of at least "
                "pw_workspace_size() = " + std::to_string(count.size()) + " bytes");
      return fail(PW_ERR_INVALID);
    }
    Carve c(workspace);
    carve_problem(p, c);
    p->ws = workspace;
    p->ws_bytes = ws_bytes;
  }
  (void)hipGetDevice(&p->device);
  const StickMap &sm = p->map;

  // kinetic energies in the caller's G order
  std::vector<double> kin(d->npw);
  for (int64_t g = 0; g < d->npw; ++g) kin[g] = kin_of(p->B, p->kpt, d->miller + 3 * g);
  if ((rc = upload(&p->d_kin, kin)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_gidx, sm.gidx)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_gpos, sm.gpos)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_tile_ptr, sm.tile_ptr)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_stick_xy, sm.stick_xy)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_xlist, sm.xlist)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_xslot, sm.xslot)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_stick_cpos, sm.stick_cpos)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_stick_cy, sm.stick_cy)) != PW_OK) return fail(rc);
  if ((rc = upload(&p->d_gfull, sm.gfull)) != PW_OK) return fail(rc);

  // twiddles (x, y, z back to back) in the FFT precision
  std::vector<unsigned char> tw;
  size_t off[3];
  for (int i = 0; i < 3; ++i) {
    off[i] = tw.size();
    if (d->precision == PW_FP64)
      make_twiddles<double>(d->nr[i], tw);
    else
      make_twiddles<float>(d->nr[i], tw);
  }
  if ((rc = upload(reinterpret_cast<unsigned char **>(&p->d_tw), tw)) != PW_OK) return fail(rc);

  // V_LOC: fetch, reorder to [z][x][y], fold in 1/N^3
  {
    std::vector<double> v((size_t)d->nr[0] * d->nr[1] * d->nr[2]);
    if (hipMemcpyAsync(v.data(), d->vloc, v.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("pw_problem_create: cannot read vloc (device pointer expected)");
      return fail(PW_ERR_HIP);
    }
    for (double x : v)
      if (!std::isfinite(x)) {
        set_error("pw_problem_create: vloc holds a non-finite value");
        return fail(PW_ERR_INVALID);
      }
    double vs = 0.0;
    for (double x : v) vs += x;
    p->vavg = vs / (double)v.size();
    rc = d->precision == PW_FP64 ? make_vplanes<double>(p, v) : make_vplanes<float>(p, v);
    if (rc != PW_OK) return fail(rc);
  }

  // nonlocal data
  if (d->nproj > 0) {
    if (hipMemsetAsync(p->d_beta, 0, (size_t)d->nproj * p->ldb * 16, s) != hipSuccess ||
        hipMemcpy2DAsync(p->d_beta, p->ldb * 16, d->beta, d->ld_beta * 16, d->npw * 16, d->nproj,
                         hipMemcpyDeviceToDevice, s) != hipSuccess) {
      set_error("pw_problem_create: cannot copy beta (device pointer expected)");
      return fail(PW_ERR_HIP);
    }
    if (d->precision != PW_FP64) {
      if ((rc = convert_beta(p->d_beta, p->d_beta_lp, d->nproj * p->ldb, d->precision, s)) != PW_OK) {
        set_error("pw_problem_create: beta conversion failed");
        return fail(rc);
      }
    }
    std::vector<int32_t> pj(d->nproj), poff(d->proj_offset, d->proj_offset + d->natom + 1),
        doff(d->natom);
    int64_t tot = 0;
    for (int a = 0; a < d->natom; ++a) {
      const int na = d->proj_offset[a + 1] - d->proj_offset[a];
      doff[a] = (int32_t)tot;
      tot += (int64_t)na * na;
      for (int j = d->proj_offset[a]; j < d->proj_offset[a + 1]; ++j) pj[j] = a;
    }
    std::vector<double> dij(d->dij, d->dij + tot);
    for (double x : dij)
      if (!std::isfinite(x)) {
        set_error("pw_problem_create: dij holds a non-finite value");
        return fail(PW_ERR_INVALID);
      }
    if ((rc = upload(&p->d_dij, dij)) != PW_OK) return fail(rc);
    if ((rc = upload(&p->d_pj_atom, pj)) != PW_OK) return fail(rc);
    if ((rc = upload(&p->d_proj_off, poff)) != PW_OK) return fail(rc);
    if ((rc = upload(&p->d_dij_off, doff)) != PW_OK) return fail(rc);
    if (p->gen) {
      std::vector<double> q(d->qij, d->qij + tot);
      for (double x : q)
        if (!std::isfinite(x)) {
          set_error("pw_problem_create: qij holds a non-finite value");
          return fail(PW_ERR_INVALID);
        }
      if ((rc = overlap_setup(p, q, poff, s)) != PW_OK) {
        if (rc != PW_ERR_NUMERIC) set_error("pw_problem_create: overlap set-up failed");
        return fail(rc);
      }
    }
  }
  {
    // band indices 0 .. max_bands-1 for the learned preconditioner of pw_precond
    std::vector<int> iota((size_t)max_bands);
    std::iota(iota.begin(), iota.end(), 0);
    if (hipMemcpyAsync(p->d_idx, iota.data(), iota.size() * sizeof(int), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("pw_problem_create: workspace initialisation failed");
      return fail(PW_ERR_HIP);
    }
  }
  p->plane_group = env_int("PW_PLANE_GROUP", 0);  // <= 0: chosen for the plane kernel below

  // device view for the FFT launchers
  FFTDev &f = p->fft;
  f.n0 = d->nr[0];
  f.n1 = d->nr[1];
  f.n2 = d->nr[2];
  f.nst = sm.nst;
  f.ts = sm.ts;
  f.ntile = sm.ntile;
  f.nst_pad = sm.nst_pad;
  f.nx = sm.nx;
  if (!make_axis_plan(f.n0, &f.px) || !make_axis_plan(f.n1, &f.py) || !make_axis_plan(f.n2, &f.pz)) {
    set_error("pw_problem_create: no radix plan for the grid");
    return fail(PW_ERR_SHAPE);
  }
  f.gidx = p->d_gidx;
  f.g_linear = sm.g_linear ? 1 : 0;
  f.gpos = p->d_gpos;
  f.tile_ptr = p->d_tile_ptr;
  f.stick_xy = p->d_stick_xy;
  f.xlist = p->d_xlist;
  f.xslot = p->d_xslot;
  f.stick_cpos = p->d_stick_cpos;
  f.stick_cy = p->d_stick_cy;
  f.tw0 = static_cast<unsigned char *>(p->d_tw) + off[0];
  f.tw1 = static_cast<unsigned char *>(p->d_tw) + off[1];
  f.tw2 = static_cast<unsigned char *>(p->d_tw) + off[2];
  f.vplanes = p->d_vplanes;
  f.kin = p->d_kin;
  p->plane_kernel = plane_kernel_default();
  if (p->plane_group <= 0) p->plane_group = plane_default_group(f, d->precision, p->plane_kernel);
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("pw_problem_create: stream synchronisation failed");
    return fail(PW_ERR_HIP);
  }
  *out = p;
  return PW_OK;
}

pw_status pw_problem_destroy(pw_problem *p) {
  if (p) {
    (void)hipDeviceSynchronize();
    if (p->ace_owner) scf_forget_problem(p->ace_owner, p);
    free_problem(p);
  }
  return PW_OK;
}

pw_status pw_problem_info(const pw_problem *p, int64_t *npw, int64_t *nsticks, int64_t *nproj) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_problem_info: null handle");
  if (npw) *npw = p->npw;
  if (nsticks) *nsticks = p->map.nst;
  if (nproj) *nproj = p->nproj;
  return PW_OK;
}

static int projections_impl(pw_problem *p, const void *psi, int64_t ld, void *P, int64_t nb,
                            hipStream_t s) {
  const int64_t M = p->nproj, N = nb, K = p->npw;
  int splits = p->ksplit > 0 ? p->ksplit : choose_splits(M, N, K);
  while (splits > 1 && (size_t)splits * M * N * 16 > p->part_bytes) --splits;
  const void *A = p->precision == PW_FP64 ? p->d_beta : p->d_beta_lp;
  if (p->precision == PW_MIXED_BF16) {
    // psi rounded once here rather than by every M tile of the GEMM
    const int rc = bf16_round(psi, ld, p->d_psi_lp, p->ldb, K, N, s);
    if (rc != PW_OK) return rc;
    return zgemm_cn_p(p->precision, M, N, K, A, p->ldb, p->d_psi_lp, p->ldb, P, M, splits, p->d_part, s);
  }
  return zgemm_cn_p(p->precision, M, N, K, A, p->ldb, psi, ld, P, M, splits, p->d_part, s);
}

pw_status pw_hpsi(pw_problem *p, const void *psi, int64_t ld_psi, void *hpsi, int64_t ld_hpsi,
                  int64_t nbands, int32_t terms, void *stream) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_hpsi: null handle");
  PW_CHECK_ARG(nbands >= 0 && nbands <= p->max_bands, PW_ERR_INVALID,
               "pw_hpsi: nbands must be in 0 .. max_bands");
  if (nbands == 0) return PW_OK;
  PW_CHECK_ARG(psi && hpsi, PW_ERR_INVALID, "pw_hpsi: null psi / hpsi");
  PW_CHECK_ARG(ld_psi >= p->npw && ld_hpsi >= p->npw, PW_ERR_INVALID, "pw_hpsi: ld < npw");
  PW_CHECK_ARG((terms & ~PW_TERM_ALL) == 0, PW_ERR_INVALID, "pw_hpsi: unknown term bits");
  {
    const char *a0 = static_cast<const char *>(psi), *b0 = static_cast<const char *>(hpsi);
    const char *a1 = a0 + ((nbands - 1) * ld_psi + p->npw) * 16;
    const char *b1 = b0 + ((nbands - 1) * ld_hpsi + p->npw) * 16;
    PW_CHECK_ARG(a1 <= b0 || b1 <= a0, PW_ERR_INVALID, "pw_hpsi: psi and hpsi overlap");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool kinetic = (terms & PW_TERM_KINETIC) != 0;
  int rc;
  if (terms & PW_TERM_LOCAL) {
    for (int64_t b0 = 0; b0 < nbands; b0 += p->band_chunk) {
      const int nb = (int)std::min<int64_t>(p->band_chunk, nbands - b0);
      const double2 *ps = static_cast<const double2 *>(psi) + b0 * ld_psi;
      double2 *hs = static_cast<double2 *>(hpsi) + b0 * ld_hpsi;
      {
        ProfScope ps_(&p->prof, PW_STAGE_ZFFT_INV, s);
        rc = launch_zfft_inv(p->fft, p->precision, ps, ld_psi, p->d_sticks, nb, s);
      }
      if (rc == PW_OK) {
        ProfScope ps_(&p->prof, PW_STAGE_PLANE, s);
        rc = launch_plane(p->fft, p->precision, p->d_sticks, nb, p->plane_group, p->plane_kernel, s);
      }
      if (rc == PW_OK) {
        ProfScope ps_(&p->prof, PW_STAGE_ZFFT_FWD, s);
        rc = launch_zfft_fwd(p->fft, p->precision, p->d_sticks, ps, ld_psi, hs, ld_hpsi, nb,
                             kinetic, s);
      }
      if (rc != PW_OK) {
        set_error("pw_hpsi: local-potential launch failed");
        return rc;
      }
    }
  } else {
    ProfScope ps_(&p->prof, PW_STAGE_KINETIC, s);
    if ((rc = launch_kinetic_only(p->d_kin, psi, ld_psi, hpsi, ld_hpsi, p->npw, (int)nbands,
                                  kinetic, s)) != PW_OK) {
      set_error("pw_hpsi: kinetic launch failed");
      return rc;
    }
  }
  if ((terms & PW_TERM_NONLOCAL) && p->nproj > 0) {
    {
      ProfScope ps_(&p->prof, PW_STAGE_PROJ, s);
      rc = projections_impl(p, psi, ld_psi, p->d_P, nbands, s);
    }
    if (rc == PW_OK) {
      ProfScope ps_(&p->prof, PW_STAGE_DMAT, s);
      rc = launch_apply_d(p->d_dij, p->d_pj_atom, p->d_proj_off, p->d_dij_off, p->d_P, p->d_Q,
                          p->nproj, (int)nbands, s);
    }
    if (rc == PW_OK) {
      ProfScope ps_(&p->prof, PW_STAGE_NLUPD, s);
      const void *A = p->precision == PW_FP64 ? p->d_beta : p->d_beta_lp;
      const void *Q = p->d_Q;
      if (p->precision == PW_MIXED_BF16) {
        rc = bf16_round(p->d_Q, p->nproj, p->d_q_lp, p->nproj, p->nproj, nbands, s);
        Q = p->d_q_lp;
      }
      if (rc == PW_OK)
        rc = zgemm_nn_p(p->precision, p->npw, nbands, p->nproj, 1.0, A, p->ldb, Q, p->nproj, 1.0, hpsi,
                        ld_hpsi, s);
    }
    if (rc != PW_OK) {
      set_error("pw_hpsi: nonlocal launch failed");
      return rc;
    }
  }
  if ((terms & PW_TERM_EXX) && (p->ace_zeta || p->exx_occ)) {
    ProfScope ps_(&p->prof, PW_STAGE_EXX, s);
    rc = p->ace_zeta ? ace_hpsi(p, psi, ld_psi, hpsi, ld_hpsi, nbands, s)
                     : exx_direct_hpsi(p, psi, ld_psi, hpsi, ld_hpsi, nbands, s);
    if (rc != PW_OK) {
      set_error("pw_hpsi: exchange launch failed");
      return rc;
    }
  }
  return PW_OK;
}

pw_status pw_projections(pw_problem *p, const void *psi, int64_t ld_psi, void *proj_out,
                         int64_t nbands, void *stream) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_projections: null handle");
  PW_CHECK_ARG(nbands >= 0 && nbands <= p->max_bands, PW_ERR_INVALID,
               "pw_projections: nbands must be in 0 .. max_bands");
  if (nbands == 0 || p->nproj == 0) return PW_OK;
  PW_CHECK_ARG(psi && proj_out && ld_psi >= p->npw, PW_ERR_INVALID,
               "pw_projections: null pointer or ld < npw");
  const int rc = projections_impl(p, psi, ld_psi, proj_out, nbands, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_projections: launch failed");
  return rc;
}

pw_status pw_precond(pw_problem *p, int32_t kind, const double *theta, const void *x,
                     const void *r, void *t, int64_t ld, int64_t nbands, const pw_mlp *net,
                     void *stream) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_precond: null handle");
  PW_CHECK_ARG(kind == PW_PRECOND_NONE || kind == PW_PRECOND_TPA || kind == PW_PRECOND_MLP, PW_ERR_INVALID,
               "pw_precond: unknown preconditioner kind");
  PW_CHECK_ARG(nbands >= 0 && nbands <= p->max_bands, PW_ERR_INVALID,
               "pw_precond: nbands must be in 0 .. max_bands");
  PW_CHECK_ARG(kind != PW_PRECOND_MLP || (net && theta), PW_ERR_INVALID,
               "pw_precond: the learned preconditioner needs a network and the Ritz values");
  if (nbands == 0) return PW_OK;
  PW_CHECK_ARG(x && r && t && ld >= p->npw, PW_ERR_INVALID, "pw_precond: null pointer or ld < npw");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProfScope ps_(&p->prof, PW_STAGE_PRECOND, s);
  int rc;
  if (kind == PW_PRECOND_MLP) {
    // features need T_n of the iterate and |r_n|; bands whose scales come
    // out non-finite are redone with TPA
    const double2 *R = static_cast<const double2 *>(r);
    double2 *T = static_cast<double2 *>(t);
    rc = band_kinetic(p->d_kin, x, ld, p->npw, (int)nbands, p->d_tn, s);
    if (rc == PW_OK) rc = col_norms(R, ld, p->npw, (int)nbands, p->d_rnorm, s);
    if (rc == PW_OK && hipMemsetAsync(p->d_bad, 0, (size_t)nbands * sizeof(int), s) != hipSuccess)
      rc = PW_ERR_HIP;
    if (rc == PW_OK)
      rc = mlp_precond_idx(net, p, theta, p->d_rnorm, p->d_idx, R, ld, T, (int)nbands, p->d_bad, p->d_tn, s);
    if (rc == PW_OK) rc = mlp_fallback(p->d_bad, p, p->d_tn, p->d_idx, R, ld, T, (int)nbands, s);
  } else {
    rc = launch_tpa(p->d_kin, x, r, t, ld, p->npw, (int)nbands, kind, p->d_tn, s);
  }
  if (rc != PW_OK) set_error("pw_precond: launch failed");
  return rc;
}

pw_status pw_profile_enable(pw_problem *p, int32_t on) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_profile_enable: null handle");
  p->prof.on = on != 0;
  return PW_OK;
}

pw_status pw_profile_read(pw_problem *p, double *ms_total, int64_t *launches, int32_t reset) {
  PW_CHECK_ARG(p, PW_ERR_INVALID, "pw_profile_read: null handle");
  const int rc = p->prof.drain();
  if (rc != PW_OK) {
    set_error("pw_profile_read: event synchronisation failed");
    return rc;
  }
  for (int i = 0; i < PW_NSTAGES; ++i) {
    if (ms_total) ms_total[i] = p->prof.ms[i];
    if (launches) launches[i] = p->prof.cnt[i];
    if (reset) {
      p->prof.ms[i] = 0.0;
      p->prof.cnt[i] = 0;
    }
  }
  return PW_OK;
}

}  // extern "C"
