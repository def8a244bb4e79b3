// Host side of the C ABI: validation, the closed-form partition, workspace
// layout, and the orchestration of setup (Alg. 1), operator application
// (Alg. 2, eqs. addSW / balSW) and the outer iterations (Alg. 3, PCG), for a
// batch of independent grids (a single grid is the batch of one).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <limits>
#include <functional>
#include <map>
#include <mutex>

#include "../../include/sfcdd.h"
#include "common.h"
#include "kernels.h"

using namespace sfcdd;

namespace {

thread_local std::string g_last_error;

struct Region {
  size_t off = 0, bytes = 0;
};

// Workspace carving: every region 256-byte aligned.
struct Planner {
  size_t top = 0;
  Region take(size_t bytes) {
    Region r;
    r.off = (top + 255) & ~size_t(255);
    r.bytes = bytes;
    top = r.off + bytes;
    return r;
  }
};

enum { V_X = 0, V_R, V_Z, V_P, V_Q, V_T, V_W, V_Y, V_V, V_IN, V_OUT, V_B, V_TMP, NVEC };

// One grid of the batch on the host.
struct GridHost {
  GridDesc desc{};
  std::vector<double> coeff;
  std::vector<int32_t> ta, Ni;
  std::vector<double> omega;
};

}  // namespace

struct sfcdd_ctx {
  int G = 0;
  std::vector<GridHost> grid;
  int weighting = 1, variant = 1, fdtype = 0, local_solver = 0, layout = 0;
  int local_order = SFCDD_ORDER_DIAGONAL;  // elimination order of the subdomain matrices
  int coarse_split = SFCDD_SPLIT_AUTO;     // dissection of a single dense coarse matrix
  int nd[3] = {0, 0, 0};                   // its tiles: first half, second half, separator
  int64_t Ntot = 0, N0tot = 0;
  int Ptot = 0, dmax = 0, duni = 0, rbx = RED_BLOCKS;
  int max_cblock = 1;  // largest coarse block (points) of any grid
  bool coarse32 = false;  // FP32 coarse Cholesky factor (see coarse_fp32_ok)
  bool coarse_x32 = false;  // FP32 coarse inverse X_0 (FP32 subdomain factors, automatic coarse precision)
  // iterative coarse solve (single grid): A_0 in ELL form (ic_kw entries per
  // row, rows padded to ic_ld = ic_nt 64-blocks), the explicit FP32 inverses of
  // its diagonal 64-blocks, and the inner CG's vectors; the dense coarse
  // regions hold the aggregated second level
  bool coarse_iter = false;
  double ic_tol2 = 1e-20;
  int ic_kw = 0, ic_nt = 0, ic_nq = 0;
  int64_t ic_ld = 0;
  int ic_k = 0;              // inner step budget of one coarse solve
  int ic_max_steps = 0, ic_unconv = 0;  // statistics of the current sfcdd_solve
  int32_t *ideg = nullptr, *icol = nullptr, *ibjnt = nullptr, *iflag = nullptr;
  int64_t* ibjoff = nullptr;
  double *ival = nullptr, *ibjt = nullptr, *ir = nullptr, *ip = nullptr, *iq = nullptr, *iz1 = nullptr;
  double *icagg = nullptr, *idagg = nullptr, *iqpart = nullptr, *ipart = nullptr;
  float* ibjm = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // internal per-device stream (default priority): the coarse setup
                               // overlaps the fine factorisation; shared by the contexts of a device
  // per-subdomain (batch-global) host tables
  std::vector<int32_t> ta, Ni, nt;
  std::vector<int64_t> off, doff, xoff, poff;
  std::vector<double> omega;
  std::vector<uint16_t> sgid;
  // coarse matrices, one per grid
  std::vector<int32_t> c_nt, c_n;
  std::vector<int64_t> c_off, c_xoff, c_poff, c_doff, c_toff;
  int max_nt = 0, max_Ni = 0, min_Ni = 0, max_nt0 = 0, max_N0 = 0;
  int64_t maxN = 1;  // points of the largest grid
  int64_t sum_Ni = 0, tiles = 0, parts = 0, xlen = 0, ctiles = 0, cparts = 0, c0len = 0;
  int64_t ctinv = 0;  // tiles of the coarse inversion workspace (all grids)
  int trsv_waves = 16;
  int trsv_stream = -1;  // non-temporal factor loads: -1 by the size rule, 0 off, 1 on (autotuned)
  int spmv_u = 2, spmv_win = 512;   // SpMV launch shape: points per thread, window 256 u (autotuned)
  int factor_rows = 0, factor_pair = -1;  // batched factorisation shape (0 / -1: rules)
  // workspace regions
  Region r_sfc, r_pos, r_nbr, r_gid, r_grids, r_ta, r_Ni, r_nt, r_off, r_doff, r_xoff, r_poff,
      r_omega, r_sgid, r_fac, r_facX, r_xloc, r_fpart, r_A0, r_X0, r_c0, r_d0, r_cpart, r_cpartk,
      r_cmeta, r_cgid, r_ctgid, r_cy, r_dbuf, r_vec, r_partials, r_scal, r_active, r_status, r_gout,
      r_ideg, r_icol, r_ival, r_ibjt, r_ibjm, r_ibjnt, r_ibjoff, r_ivec, r_icagg, r_idagg, r_iqpart, r_ipart,
      r_lperm, r_liperm, r_tlo, r_trb, r_gtiles, r_ztile, r_cperm, r_ccen, r_cfnz, r_clo, r_crb;
  size_t total = 0;
  unsigned char* ws = nullptr;
  // device pointers
  int32_t *sfc_index = nullptr, *pos = nullptr, *nbr = nullptr;
  uint16_t *gid = nullptr, *d_sgid = nullptr, *cgid = nullptr, *ctgid = nullptr;
  GridDesc* d_grids = nullptr;
  int32_t *d_ta = nullptr, *d_Ni = nullptr, *d_nt = nullptr;
  int64_t *d_off = nullptr, *d_doff = nullptr, *d_xoff = nullptr, *d_poff = nullptr;
  double* d_omega = nullptr;
  // local elimination order and tile envelopes of the subdomain factors
  int32_t *lperm = nullptr, *liperm = nullptr, *tlo = nullptr, *trb = nullptr;
  unsigned long long* gtiles = nullptr;   // per grid: tiles stored, entries per sweep, tile products
  void* ztile = nullptr;                  // a tile of zeros (the substitution kernel's unused slots)
  // coarse elimination order and the envelopes of the dense coarse factors
  int32_t *cperm = nullptr, *ccen = nullptr, *cfnz = nullptr, *clo = nullptr, *crb = nullptr;
  void *fac = nullptr, *facX = nullptr, *xloc = nullptr, *fpart = nullptr;
  double *A0 = nullptr, *X0 = nullptr, *c0 = nullptr, *d0 = nullptr, *cpart = nullptr;
  double* cy = nullptr;  // tile-padded coarse vector X_0 R_0 v between the two products
  double* cpartk = nullptr;  // split-K partial tiles of a single coarse factorisation
  int32_t *dc_nt = nullptr, *dc_n = nullptr;
  int64_t *dc_off = nullptr, *dc_xoff = nullptr, *dc_poff = nullptr, *dc_doff = nullptr;
  int64_t* dc_toff = nullptr;  // first tile of each coarse matrix's inversion workspace
  double* dbuf = nullptr;
  double* vec[NVEC] = {};
  double *partials = nullptr, *scal = nullptr, *gout = nullptr;
  int32_t *active = nullptr, *status = nullptr;
  double* host_scal = nullptr;  // pinned: an image of the workspace bytes from the scalars
                                // to the end of the flags (rb_bytes; flags at byte rb_flags),
                                // then the flag upload buffer (G int32 at byte hb_off)
  // allocation-free context (sfcdd_setup_noalloc): the workspace is the device's
  // static array, host_scal points into this pageable buffer, and the context
  // is valid while no later allocation-free setup on its device has run
  bool noalloc = false;
  int noalloc_dev = -1;
  uint64_t noalloc_gen = 0;
  std::vector<unsigned char> host_pageable;
  size_t rb_bytes = 0, rb_flags = 0, hb_off = 0;
  size_t hnd_off = 0;  // byte offset in host_scal of the coarse dissection readback (4 int32)
  std::vector<int32_t> last_iters;
  hipEvent_t ev_rb = nullptr;  // readback of the per-iteration scalars
  // host copy of the device activity flags (valid after the first upload)
  std::vector<int32_t> active_shadow;
  std::vector<int64_t> gfac_bytes;  // subdomain factor bytes per grid
  bool active_valid = false, active_in_flight = false;
  std::vector<double> last_relres;
  std::string err;
  sfcdd_info info{};
  // per-kernel profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double k_ms[SFCDD_K_COUNT] = {};
  int64_t k_n[SFCDD_K_COUNT] = {};

  Batch batch() const {
    Batch B;
    B.grids = d_grids;
    B.G = G;
    B.dmax = dmax;
    B.duni = duni;
    B.Ntot = Ntot;
    B.Ptot = Ptot;
    B.N0tot = N0tot;
    B.gid = gid;
    B.sgid = d_sgid;
    B.cgid = cgid;
    B.ctgid = ctgid;
    B.rbx = rbx;
    B.spmv_u = spmv_u;
    B.maxN = maxN;
    B.cperm = cperm;
    return B;
  }
};

#define FAIL(ctx, code, ...)                                   \
  do {                                                         \
    char _b[512];                                              \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                     \
    if (ctx) (ctx)->err = _b; else g_last_error = _b;          \
    return code;                                               \
  } while (0)

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t _e = (call);                                                                    \
    if (_e != hipSuccess) FAIL(ctx, SFCDD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
  } while (0)

namespace {
bool noalloc_stale(const sfcdd_ctx* c);
}  // namespace

// A context from sfcdd_setup_noalloc whose device workspace a later
// allocation-free setup has taken over may not run device work.
#define LIVE(ctx)                                                                             \
  do {                                                                                        \
    if (noalloc_stale(ctx))                                                                   \
      FAIL(ctx, SFCDD_EINVAL, "allocation-free context superseded by a later "                \
           "sfcdd_setup_noalloc on its device");                                              \
  } while (0)

namespace {

// Event pair around one timed launch (no-op unless profiling is on).
struct ProfScope {
  sfcdd_ctx* c;
  int kind;
  size_t idx = SIZE_MAX;
  ProfScope(sfcdd_ctx* c_, int kind_) : c(c_), kind(kind_) {
    if (!c->prof) return;
    if (c->ev_used + 2 > c->ev_pool.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->ev_pool.push_back(e);
        c->ev_kind.push_back(0);
      }
    }
    idx = c->ev_used;
    c->ev_used += 2;
    c->ev_kind[idx] = kind;
    (void)hipEventRecord(c->ev_pool[idx], c->stream);
  }
  ~ProfScope() {
    if (idx != SIZE_MAX) (void)hipEventRecord(c->ev_pool[idx + 1], c->stream);
  }
};

// Folds the recorded event pairs into the per-kernel totals (stream must be idle).
void prof_collect(sfcdd_ctx* c) {
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]) == hipSuccess) {
      c->k_ms[c->ev_kind[i]] += ms;
      c->k_n[c->ev_kind[i]] += 1;
    }
  }
  c->ev_used = 0;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Validation and host partition of one grid (eqs. dof, sloc, enlarge, omegai,
// restr).  err receives the message on failure.
sfcdd_status plan_grid(GridHost& h, const sfcdd_params* p, std::string& err) {
  char buf[512];
#define GFAIL(code, ...)                     \
  do {                                       \
    snprintf(buf, sizeof(buf), __VA_ARGS__); \
    err = buf;                               \
    return code;                             \
  } while (0)
  if (!p) GFAIL(SFCDD_EINVAL, "params is NULL");
  if (p->d < 1 || p->d > MAXD) GFAIL(SFCDD_EINVAL, "d = %d out of range 1..%d", p->d, MAXD);
  if ((p->level == nullptr) == (p->npts == nullptr)) GFAIL(SFCDD_EINVAL, "give exactly one of level / npts");
  GridDesc& g = h.desc;
  memset(&g, 0, sizeof(g));
  g.d = p->d;
  int nres = 0;
  for (int j = 0; j < p->d; ++j) {
    int n;
    if (p->level) {
      const int l = p->level[j];
      if (l < 1 || l > 30) GFAIL(SFCDD_EINVAL, "level[%d] = %d out of range 1..30", j, l);
      n = (1 << l) - 1;
      nres = std::max(nres, l);
    } else {
      n = p->npts[j];
      if (n < 1) GFAIL(SFCDD_EINVAL, "npts[%d] = %d < 1", j, n);
    }
    g.n[j] = n;
  }
  if (!p->level) {
    int mx = 0;
    for (int j = 0; j < p->d; ++j) mx = std::max(mx, g.n[j]);
    while ((int64_t(1) << nres) < (int64_t)mx + 1) ++nres;
    if (nres < 1) nres = 1;
  }
  if ((int64_t)nres * p->d > 64) GFAIL(SFCDD_EOVERFLOW, "Morton key needs %d bits > 64", nres * p->d);
  g.nres = nres;
  int64_t N = 1;
  for (int j = 0; j < p->d; ++j) {
    g.stride[j] = N;
    N *= g.n[j];
    if (N >= (int64_t(1) << 31)) GFAIL(SFCDD_EOVERFLOW, "N >= 2^31");
    g.shift[j] = p->level ? nres - p->level[j] : 0;
  }
  g.N = N;
  h.coeff.assign(p->d, 1.0);
  if (p->coeff)
    for (int j = 0; j < p->d; ++j) {
      if (!(p->coeff[j] > 0.0) || !std::isfinite(p->coeff[j]))
        GFAIL(SFCDD_EINVAL, "coeff[%d] must be positive and finite", j);
      h.coeff[j] = p->coeff[j];
    }
  double diag = 0.0;
  for (int j = 0; j < p->d; ++j) {
    const double ih2 = (double)((int64_t)(g.n[j] + 1) * (g.n[j] + 1));
    g.inv_h2[j] = ih2;
    g.c[j] = h.coeff[j] * ih2;
    diag += 2.0 * g.c[j];
  }
  g.diag = diag;
  if (p->P < 1 || p->P > N) GFAIL(SFCDD_EINVAL, "P = %d must satisfy 1 <= P <= N = %lld", p->P, (long long)N);
  if (p->gamma_den < 1 || p->gamma_den > (int64_t(1) << 30) || p->gamma_num < 0)
    GFAIL(SFCDD_EINVAL, "gamma = %lld/%lld must be >= 0 with 1 <= den <= 2^30",
          (long long)p->gamma_num, (long long)p->gamma_den);
  if (p->weighting != SFCDD_WEIGHT_NONE && p->weighting != SFCDD_WEIGHT_OMEGA && p->weighting != SFCDD_WEIGHT_D)
    GFAIL(SFCDD_EINVAL, "weighting = %d", p->weighting);
  if (p->variant != SFCDD_ADDITIVE && p->variant != SFCDD_BALANCED && p->variant != SFCDD_DEFLATED)
    GFAIL(SFCDD_EINVAL, "variant = %d", p->variant);
  if (p->factor_dtype != SFCDD_FP64 && p->factor_dtype != SFCDD_FP32)
    GFAIL(SFCDD_EINVAL, "factor_dtype = %d", p->factor_dtype);
  if (p->local_solver != SFCDD_LOCAL_CHOLESKY && p->local_solver != SFCDD_LOCAL_INVERSE)
    GFAIL(SFCDD_EINVAL, "local_solver = %d", p->local_solver);
  if (p->layout != 0 && p->layout != 1) GFAIL(SFCDD_EINVAL, "layout = %d", p->layout);
  if (p->coarse_precision != SFCDD_COARSE_AUTO && p->coarse_precision != SFCDD_COARSE_FP64)
    GFAIL(SFCDD_EINVAL, "coarse_precision = %d", p->coarse_precision);
  if (p->curve != SFCDD_CURVE_ZORDER && p->curve != SFCDD_CURVE_HILBERT)
    GFAIL(SFCDD_EINVAL, "curve = %d", p->curve);
  if (p->local_order != SFCDD_ORDER_DIAGONAL && p->local_order != SFCDD_ORDER_CURVE &&
      p->local_order != SFCDD_ORDER_DENSE)
    GFAIL(SFCDD_EINVAL, "local_order = %d", p->local_order);
  if (p->coarse_split != SFCDD_SPLIT_AUTO && p->coarse_split != SFCDD_SPLIT_OFF)
    GFAIL(SFCDD_EINVAL, "coarse_split = %d", p->coarse_split);
  g.curve = p->curve;

  if (p->coarse_solver != SFCDD_COARSE_DENSE && p->coarse_solver != SFCDD_COARSE_ITERATIVE)
    GFAIL(SFCDD_EINVAL, "coarse_solver = %d", p->coarse_solver);
  const bool iter = p->coarse_solver == SFCDD_COARSE_ITERATIVE;
  if (iter && !(p->coarse_tol >= 0.0 && p->coarse_tol < 1.0))
    GFAIL(SFCDD_EINVAL, "coarse_tol = %g must lie in [0, 1)", p->coarse_tol);
  const int P = p->P;
  const int64_t base = N / P, rem = N % P;
  // coarse points per subdomain
  int q = p->q;
  if (q == 0) {
    // floor(log2(N/P)) = floor(log2(floor(N/P))) for N >= P
    int e = -4;
    for (int64_t v = base; v > 1; v >>= 1) ++e;
    if (e < 0) e = 0;
    int64_t qq = int64_t(1) << e;
    if (!iter) qq = std::min<int64_t>(qq, std::max<int64_t>(1, 16384 / P));
    qq = std::min<int64_t>(qq, base);
    q = (int)std::max<int64_t>(1, qq);
  }
  if (q < 1 || q > base) GFAIL(SFCDD_EINVAL, "q = %d must satisfy 1 <= q <= floor(N/P) = %lld", q, (long long)base);
  const int64_t n0max = iter ? (int64_t(1) << 22) : (int64_t(1) << 17);
  if ((int64_t)q * P > n0max)
    GFAIL(SFCDD_EINVAL, "coarse size qP = %lld exceeds %lld", (long long)q * P, (long long)n0max);
  g.P = P;
  g.q = q;
  g.N0 = q * P;
  g.nt0 = (int)ceil_div(g.N0, TS);
  g.base = base;
  g.rem = rem;
  // dense coarse level: A_0 itself, or (iterative) its aggregation over
  // groups of TS consecutive coarse unknowns
  g.agg = iter ? TS : 1;
  g.N0d = (int)ceil_div(g.N0, g.agg);
  g.nt0d = (int)ceil_div(g.N0d, TS);

  // overlapping subdomains, eq. (enlarge), cyclic closure
  const int64_t F = p->gamma_num / p->gamma_den;
  const int64_t enm = p->gamma_num - F * p->gamma_den;  // eta = enm / gden
  auto size_of = [&](int64_t i) -> int64_t {
    i %= P;
    if (i < 0) i += P;
    return base + (i < rem ? 1 : 0);
  };
  auto start_of = [&](int64_t i) -> int64_t {
    i %= P;
    if (i < 0) i += P;
    return piece_start((int)i, base, rem);
  };
  h.ta.assign(P, 0);
  h.Ni.assign(P, 0);
  for (int i = 0; i < P; ++i) {
    int64_t len;
    int64_t nl = 0;
    if (2 * F + 1 >= P) {
      len = N;
    } else {
      nl = (enm * size_of(i - F - 1) + p->gamma_den - 1) / p->gamma_den;
      const int64_t nr = (enm * size_of(i + F + 1)) / p->gamma_den;
      len = nl + nr;
      for (int64_t k = -F; k <= F; ++k) len += size_of(i + k);
    }
    if (len >= N) {
      h.ta[i] = 0;
      h.Ni[i] = (int32_t)N;
    } else {
      int64_t t = (start_of(i - F) - nl) % N;
      if (t < 0) t += N;
      h.ta[i] = (int32_t)t;
      h.Ni[i] = (int32_t)len;
    }
  }
  g.F = (int)std::min<int64_t>(F, P);
  g.ncand = (int)std::min<int64_t>(P, 2 * F + 3);
  // multiplicities and omega_i = 1 / min_{p in Omega_i} m_p (eq. omegai).
  // m is constant between subdomain ends, so it is kept as at most 2P + 1
  // runs (start position, value) and each subdomain takes the minimum over
  // the runs its cyclic range meets: O(P log P + sum of runs met), not O(N).
  h.omega.assign(P, 1.0);
  if (p->weighting == SFCDD_WEIGHT_OMEGA) {
    std::vector<std::pair<int64_t, int32_t>> ev;  // (position, change of m)
    ev.reserve(4 * (size_t)P + 1);
    ev.emplace_back(0, 0);
    for (int i = 0; i < P; ++i) {
      const int64_t a = h.ta[i], e = a + h.Ni[i];
      ev.emplace_back(a, 1);
      if (e <= N) {
        ev.emplace_back(e, -1);
      } else {
        ev.emplace_back(N, -1);
        ev.emplace_back(0, 1);
        ev.emplace_back(e - N, -1);
      }
    }
    std::sort(ev.begin(), ev.end());
    std::vector<int64_t> rs;  // run starts, strictly increasing, rs[0] = 0, all < N
    std::vector<int32_t> rv;  // m on [rs[k], rs[k + 1])
    int32_t cur = 0;
    for (size_t k = 0; k < ev.size();) {
      const int64_t pos = ev[k].first;
      for (; k < ev.size() && ev[k].first == pos; ++k) cur += ev[k].second;
      if (pos >= N) break;
      rs.push_back(pos);
      rv.push_back(cur);
    }
    auto run_min = [&](int64_t lo, int64_t hi, int32_t mn) {  // min over [lo, hi), 0 <= lo < hi <= N
      size_t k = (size_t)(std::upper_bound(rs.begin(), rs.end(), lo) - rs.begin()) - 1;
      for (; k < rs.size() && rs[k] < hi; ++k) mn = std::min(mn, rv[k]);
      return mn;
    };
    for (int i = 0; i < P; ++i) {
      const int64_t a = h.ta[i], e = a + h.Ni[i];
      int32_t mn = run_min(a, std::min<int64_t>(e, N), INT32_MAX);
      if (e > N) mn = run_min(0, e - N, mn);
      h.omega[i] = 1.0 / (double)mn;
    }
  }
  for (int i = 0; i < P; ++i)
    if ((int64_t)ceil_div(h.Ni[i], TS) * TS > 8192)
      GFAIL(SFCDD_EINVAL, "subdomain N_i = %d exceeds 8192 points", h.Ni[i]);
  return SFCDD_OK;
#undef GFAIL
}

// Bound on the condition number of a coarse matrix: with R_0 R_0^T =
// diag(block sizes), the Rayleigh quotients of A_0 = R_0 A R_0^T lie in
// [lambda_min(A) b_min, lambda_max(A) b_max], so kappa(A_0) <= kappa(A)
// b_max / b_min, with the stencil's extreme eigenvalues
// sum_j (a_j / h_j^2) 4 sin^2(k pi h_j / 2), k = 1 and n_j.  Pieces of
// floor(N/P) or that + 1 points are cut into q blocks of near-equal size.
double coarse_kappa_bound(const GridDesc& gd) {
  const double pi = 3.14159265358979323846;
  double lmin = 0.0, lmax = 0.0;
  for (int j = 0; j < gd.d; ++j) {
    const double t = pi / (2.0 * (gd.n[j] + 1));
    lmin += gd.c[j] * 4.0 * std::sin(t) * std::sin(t);
    lmax += gd.c[j] * 4.0 * std::cos(t) * std::cos(t);
  }
  const double bmin = (double)std::max<int64_t>(1, gd.base / gd.q);
  const double bmax = (double)ceil_div(gd.base + 1, (int64_t)gd.q);
  return lmax / lmin * bmax / bmin;
}

// The coarse factorisation may run in FP32 (beside FP32 subdomain factors)
// when every coarse matrix of the context is well conditioned: solves with
// an FP32 Cholesky factor are accurate to about kappa * 6e-8, so the bound
// 4096 keeps them within a few 1e-4 (the 8192 coarse unknowns of the
// (7,6,5) grid with 256 subdomains: bound 3.0e3, kappa(A_0) = 99, error
// about 2e-7), an error of the order the FP32 subdomain solves already make
// (their matrices are principal submatrices of A, kappa(A_i) <= kappa(A)).
constexpr double COARSE32_KAPPA = 4096.0;
bool coarse_fp32_ok(const sfcdd_ctx* c) {
  for (int k = 0; k < c->G; ++k)
    if (!(coarse_kappa_bound(c->grid[k].desc) <= COARSE32_KAPPA)) return false;
  return true;
}

// Plans the whole batch: per-grid partitions, batch placement, workspace.
sfcdd_status plan(sfcdd_ctx* c, int G, const sfcdd_params* params) {
  if (G < 1 || G > 65535) FAIL(c, SFCDD_EINVAL, "number of grids %d out of range 1..65535", G);
  if (!params) FAIL(c, SFCDD_EINVAL, "params is NULL");
  c->G = G;
  c->grid.assign(G, GridHost());
  for (int k = 0; k < G; ++k) {
    std::string e;
    const sfcdd_status st = plan_grid(c->grid[k], &params[k], e);
    if (st != SFCDD_OK) {
      if (G > 1) e = "grid " + std::to_string(k) + ": " + e;
      FAIL(c, st, "%s", e.c_str());
    }
    if (params[k].weighting != params[0].weighting || params[k].variant != params[0].variant ||
        params[k].factor_dtype != params[0].factor_dtype ||
        params[k].local_solver != params[0].local_solver || params[k].layout != params[0].layout ||
        params[k].coarse_precision != params[0].coarse_precision ||
        params[k].local_order != params[0].local_order)
      FAIL(c, SFCDD_EINVAL, "grid %d: weighting, variant, factor_dtype, local_solver, layout, local_order and "
           "coarse_precision must be the same for every grid of a batch", k);
    if (params[k].coarse_solver == SFCDD_COARSE_ITERATIVE && G > 1)
      FAIL(c, SFCDD_EINVAL, "grid %d: the iterative coarse solver is for single grids", k);
  }
  c->weighting = params[0].weighting;
  c->variant = params[0].variant;
  c->fdtype = params[0].factor_dtype;
  c->local_solver = params[0].local_solver;
  c->local_order = c->local_solver == SFCDD_LOCAL_INVERSE ? SFCDD_ORDER_DENSE : params[0].local_order;
  c->coarse_split = params[0].coarse_split;
  c->layout = params[0].layout;
  c->coarse_iter = params[0].coarse_solver == SFCDD_COARSE_ITERATIVE;
  if (c->coarse_iter) {
    const double t = params[0].coarse_tol > 0.0 ? params[0].coarse_tol : 1e-6;
    c->ic_tol2 = t * t;
  }
  // batch placement
  int64_t goff = 0, c0off = 0, c0pad = 0;
  int soff = 0;
  c->dmax = 0;
  c->ta.clear(); c->Ni.clear(); c->nt.clear(); c->off.clear(); c->doff.clear();
  c->xoff.clear(); c->poff.clear(); c->omega.clear(); c->sgid.clear();
  c->c_nt.clear(); c->c_n.clear(); c->c_off.clear(); c->c_xoff.clear(); c->c_poff.clear();
  c->c_doff.clear(); c->c_toff.clear();
  int64_t toff = 0, dof = 0, xof = 0, pof = 0, ctoff = 0, cpof = 0, ctt = 0;
  c->max_nt = 0; c->max_Ni = 0; c->min_Ni = INT32_MAX; c->max_nt0 = 0; c->max_N0 = 0;
  c->gfac_bytes.assign(G, 0);
  for (int k = 0; k < G; ++k) {
    GridHost& h = c->grid[k];
    GridDesc& g = h.desc;
    const int64_t toff0 = toff;
    g.goff = goff;
    g.soff = soff;
    g.c0off = c0off;
    g.c0pad = c0pad;
    goff += g.N;
    soff += g.P;
    c0off += g.N0;
    c0pad += (int64_t)g.nt0 * TS;
    c->dmax = std::max(c->dmax, g.d);
    for (int i = 0; i < g.P; ++i) {
      const int ntb = (int)ceil_div(h.Ni[i], TS);
      c->ta.push_back(h.ta[i]);
      c->Ni.push_back(h.Ni[i]);
      c->nt.push_back(ntb);
      c->off.push_back(toff);
      c->doff.push_back(dof);
      c->xoff.push_back(xof);
      c->poff.push_back(pof);
      c->omega.push_back(h.omega[i]);
      c->sgid.push_back((uint16_t)k);
      toff += (int64_t)ntb * (ntb + 1) / 2;
      dof += h.Ni[i];
      xof += (int64_t)ntb * TS;
      pof += (int64_t)ntb * ntb * TS;
      c->max_nt = std::max(c->max_nt, ntb);
      c->max_Ni = std::max(c->max_Ni, h.Ni[i]);
      c->min_Ni = std::min(c->min_Ni, h.Ni[i]);
    }
    c->gfac_bytes[k] = (toff - toff0) * TS2 * (c->fdtype == SFCDD_FP32 ? 4 : 8);  // until the envelopes are known
    // the dense coarse level (A_0, or its aggregation for the iterative solve)
    c->c_nt.push_back(g.nt0d);
    c->c_n.push_back(g.N0d);
    c->c_off.push_back(ctoff);
    c->c_xoff.push_back(g.c0pad);
    c->c_poff.push_back(cpof);
    c->c_doff.push_back(g.c0off);
    c->c_toff.push_back(ctt);
    ctt += ((int64_t)g.nt0d * g.nt0d + 3) / 4;
    ctoff += (int64_t)g.nt0d * (g.nt0d + 1) / 2;
    cpof += (int64_t)g.nt0d * g.nt0d * TS;
    c->max_nt0 = std::max(c->max_nt0, g.nt0d);
    c->max_N0 = std::max(c->max_N0, g.N0d);
  }
  // the substitution kernel stages the subdomain's right-hand side in LDS
  if (c->local_solver == SFCDD_LOCAL_CHOLESKY && !trsv_fits(c->max_nt, c->fdtype == SFCDD_FP32 ? 4 : 8, 4))
    FAIL(c, SFCDD_EINVAL, "a subdomain of %d points is too large for the substitution kernel (%s factors)",
         c->max_Ni, c->fdtype == SFCDD_FP32 ? "FP32" : "FP64");
  // subdomains of at most eight tile rows: four waves per workgroup (a wider
  // workgroup splits too short a row of tiles and idles most of its waves)
  c->trsv_waves = c->max_nt <= 8 ? 4 : 16;
  c->duni = c->grid[0].desc.d;
  for (int k = 1; k < G; ++k)
    if (c->grid[k].desc.d != c->duni) c->duni = 0;
  c->Ntot = goff;
  if (c->Ntot >= (int64_t(1) << 31)) FAIL(c, SFCDD_EOVERFLOW, "total size of the batch >= 2^31");
  c->Ptot = soff;
  c->N0tot = c0off;
  c->c0len = c0pad;
  c->tiles = toff;
  c->sum_Ni = dof;
  c->xlen = xof;
  c->parts = pof;
  c->ctiles = ctoff;
  c->cparts = cpof;
  c->ctinv = ctt;
  // reduction blocks per grid: one pass of RED_THREADS per point of the
  // largest grid (so that every point has its own thread), at most RED_BLOCKS
  int64_t maxN = 1;
  for (int k = 0; k < G; ++k) maxN = std::max<int64_t>(maxN, c->grid[k].desc.N);
  c->rbx = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(8, ceil_div(maxN, (int64_t)RED_THREADS)));
  c->maxN = maxN;
  c->max_cblock = 1;
  for (int k = 0; k < G; ++k) {
    const GridDesc& gd = c->grid[k].desc;
    c->max_cblock = (int)std::max<int64_t>(c->max_cblock, ceil_div(gd.base + 1, gd.q));
  }
  c->coarse_x32 = c->fdtype == SFCDD_FP32 && params[0].coarse_precision == SFCDD_COARSE_AUTO;
  c->coarse32 = c->coarse_x32 && !c->coarse_iter && coarse_fp32_ok(c);

  // workspace layout
  const size_t es = c->fdtype == SFCDD_FP32 ? 4 : 8;
  const int64_t Nt = c->Ntot;
  const int Pt = c->Ptot;
  Planner pl;
  c->r_sfc = pl.take(4 * Nt);
  c->r_pos = pl.take(4 * Nt);
  c->r_nbr = pl.take((size_t)8 * c->dmax * Nt);
  c->r_gid = pl.take(2 * Nt);
  c->r_grids = pl.take(sizeof(GridDesc) * G);
  c->r_ta = pl.take(4 * Pt);
  c->r_Ni = pl.take(4 * Pt);
  c->r_nt = pl.take(4 * Pt);
  c->r_off = pl.take(8 * Pt);
  c->r_doff = pl.take(8 * Pt);
  c->r_xoff = pl.take(8 * Pt);
  c->r_poff = pl.take(8 * Pt);
  c->r_omega = pl.take(8 * Pt);
  c->r_sgid = pl.take(2 * Pt);
  c->r_fac = pl.take((size_t)c->tiles * TS2 * es);
  const bool inv = c->local_solver == SFCDD_LOCAL_INVERSE;
  c->r_facX = pl.take(inv ? (size_t)c->tiles * TS2 * es : 0);
  c->r_xloc = pl.take(inv ? (size_t)c->xlen * es : 0);
  c->r_fpart = pl.take(inv ? (size_t)c->parts * es : 0);
  c->r_A0 = pl.take((size_t)c->ctiles * TS2 * 8);
  c->r_X0 = pl.take((size_t)c->ctiles * TS2 * 8);
  c->r_c0 = pl.take((size_t)c->c0len * 8);
  c->r_d0 = pl.take((size_t)std::max<int64_t>(c->N0tot, c->c0len) * 8);
  c->r_cpart = pl.take((size_t)c->cparts * 8);
  // split-K partials of the single-matrix factorisation (three slots), later
  // reused by the triangular inversion; a dissected coarse matrix takes six
  // (three per half's chain) and V (at most nt0^2 / 8 tiles) after them
  const size_t kparts = G == 1 ? 6 * (size_t)c->max_nt0 * ceil_div(c->max_nt0, SPLITK) +
                                     ceil_div((int64_t)c->max_nt0 * c->max_nt0, 8)
                               : 0;
  c->r_cpartk = pl.take(std::max(kparts, (size_t)c->ctinv) * TS2 * 8);
  c->r_cmeta = pl.take((size_t)G * (5 * 8 + 2 * 4));
  c->r_cgid = pl.take(2 * c->N0tot);
  c->r_ctgid = pl.take(2 * c->ctiles);
  c->r_cy = pl.take((size_t)c->c0len * 8);
  c->r_dbuf = pl.take((size_t)c->sum_Ni * 8);
  c->r_vec = pl.take((size_t)NVEC * (((size_t)Nt * 8 + 255) & ~size_t(255)));
  // reductions: rbx partials per grid (two sums), or one per SpMV block
  c->r_partials = pl.take((size_t)8 * (2 * (size_t)G * std::max(c->rbx, spmv_blocks(maxN, 1)) +
                                      (size_t)MAXD * RED_BLOCKS));
  c->r_scal = pl.take((size_t)8 * G * S_COUNT);
  c->r_active = pl.take((size_t)4 * G);
  c->r_status = pl.take(64);
  c->r_gout = pl.take(MAXD * 8);
  c->r_lperm = pl.take(4 * (size_t)c->xlen);
  c->r_liperm = pl.take(4 * (size_t)c->sum_Ni);
  c->r_tlo = pl.take(4 * (size_t)(c->xlen / TS));
  c->r_trb = pl.take(4 * (size_t)(c->xlen / TS));
  c->r_gtiles = pl.take(24 * (size_t)G);
  c->r_ztile = pl.take((size_t)TS2 * 8);
  c->r_cperm = pl.take(4 * (size_t)c->N0tot);
  c->r_ccen = pl.take(4 * (size_t)c->N0tot * c->dmax);
  c->r_cfnz = pl.take(4 * (size_t)c->c0len);
  c->r_clo = pl.take(4 * (size_t)(c->c0len / TS));
  c->r_crb = pl.take(4 * (size_t)(c->c0len / TS));
  if (c->coarse_iter) {
    const GridDesc& g = c->grid[0].desc;
    c->ic_nt = g.nt0;
    c->ic_ld = (int64_t)g.nt0 * TS;
    c->ic_nq = (int)ceil_div(c->ic_ld, 256);
    // a row holds the block itself and at most 2 d entries per point
    c->ic_kw = (int)std::min<int64_t>(std::min<int64_t>(256, 2LL * g.d * c->max_cblock + 1), g.N0);
    const size_t ld = (size_t)c->ic_ld;
    c->r_ideg = pl.take(4 * ld);
    c->r_icol = pl.take(4 * ld * c->ic_kw);
    c->r_ival = pl.take(8 * ld * c->ic_kw);
    c->r_ibjt = pl.take((size_t)c->ic_nt * TS2 * 8);
    c->r_ibjm = pl.take((size_t)c->ic_nt * TS2 * 4);
    c->r_ibjnt = pl.take((size_t)c->ic_nt * 4);
    c->r_ibjoff = pl.take((size_t)c->ic_nt * 8);
    c->r_ivec = pl.take(4 * ld * 8);
    c->r_icagg = pl.take((size_t)g.nt0d * TS * 8);
    c->r_idagg = pl.take((size_t)g.nt0d * TS * 8);
    c->r_iqpart = pl.take((size_t)c->ic_nq * 8);
    c->r_ipart = pl.take((size_t)c->ic_nt * 2 * 8);
  }
  c->total = pl.top + 256;
  return SFCDD_OK;
}

template <typename T> T* at(sfcdd_ctx* c, const Region& r) {
  return reinterpret_cast<T*>(c->ws + r.off);
}

void bind(sfcdd_ctx* c) {
  c->sfc_index = at<int32_t>(c, c->r_sfc);
  c->pos = at<int32_t>(c, c->r_pos);
  c->nbr = at<int32_t>(c, c->r_nbr);
  c->gid = at<uint16_t>(c, c->r_gid);
  c->d_grids = at<GridDesc>(c, c->r_grids);
  c->d_ta = at<int32_t>(c, c->r_ta);
  c->d_Ni = at<int32_t>(c, c->r_Ni);
  c->d_nt = at<int32_t>(c, c->r_nt);
  c->d_off = at<int64_t>(c, c->r_off);
  c->d_doff = at<int64_t>(c, c->r_doff);
  c->d_xoff = at<int64_t>(c, c->r_xoff);
  c->d_poff = at<int64_t>(c, c->r_poff);
  c->d_omega = at<double>(c, c->r_omega);
  c->d_sgid = at<uint16_t>(c, c->r_sgid);
  c->fac = at<void>(c, c->r_fac);
  c->facX = at<void>(c, c->r_facX);
  c->xloc = at<void>(c, c->r_xloc);
  c->fpart = at<void>(c, c->r_fpart);
  c->A0 = at<double>(c, c->r_A0);
  c->X0 = at<double>(c, c->r_X0);
  c->c0 = at<double>(c, c->r_c0);
  c->d0 = at<double>(c, c->r_d0);
  c->cpart = at<double>(c, c->r_cpart);
  c->cpartk = at<double>(c, c->r_cpartk);
  c->cy = at<double>(c, c->r_cy);
  unsigned char* cm = c->ws + c->r_cmeta.off;
  const int G = c->G;
  c->dc_off = reinterpret_cast<int64_t*>(cm);
  c->dc_xoff = c->dc_off + G;
  c->dc_poff = c->dc_xoff + G;
  c->dc_doff = c->dc_poff + G;
  c->dc_toff = c->dc_doff + G;
  c->dc_nt = reinterpret_cast<int32_t*>(c->dc_toff + G);
  c->dc_n = c->dc_nt + G;
  c->cgid = at<uint16_t>(c, c->r_cgid);
  c->ctgid = at<uint16_t>(c, c->r_ctgid);
  c->dbuf = at<double>(c, c->r_dbuf);
  const size_t vstride = ((size_t)c->Ntot * 8 + 255) & ~size_t(255);
  for (int k = 0; k < NVEC; ++k)
    c->vec[k] = reinterpret_cast<double*>(c->ws + c->r_vec.off + k * vstride);
  c->partials = at<double>(c, c->r_partials);
  c->scal = at<double>(c, c->r_scal);
  c->active = at<int32_t>(c, c->r_active);
  c->status = at<int32_t>(c, c->r_status);
  c->gout = at<double>(c, c->r_gout);
  c->lperm = at<int32_t>(c, c->r_lperm);
  c->liperm = at<int32_t>(c, c->r_liperm);
  c->tlo = at<int32_t>(c, c->r_tlo);
  c->trb = at<int32_t>(c, c->r_trb);
  c->gtiles = at<unsigned long long>(c, c->r_gtiles);
  c->ztile = at<void>(c, c->r_ztile);
  c->cperm = at<int32_t>(c, c->r_cperm);
  c->ccen = at<int32_t>(c, c->r_ccen);
  c->cfnz = at<int32_t>(c, c->r_cfnz);
  c->clo = at<int32_t>(c, c->r_clo);
  c->crb = at<int32_t>(c, c->r_crb);
  if (c->coarse_iter) {
    c->ideg = at<int32_t>(c, c->r_ideg);
    c->icol = at<int32_t>(c, c->r_icol);
    c->ival = at<double>(c, c->r_ival);
    c->ibjt = at<double>(c, c->r_ibjt);
    c->ibjm = at<float>(c, c->r_ibjm);
    c->ibjnt = at<int32_t>(c, c->r_ibjnt);
    c->ibjoff = at<int64_t>(c, c->r_ibjoff);
    double* v = at<double>(c, c->r_ivec);
    c->ir = v;
    c->ip = v + c->ic_ld;
    c->iq = v + 2 * c->ic_ld;
    c->iz1 = v + 3 * c->ic_ld;
    c->icagg = at<double>(c, c->r_icagg);
    c->idagg = at<double>(c, c->r_idagg);
    c->iqpart = at<double>(c, c->r_iqpart);
    c->ipart = at<double>(c, c->r_ipart);
    c->iflag = c->status + 4;
  }
}

// Batched left-looking factorisation: each workgroup keeps its output tile in
// registers across the K loop.  A single matrix (part != nullptr) uses the
// split-K form instead, so that every column step runs on many workgroups.
// xoff / tlo / trb: the envelope tables of the matrices (first tile column and
// row base per tile row at xoff[b] / TS; a single matrix uses those of
// matrix 0 at tlo / trb).
// wide (single matrix): device-side envelope width, which picks the inversion
// beside the column steps (narrow envelopes) or after them.
template <typename T>
void factor_batch(int nb, int max_nt, const int32_t* nt, const int64_t* off, T* fac, T* X,
                  bool invert, bool product, int32_t* status, T* part, T* tbuf,
                  const int64_t* toff, bool pair, hipStream_t s, int rows = 0,
                  const int64_t* xoff = nullptr, const int32_t* tlo = nullptr, const int32_t* trb = nullptr,
                  const int32_t* wide = nullptr) {
  const int maxc = (max_nt + SPLITK - 1) / SPLITK;
  if (!part) {
    // batch: one workgroup factors a whole matrix
    launch_potrf_full<T>(nb, nt, off, xoff, tlo, trb, fac, status, pair, s, rows);
  } else {
    // one matrix: the first diagonal tile, then one step per column (its
    // sub-diagonal tiles, the next diagonal tile, split-K partials two
    // columns ahead in three slots)
    // (inverting a narrow envelope: row J of X = L^{-1} formed in step J
    // beside the chain; the recursive inversion below then skips)
    launch_potrf_diag<T>(0, 0, 0, maxc, part, 1, nt, off, fac, status, s, tlo, trb);
    for (int J = 0; J + 1 < max_nt; ++J)
      launch_potrf_step<T>(J, max_nt, maxc, part, (int64_t)max_nt * maxc, nt, off, fac, status, s, tlo, trb,
                           invert && wide ? X : nullptr, wide);
    if (invert && wide) launch_xrow<T>(max_nt - 1, off, fac, X, s, tlo, trb, wide);
  }
  if (invert) {
    if (tbuf) {
      launch_trtri_rec<T>(nb, max_nt, nt, off, toff, fac, X, tbuf, s, xoff, tlo, part ? wide : nullptr);
    } else {
      for (int J = max_nt - 1; J >= 0; --J) launch_trtri_col<T>(J, nb, max_nt, nt, off, fac, X, s);
    }
    if (product) launch_lauum<T>(nb, max_nt, nt, off, X, fac, s);
  }
}

// F v = R_0^T A_0^{-1} R_0 v: restriction into c0, then
// d0 = A_0^{-1} c0 = X_0^T (X_0 c0) with X_0 = L_0^{-1} (per grid; FP32
// entries in the second half of the X0 region beside FP32 subdomain factors,
// FP64 otherwise).
// Second level of the inner CG: d = A_agg^{-1} c with the dense aggregated
// matrix's inverse factor (FP32 beside FP32 subdomain factors).
void ic_second_level(sfcdd_ctx* c) {
  BatchMeta bm{c->dc_nt, c->dc_off, c->dc_xoff, c->dc_poff};
  if (c->coarse_x32)
    launch_coarse_apply<float>(1, c->max_nt0, bm, c->dc_n, c->dc_doff,
                               reinterpret_cast<const float*>(c->X0) + c->ctiles * TS2, c->icagg, c->cy,
                               c->cpart, c->idagg, c->iflag, c->stream);
  else
    launch_coarse_apply<double>(1, c->max_nt0, bm, c->dc_n, c->dc_doff, c->X0, c->icagg, c->cy, c->cpart,
                                c->idagg, c->iflag, c->stream);
}

// Iterative coarse solve d0 = A_0^{-1} b with b in c0 (single grid): inner
// CG on the sparse A_0, at most `steps` steps after the first direction; the
// device stops it at relative residual coarse_tol.  mask: the outer grid's
// flag (a grid that is not updating skips the solve).
void ic_solve(sfcdd_ctx* c, int steps, const int32_t* mask) {
  const hipStream_t s = c->stream;
  const int64_t n0 = c->grid[0].desc.N0;
  const int nt = c->ic_nt;
  launch_ic_begin(mask, c->iflag, c->scal, s);
  launch_ic_update(1, 0, n0, nt, c->ic_nq, c->iqpart, c->scal, c->c0, c->d0, c->ir, c->ip, c->iq, c->ibjm,
                   c->iz1, c->icagg, c->ipart, c->iflag, s);
  ic_second_level(c);
  launch_ic_dir(1, 0, n0, nt, c->ic_tol2, c->ipart, c->icagg, c->idagg, c->scal, c->iz1, c->ip, c->iflag, s);
  for (int it = 1; it <= steps; ++it) {
    launch_ic_spmv(c->ic_ld, c->ideg, c->icol, c->ival, c->ip, c->iq, c->iqpart, c->iflag, s);
    launch_ic_update(0, it, n0, nt, c->ic_nq, c->iqpart, c->scal, c->c0, c->d0, c->ir, c->ip, c->iq, c->ibjm,
                     c->iz1, c->icagg, c->ipart, c->iflag, s);
    ic_second_level(c);
    launch_ic_dir(0, it, n0, nt, c->ic_tol2, c->ipart, c->icagg, c->idagg, c->scal, c->iz1, c->ip, c->iflag, s);
  }
}

void coarse_solve(sfcdd_ctx* c, const double* v, const int32_t* mask = nullptr) {
  ProfScope ps(c, SFCDD_K_COARSE);
  const Batch B = c->batch();
  BatchMeta bm{c->dc_nt, c->dc_off, c->dc_xoff, c->dc_poff};
  launch_restrict(B, c->max_cblock, v, c->c0, c->stream);
  if (c->coarse_iter) {
    ic_solve(c, c->ic_k, mask);
    return;
  }
  if (c->coarse_x32)
    launch_coarse_apply<float>(c->G, c->max_nt0, bm, c->dc_n, c->dc_doff,
                               reinterpret_cast<const float*>(c->X0) + c->ctiles * TS2, c->c0, c->cy,
                               c->cpart, c->d0, mask, c->stream, c->nd[2] > 0 ? c->status + 13 : nullptr);
  else
    launch_coarse_apply<double>(c->G, c->max_nt0, bm, c->dc_n, c->dc_doff, c->X0, c->c0, c->cy, c->cpart,
                                c->d0, mask, c->stream, c->nd[2] > 0 ? c->status + 13 : nullptr);
}

// Subdomain solves d_i = A_i^{-1} R_i w into dbuf (Alg. 2, first two steps).
// Whether the substitution kernel reads its factors with the non-temporal
// hint: off unless the tuner found it faster.  The tile envelopes are read
// faster without it both at a few hundred MB (the backward sweep finds the
// tiles of the forward sweep's last rows again in the last-level cache) and
// at several GB.
bool stream_factors(const sfcdd_ctx* c) { return c->trsv_stream > 0; }

void local_solves(sfcdd_ctx* c, const double* w, int waves, const int32_t* mask = nullptr) {
  const hipStream_t s = c->stream;
  const Batch B = c->batch();
  if (c->local_solver == SFCDD_LOCAL_CHOLESKY) {
    const bool nt = stream_factors(c);
    if (c->fdtype == SFCDD_FP32)
      launch_schwarz_trsv<float>(B, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_doff, c->d_xoff, c->lperm, c->tlo,
                                 c->trb, c->max_nt, waves, nt,
                                 (const float*)c->fac, (const float*)c->ztile, w, c->dbuf, mask, s);
    else
      launch_schwarz_trsv<double>(B, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_doff, c->d_xoff, c->lperm, c->tlo,
                                  c->trb, c->max_nt, waves, nt,
                                  (const double*)c->fac, (const double*)c->ztile, w, c->dbuf, mask, s);
  } else {
    BatchMeta bm{c->d_nt, c->d_off, c->d_xoff, c->d_poff};
    if (c->fdtype == SFCDD_FP32) {
      launch_gather_local<float>(B, c->max_nt, bm, c->d_ta, c->d_Ni, w, (float*)c->xloc, s);
      launch_symv_tiles<float>(c->Ptot, c->max_nt, bm, (const float*)c->fac, (const float*)c->xloc,
                               (float*)c->fpart, s);
      launch_symv_reduce<float>(c->Ptot, c->max_Ni, bm, c->d_Ni, c->d_doff, (const float*)c->fpart,
                                c->dbuf, s);
    } else {
      launch_gather_local<double>(B, c->max_nt, bm, c->d_ta, c->d_Ni, w, (double*)c->xloc, s);
      launch_symv_tiles<double>(c->Ptot, c->max_nt, bm, (const double*)c->fac, (const double*)c->xloc,
                                (double*)c->fpart, s);
      launch_symv_reduce<double>(c->Ptot, c->max_Ni, bm, c->d_Ni, c->d_doff, (const double*)c->fpart,
                                 c->dbuf, s);
    }
  }
}

// y = sum_i R_i^T omega_i A_i^{-1} R_i w (eq. w1levprec).
void fine_apply(sfcdd_ctx* c, const double* w, double* y, const int32_t* mask = nullptr) {
  {
    ProfScope ps(c, SFCDD_K_LOCAL_SOLVE);
    local_solves(c, w, c->trsv_waves, mask);
  }
  ProfScope ps(c, SFCDD_K_SCATTER);
  launch_scatter(c->batch(), c->weighting == SFCDD_WEIGHT_D, c->d_ta, c->d_Ni, c->d_doff, c->d_omega,
                 c->dbuf, y, c->stream);
}

// Returns the per-grid partials written (modes 1 and 2), for the finalize.
int spmv(sfcdd_ctx* c, int mode, const double* x, double* y, const double* b, double* partials) {
  ProfScope ps(c, mode >= 2 ? SFCDD_K_SPMV_B : SFCDD_K_SPMV);
  return launch_spmv(c->batch(), mode, c->nbr, x, y, b, partials, c->stream);
}

void apply_s_defl(sfcdd_ctx* c, const double* r, double* h, const int32_t* mask, const double* db = nullptr,
                  const double* dc = nullptr);

// h = C^{-1} g in curve order (Alg. 2; balanced form eq. balSW).
// mask (nullable): solver flags; grids that are not updating may skip the
// subdomain and coarse solves (their output is then unspecified).
void apply_s(sfcdd_ctx* c, const double* g, double* h, const int32_t* mask = nullptr) {
  const hipStream_t s = c->stream;
  const Batch B = c->batch();
  if (c->variant == SFCDD_BALANCED) {
    double *t = c->vec[V_T], *w = c->vec[V_W], *y = c->vec[V_Y], *v = c->vec[V_V];
    coarse_solve(c, g, mask);                                   // d0 = A0^{-1} R0 g
    launch_combine(B, COMB_PROLONG, c->d0, nullptr, nullptr, t, s);  // t = F g
    spmv(c, 3, t, w, g, nullptr);                               // w = g - A t = G g
    fine_apply(c, w, y, mask);                                  // y = C1^{-1} G g
    spmv(c, 0, y, v, nullptr, nullptr);                         // v = A y
    coarse_solve(c, v, mask);                                   // d0 = A0^{-1} R0 A y
    launch_combine(B, COMB_BAL_FINAL, c->d0, y, t, h, s);      // h = y - F A y + F g
  } else if (c->variant == SFCDD_DEFLATED) {
    apply_s_defl(c, g, h, mask);                                // h = G^T C1^{-1} g + F g
  } else {
    coarse_solve(c, g, mask);
    fine_apply(c, g, h, mask);
    launch_combine(B, COMB_ADD_PROLONG, c->d0, h, nullptr, h, s);
  }
}

// Deflated operator h = G^T C1^{-1} r + F r = y + F (r - A y), y = C1^{-1} r:
// one coarse solve.  On a residual with R_0 r = 0 (F r = 0) it equals the
// balanced operator of eq. balSW, whose terms t = F r and A t vanish there.
// PCG and Richardson keep R_0 r_k = 0 once the start is coarse-corrected,
// because R_0 A (I - F A) = 0, so the balanced iteration runs on this form.
// Unlike y - F A y (the same operator in exact arithmetic), it also corrects
// the coarse component that rounding adds to r_k over the iterations, which
// would otherwise stall the residual once it reaches that level.  db
// (nullable): the last step also forms the partials of h . db and h . dc
// (launch_dot's layout).
void apply_s_defl(sfcdd_ctx* c, const double* r, double* h, const int32_t* mask, const double* db,
                  const double* dc) {
  const Batch B = c->batch();
  double *y = c->vec[V_Y], *v = c->vec[V_V];
  fine_apply(c, r, y, mask);                                   // y = C1^{-1} r
  spmv(c, 3, y, v, r, nullptr);                                // v = r - A y
  coarse_solve(c, v, mask);                                    // d0 = A0^{-1} R0 (r - A y)
  if (db)  // h = y + F (r - A y), with the partials of h . db (and h . dc)
    launch_combine_dot(B, c->d0, y, h, db, dc, c->partials, c->stream);
  else
    launch_combine(B, COMB_ADD_PROLONG, c->d0, y, nullptr, h, c->stream);  // h = y + F (r - A y)
}

// Inner step statistics of the latest iterative coarse solve, from the
// scalars just read back: the most steps seen, and a solve that ran out of
// its budget doubles the budget of the later ones.
constexpr int IC_TRIAL_STEPS = 500, IC_MAX_STEPS = 4000;
void ic_note(sfcdd_ctx* c) {
  if (!c->coarse_iter) return;
  const int its = (int)c->host_scal[IC_ITS];
  const bool conv = c->host_scal[IC_CONV] != 0.0;
  c->ic_max_steps = std::max(c->ic_max_steps, its);
  if (!conv && its >= c->ic_k && c->ic_k > 0) {
    ++c->ic_unconv;
    c->ic_k = std::min(2 * c->ic_k, IC_MAX_STEPS);
  }
}

// Copies the per-grid scalars to the pinned host buffer.
sfcdd_status read_scal(sfcdd_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, sizeof(double) * c->G * S_COUNT,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->active_in_flight = false;
  ic_note(c);
  return SFCDD_OK;
}
double hs(sfcdd_ctx* c, int g, int slot) { return c->host_scal[(size_t)g * S_COUNT + slot]; }

// Uploads the per-grid activity flags when they changed since the last
// upload.  The copy is asynchronous; its pinned source is rewritten only after
// a stream synchronisation has retired it.
sfcdd_status write_active(sfcdd_ctx* c, const std::vector<int32_t>& act) {
  if (c->active_valid && act == c->active_shadow) return SFCDD_OK;
  if (c->active_in_flight) HIPCHK(c, hipStreamSynchronize(c->stream));
  int32_t* hb = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(c->host_scal) + c->hb_off);
  for (int g = 0; g < c->G; ++g) hb[g] = act[g];
  HIPCHK(c, hipMemcpyAsync(c->active, hb, 4 * c->G, hipMemcpyHostToDevice, c->stream));
  c->active_in_flight = true;
  c->active_shadow = act;
  c->active_valid = true;
  return SFCDD_OK;
}

// Extreme eigenvalues of the symmetric tridiagonal Lanczos matrix by
// bisection on Sturm counts.
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double* lmin,
                      double* lmax) {
  const int m = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double dd = 1.0;
    for (int i = 0; i < m; ++i) {
      const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      dd = a[i] - x - (i > 0 ? bb / dd : 0.0);
      if (dd == 0.0) dd = -1e-300;
      if (dd < 0.0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {  // k-th smallest eigenvalue, 0-based
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + h);
      if (count_below(mid) > k) h = mid; else l = mid;
    }
    return 0.5 * (l + h);
  };
  *lmin = kth(0);
  *lmax = kth(m - 1);
}

// Device setup of a planned context (Alg. 1).
// The internal side stream of the current device, created on first use and
// kept for the life of the process: creating and destroying a stream per
// context now and then stalled a setup by tens of milliseconds.  Contexts of
// one device share it; their coarse setups then run one after the other on
// it (each joins the caller's stream before setup returns).
sfcdd_status device_side_stream(sfcdd_ctx* c, hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it == streams.end()) {
    hipStream_t st = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    it = streams.emplace(dev, st).first;
  }
  *out = it->second;
  return SFCDD_OK;
}

sfcdd_status setup_device(sfcdd_ctx* c) {
  const hipStream_t s = c->stream;
  const int G = c->G;
  const int Pt = c->Ptot;
  const Batch B = c->batch();
  hipEvent_t ev[6];
  for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
  HIPCHK(c, hipEventRecord(ev[0], s));

  // tables (host temporaries: synchronised before they go out of scope)
  std::vector<GridDesc> gd(G);
  for (int k = 0; k < G; ++k) gd[k] = c->grid[k].desc;
  std::vector<uint16_t> gid, cgid, ctgid;
  std::vector<unsigned char> img, cimg;
  if (G > 1) {
    gid.resize(c->Ntot);
    cgid.resize(c->N0tot);
    ctgid.resize(c->ctiles);
    for (int k = 0; k < G; ++k) {
      const GridDesc& g = gd[k];
      std::fill(gid.begin() + g.goff, gid.begin() + g.goff + g.N, (uint16_t)k);
      std::fill(cgid.begin() + g.c0off, cgid.begin() + g.c0off + g.N0, (uint16_t)k);
      std::fill(ctgid.begin() + c->c_off[k],
                ctgid.begin() + c->c_off[k] + (int64_t)g.nt0 * (g.nt0 + 1) / 2, (uint16_t)k);
    }
    HIPCHK(c, hipMemcpyAsync(c->gid, gid.data(), 2 * c->Ntot, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->cgid, cgid.data(), 2 * c->N0tot, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->ctgid, ctgid.data(), 2 * c->ctiles, hipMemcpyHostToDevice, s));
  }
  // the per-grid and per-subdomain tables (consecutive workspace regions)
  // and the coarse metadata go up as one host image each
  {
    const Region* tabs[] = {&c->r_grids, &c->r_ta, &c->r_Ni, &c->r_nt, &c->r_off, &c->r_doff,
                            &c->r_xoff, &c->r_poff, &c->r_omega, &c->r_sgid};
    const void* srcs[] = {gd.data(), c->ta.data(), c->Ni.data(), c->nt.data(), c->off.data(),
                          c->doff.data(), c->xoff.data(), c->poff.data(), c->omega.data(), c->sgid.data()};
    const size_t t0 = c->r_grids.off, t1 = c->r_sgid.off + c->r_sgid.bytes;
    img.assign(t1 - t0, 0);
    for (int k = 0; k < 10; ++k) std::memcpy(img.data() + (tabs[k]->off - t0), srcs[k], tabs[k]->bytes);
    HIPCHK(c, hipMemcpyAsync(c->ws + t0, img.data(), t1 - t0, hipMemcpyHostToDevice, s));
    cimg.assign(c->r_cmeta.bytes, 0);
    unsigned char* q = cimg.data();
    const std::vector<int64_t>* c64[] = {&c->c_off, &c->c_xoff, &c->c_poff, &c->c_doff, &c->c_toff};
    for (auto* v : c64) { std::memcpy(q, v->data(), 8 * (size_t)G); q += 8 * (size_t)G; }
    std::memcpy(q, c->c_nt.data(), 4 * (size_t)G);
    std::memcpy(q + 4 * (size_t)G, c->c_n.data(), 4 * (size_t)G);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->r_cmeta.off, cimg.data(), c->r_cmeta.bytes, hipMemcpyHostToDevice, s));
  }
  // block-diagonal part of the iterative coarse solve: ic_nt single-tile matrices
  std::vector<int32_t> bjnt;
  std::vector<int64_t> bjoff;
  if (c->coarse_iter) {
    bjnt.assign(c->ic_nt, 1);
    bjoff.resize(c->ic_nt);
    for (int t = 0; t < c->ic_nt; ++t) bjoff[t] = t;
    HIPCHK(c, hipMemcpyAsync(c->ibjnt, bjnt.data(), 4 * (size_t)c->ic_nt, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->ibjoff, bjoff.data(), 8 * (size_t)c->ic_nt, hipMemcpyHostToDevice, s));
  }
  HIPCHK(c, hipMemsetAsync(c->status, 0, 64, s));
  HIPCHK(c, hipStreamSynchronize(s));

  // curve order and neighbours (Alg. 1: sfc_index, neighbour map)
  HIPCHK(c, hipMemsetAsync(c->sfc_index, 0, 4 * c->Ntot, s));
  launch_sfc_rank(B, c->pos, c->sfc_index, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(ev[1], s));
  launch_build_nbr(B, c->pos, c->sfc_index, c->nbr, s);
  HIPCHK(c, hipEventRecord(ev[2], s));

  // The coarse setup (small, latency-bound steps) runs on an internal stream
  // forked from the caller's, concurrently with the batched subdomain
  // factorisation; both join before setup returns.
  hipEvent_t fork, join, cev0, cev1;
  HIPCHK(c, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&join, hipEventDisableTiming));
  HIPCHK(c, hipEventCreate(&cev0));
  HIPCHK(c, hipEventCreate(&cev1));
  if (!c->side) {
    const sfcdd_status st = device_side_stream(c, &c->side);
    if (st != SFCDD_OK) return st;
  }
  HIPCHK(c, hipEventRecord(fork, s));
  HIPCHK(c, hipStreamWaitEvent(c->side, fork, 0));
  // One-level dissection of a single dense coarse matrix whose factor and
  // inverse have the same precision (FP32 beside FP32 subdomain factors when
  // the coarse matrix is well conditioned, else FP64 throughout; not the FP64
  // factor rounded to an FP32 inverse).
  const int n0s = c->grid[0].desc.N0;
  const bool nd_try = G == 1 && !c->coarse_iter && (!c->coarse_x32 || c->coarse32) &&
                      c->coarse_split == SFCDD_SPLIT_AUTO && c->max_nt0 >= 16;
  int32_t* const nd_sep = reinterpret_cast<int32_t*>(c->cy);
  c->nd[0] = c->nd[1] = c->nd[2] = 0;
  {
    const hipStream_t cs = c->side;
    HIPCHK(c, hipEventRecord(cev0, cs));
    // coarse matrices A_0 = R_0 A R_0^T = sum_j c_j E_j (eq. csm), then A_0^{-1}
    HIPCHK(c, hipMemsetAsync(c->c0, 0, c->r_c0.bytes, cs));
    // coarse elimination order (key levels: 4 x the sum of the grid extents)
    int ckcap = 1;
    for (int k = 0; k < G; ++k) {
      int r = 1;
      for (int j = 0; j < c->grid[k].desc.d; ++j) r += 4 * (c->grid[k].desc.n[j] - 1);
      ckcap = std::max(ckcap, std::min(r, ORDER_MAX_KEYS));
    }
    int max_n0 = 1;
    for (int k = 0; k < G; ++k) max_n0 = std::max(max_n0, c->grid[k].desc.N0);
    launch_coarse_order(B, ckcap, max_n0, c->sfc_index, c->ccen, c->cperm, c->cfnz, cs);
    if (nd_try) {
      // one-level dissection (halves of the curve, separator last); its
      // scratch: the separator marks and the previous order in cy
      HIPCHK(c, hipMemsetAsync(nd_sep, 0, 4 * (size_t)n0s, cs));
      launch_nd_order(B, c->nbr, nd_sep, nd_sep + n0s, c->cperm, c->status + 13, n0s, cs);
    }
    // the envelopes first (only their tiles are cleared, assembled and read)
    launch_coarse_fnz(B, c->nbr, c->cfnz, cs);
    launch_coarse_env(B, c->max_nt0, c->cfnz, c->clo, c->crb, c->status + 12, nd_try ? c->status + 13 : nullptr,
                      cs);
    // the dissection's tiles and the halves' envelope width, read back before
    // the rest of the coarse setup is enqueued (the subdomain side follows it:
    // enqueued first, a batched factorisation that fills every CU would hold
    // back the coarse chain's first steps)
    if (nd_try)
      HIPCHK(c, hipMemcpyAsync(reinterpret_cast<unsigned char*>(c->host_scal) + c->hnd_off, c->status + 12, 16,
                               hipMemcpyDeviceToHost, cs));
    HIPCHK(c, hipGetLastError());
  }

  // The subdomain side: enqueued before the coarse chain (whose first steps a
  // batched factorisation filling every CU would otherwise hold back), or,
  // while the dissection's readback is awaited, before that wait.
  bool pair = false;
  int rows = 0;
  auto enqueue_fine = [&]() -> sfcdd_status {
    // local elimination order and tile envelopes, then the local matrices
    // A_i = R_i A R_i^T in that order (only the envelope tiles are written)
    HIPCHK(c, hipMemsetAsync(c->gtiles, 0, c->r_gtiles.bytes, s));
    HIPCHK(c, hipMemsetAsync(c->ztile, 0, c->r_ztile.bytes, s));
    const int omode = c->local_order == SFCDD_ORDER_DIAGONAL ? 2 : c->local_order == SFCDD_ORDER_CURVE ? 1 : 0;
    // key levels: at most the sum of the grid extents of the widest grid
    int kcap = 1;
    for (int k = 0; k < G; ++k) {
      int r = 1;
      for (int j = 0; j < c->grid[k].desc.d; ++j) r += c->grid[k].desc.n[j] - 1;
      kcap = std::max(kcap, std::min(r, ORDER_MAX_KEYS));
    }
    launch_local_order(B, omode, kcap, c->max_nt, c->d_ta, c->d_Ni, c->d_nt, c->d_xoff, c->d_doff, c->sfc_index, c->nbr,
                       c->lperm, c->liperm, c->tlo, c->trb, c->gtiles, s);
    if (c->fdtype == SFCDD_FP32)
      launch_assemble_local<float>(B, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_xoff, c->d_doff, c->lperm, c->liperm,
                                   c->tlo, c->trb, c->nbr, c->max_nt, (float*)c->fac, s);
    else
      launch_assemble_local<double>(B, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_xoff, c->d_doff, c->lperm,
                                    c->liperm, c->tlo, c->trb, c->nbr, c->max_nt, (double*)c->fac, s);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(ev[3], s));

    // factor once (Sec. 3.1).  The two-column batched kernel (380 registers
    // per lane in FP32) is the fastest alone; the one-column kernel (264)
    // leaves more room on the SIMDs for the concurrent coarse setup.
    const bool inv = c->local_solver == SFCDD_LOCAL_INVERSE;
    double fine_work = 0.0;
    for (int i = 0; i < Pt; ++i) fine_work += std::pow((double)c->Ni[i], 3.0);
    const double coarse_work = G == 1 ? std::pow((double)c->max_N0, 3.0) : 0.0;
    pair = c->factor_pair >= 0 ? c->factor_pair != 0
                               : (c->fdtype == SFCDD_FP64 || c->coarse32 || coarse_work < 0.15 * fine_work);
    // The light kernel (one row per panel step, no prefetch in the diagonal
    // update) for matrices of at most four tile rows, whose small LDS staging
    // lets several workgroups share a CU, and beside a single grid's coarse
    // chain at least twice as long as a subdomain's: its registers and LDS
    // leave room on every CU for the chain's workgroups, which set the
    // setup's critical path.
    const bool chain_bound = G == 1 && !c->coarse_iter && c->max_nt0 >= 2 * c->max_nt;
    rows = c->factor_rows > 0 ? c->factor_rows : ((c->max_nt <= 4 || chain_bound) ? 1 : 0);
    if (c->fdtype == SFCDD_FP32)
      factor_batch<float>(Pt, c->max_nt, c->d_nt, c->d_off, (float*)c->fac, (float*)c->facX, inv, inv,
                          c->status, (float*)nullptr, (float*)nullptr, nullptr, pair && rows != 1, s, rows,
                          c->d_xoff, c->tlo, c->trb);
    else
      factor_batch<double>(Pt, c->max_nt, c->d_nt, c->d_off, (double*)c->fac, (double*)c->facX, inv, inv,
                           c->status, (double*)nullptr, (double*)nullptr, nullptr, pair && rows != 1, s, rows,
                           c->d_xoff, c->tlo, c->trb);
    // the substitution kernel sweeps with the unit block-lower factor
    if (!inv) {
      if (c->fdtype == SFCDD_FP32)
        launch_unit_lower<float>(Pt, c->max_nt, c->d_nt, c->d_off, c->d_xoff, c->tlo, c->trb, (float*)c->fac, s);
      else
        launch_unit_lower<double>(Pt, c->max_nt, c->d_nt, c->d_off, c->d_xoff, c->tlo, c->trb, (double*)c->fac, s);
    }
    return SFCDD_OK;
  };
  if (nd_try) {
    const sfcdd_status fst = enqueue_fine();
    if (fst != SFCDD_OK) return fst;
  }
  {
    const hipStream_t cs = c->side;
    if (nd_try) {
      HIPCHK(c, hipStreamSynchronize(cs));
      const int32_t* h = reinterpret_cast<const int32_t*>(reinterpret_cast<const unsigned char*>(c->host_scal) +
                                                          c->hnd_off);
      const int wide = h[0];
      if (h[3] > 0 && wide <= XROW_MAXW) {
        c->nd[0] = h[1];
        c->nd[1] = h[2];
        c->nd[2] = h[3];
      } else if (h[3] > 0) {
        // the halves' envelopes are too wide for the inverse rows beside the
        // column steps: back to the undissected order
        launch_nd_undo(B, nd_sep + n0s, c->cperm, c->cfnz, c->status + 13, c->max_nt0 * TS, cs);
        launch_coarse_fnz(B, c->nbr, c->cfnz, cs);
        launch_coarse_env(B, c->max_nt0, c->cfnz, c->clo, c->crb, c->status + 12, nullptr, cs);
      }
    }
    int32_t* cnt = reinterpret_cast<int32_t*>(c->X0);   // count scratch (the inverse comes later)
    launch_coarse_zero_env(B, c->max_nt0, c->dc_off, c->clo, c->A0, cnt, cs);
    for (int j = 0; j < c->dmax; ++j) {
      launch_coarse_counts(B, j, c->nbr, c->dc_off, cnt, cs);
      launch_coarse_accumulate(B, c->max_nt0, c->dc_off, c->clo, j, cnt, c->A0, cs);
    }
    launch_coarse_pad(B, c->max_nt0, c->dc_off, c->A0, cs);
    // Beside FP32 subdomain factors the inverse X_0 = L_0^{-1} is FP32: A_0
    // is an M-matrix (a Galerkin aggregation of the stencil matrix), so L_0
    // has non-positive off-diagonal entries, X_0 is entrywise non-negative
    // and every sum that forms it has terms of one sign (no cancellation).
    // The factor itself is FP32 as well when the coarse matrices are well
    // conditioned (coarse_fp32_ok), else FP64 and rounded.  FP32 tiles: L_0
    // in the first half of the X0 region, X_0 in the second.
    if (c->coarse_x32) {
      float* L32 = reinterpret_cast<float*>(c->X0);
      float* part32 = reinterpret_cast<float*>(c->cpartk);
      if (c->coarse32) {
        launch_round_env(B, c->max_nt0, c->dc_off, c->clo, c->A0, L32, cs);
        if (c->nd[2] > 0) {
          // the three chains' row tables in d0 (free until the solves)
          int32_t* vinfo = reinterpret_cast<int32_t*>(c->d0);
          int32_t* vlo = vinfo + 16;
          int32_t* vrb = vlo + 3 * c->max_nt0;
          launch_nd_views(c->status + 13, c->clo, c->max_nt0, vinfo, vlo, vrb, cs);
          // V = L_S,half X_half,half in the FP64 coarse matrix's region (read
          // only by the rounding above)
          factor_nd<float>(c->nd[0], c->nd[1], c->nd[2], (int)ceil_div(c->max_nt0, SPLITK), part32, c->dc_off,
                           L32, L32 + c->ctiles * TS2, c->status + 1, c->dc_nt, c->clo, vinfo, vlo, vrb,
                           c->max_nt0, reinterpret_cast<float*>(c->A0), cs);
        } else {
          factor_batch<float>(G, c->max_nt0, c->dc_nt, c->dc_off, L32, L32 + c->ctiles * TS2, true, false,
                              c->status + 1, G == 1 ? part32 : (float*)nullptr, part32, c->dc_toff, false, cs, 0,
                              c->dc_xoff, c->clo, c->crb, G == 1 ? c->status + 12 : nullptr);
        }
      } else {
        factor_batch<double>(G, c->max_nt0, c->dc_nt, c->dc_off, c->A0, c->X0, false, false, c->status + 1,
                             G == 1 ? c->cpartk : (double*)nullptr, c->cpartk, c->dc_toff, false, cs, 0,
                             c->dc_xoff, c->clo, c->crb);
        launch_round_env(B, c->max_nt0, c->dc_off, c->clo, c->A0, L32, cs);
        launch_trtri_rec<float>(G, c->max_nt0, c->dc_nt, c->dc_off, c->dc_toff, L32, L32 + c->ctiles * TS2,
                                part32, cs, c->dc_xoff, c->clo);
      }
    } else if (c->nd[2] > 0) {
      int32_t* vinfo = reinterpret_cast<int32_t*>(c->d0);
      int32_t* vlo = vinfo + 16;
      int32_t* vrb = vlo + 3 * c->max_nt0;
      launch_nd_views(c->status + 13, c->clo, c->max_nt0, vinfo, vlo, vrb, cs);
      const int maxc = (int)ceil_div(c->max_nt0, SPLITK);
      factor_nd<double>(c->nd[0], c->nd[1], c->nd[2], maxc, c->cpartk, c->dc_off, c->A0, c->X0, c->status + 1,
                        c->dc_nt, c->clo, vinfo, vlo, vrb, c->max_nt0,
                        c->cpartk + 6 * (int64_t)c->max_nt0 * maxc * TS2, cs);
    } else {
      factor_batch<double>(G, c->max_nt0, c->dc_nt, c->dc_off, c->A0, c->X0, true, false, c->status + 1,
                           G == 1 ? c->cpartk : (double*)nullptr, c->cpartk, c->dc_toff, false, cs, 0,
                           c->dc_xoff, c->clo, c->crb, G == 1 ? c->status + 12 : nullptr);
    }
    if (c->coarse_iter) {
      // the sparse rows of A_0 (one workgroup per coarse block), then the
      // explicit inverses of its diagonal 64-blocks
      const int64_t n0 = c->grid[0].desc.N0;
      HIPCHK(c, hipMemsetAsync(c->ideg, 0, c->r_ideg.bytes, cs));
      launch_coarse_ell(B, n0, c->nbr, c->ic_kw, c->ic_ld, c->ideg, c->icol, c->ival, c->status + 2, cs);
      HIPCHK(c, hipMemsetAsync(c->ibjt, 0, c->r_ibjt.bytes, cs));
      launch_bj_extract(n0, c->ic_ld, c->ideg, c->icol, c->ival, c->ibjt, cs);
      launch_potrf_full<double>(c->ic_nt, c->ibjnt, c->ibjoff, nullptr, nullptr, nullptr, c->ibjt, c->status + 3,
                                false, cs);
      launch_bj_form(c->ic_nt, c->ibjt, c->ibjm, cs);
      HIPCHK(c, hipMemsetAsync(c->icagg, 0, c->r_icagg.bytes, cs));
      HIPCHK(c, hipMemsetAsync(c->idagg, 0, c->r_idagg.bytes, cs));
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(cev1, cs));
    HIPCHK(c, hipEventRecord(join, cs));
  }


  if (!nd_try) {
    const sfcdd_status fst = enqueue_fine();
    if (fst != SFCDD_OK) return fst;
  }
  c->info.factor_pair = pair && rows != 1 ? 1 : 0;
  c->info.factor_rows = rows > 0 ? rows : (c->fdtype == SFCDD_FP32 ? 3 : 2);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(ev[4], s));
  HIPCHK(c, hipStreamWaitEvent(s, join, 0));
  HIPCHK(c, hipEventRecord(ev[5], s));
  HIPCHK(c, hipStreamSynchronize(s));
  HIPCHK(c, hipStreamSynchronize(c->side));

  float ms[5];
  for (int k = 0; k < 4; ++k) HIPCHK(c, hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
  HIPCHK(c, hipEventElapsedTime(&ms[4], cev0, cev1));  // coarse setup (overlapped)
  float tot;
  HIPCHK(c, hipEventElapsedTime(&tot, ev[0], ev[5]));
  for (auto& e : ev) (void)hipEventDestroy(e);
  (void)hipEventDestroy(cev0);
  (void)hipEventDestroy(cev1);
  (void)hipEventDestroy(fork);
  (void)hipEventDestroy(join);
  sfcdd_info& I = c->info;
  I.N = c->Ntot;
  I.P = c->Ptot;
  I.q = c->grid[0].desc.q;
  I.N0 = (int32_t)c->N0tot;
  I.max_Ni = c->max_Ni;
  I.min_Ni = c->min_Ni;
  I.tile = TS;
  I.sum_Ni = c->sum_Ni;
  const int64_t es = c->fdtype == SFCDD_FP32 ? 4 : 8;
  {
    std::vector<unsigned long long> gt(3 * (size_t)G);
    HIPCHK(c, hipMemcpy(gt.data(), c->gtiles, 24 * (size_t)G, hipMemcpyDeviceToHost));
    int64_t tiles = 0, entries = 0, diag = 0;
    double products = 0.0;
    for (int k = 0; k < G; ++k) {
      c->gfac_bytes[k] = (int64_t)gt[3 * k] * TS2 * es;
      tiles += (int64_t)gt[3 * k];
      entries += (int64_t)gt[3 * k + 1];
      products += (double)gt[3 * k + 2];
    }
    for (int i = 0; i < Pt; ++i) diag += c->nt[i];
    I.factor_bytes = tiles * TS2 * es;
    I.factor_algo_bytes = entries * es;
    // every tile product 2 TS^3; a diagonal tile's Cholesky and inversion
    // TS^3 / 3 each
    I.factor_flops = products * 2.0 * TS * TS * TS + (double)diag * 2.0 * TS * TS * TS / 3.0;
  }
  I.local_order = c->local_order;
  I.coarse_bytes = (int64_t)c->r_A0.bytes;
  for (int k = 0; k < 5; ++k) I.setup_ms[k] = ms[k];
  I.setup_ms[5] = tot;
  I.ngrids = G;
  I.trsv_waves = c->trsv_waves;
  I.coarse_fp32 = c->coarse32 ? 1 : 0;
  I.coarse_inv_fp32 = c->coarse_x32 ? 1 : 0;
  I.coarse_iterative = c->coarse_iter ? 1 : 0;
  I.spmv_points = c->spmv_u;
  I.spmv_window = c->spmv_win;
  I.N0d = c->max_N0;
  I.ell_width = c->ic_kw;
  for (int k = 0; k < 3; ++k) I.coarse_split[k] = c->nd[k];

  int32_t stat[4] = {0, 0, 0, 0};
  HIPCHK(c, hipMemcpy(stat, c->status, 16, hipMemcpyDeviceToHost));
  if (stat[0] != 0) FAIL(c, SFCDD_ENOTSPD, "a local matrix is not positive definite");
  if (stat[1] != 0) FAIL(c, SFCDD_ENOTSPD, "a coarse matrix is not positive definite");
  if (stat[2] != 0)
    FAIL(c, SFCDD_EINVAL, "a coarse block couples to more than %d blocks (iterative coarse solver)", c->ic_kw);
  if (stat[3] != 0) FAIL(c, SFCDD_ENOTSPD, "a diagonal block of the coarse matrix is not positive definite");
  if (c->coarse_iter) {
    // size the inner step budget with a trial solve on a fixed right-hand side
    const int64_t n0 = c->grid[0].desc.N0;
    launch_ic_trial(n0, c->ic_ld, c->c0, s);
    ic_solve(c, IC_TRIAL_STEPS, nullptr);
    HIPCHK(c, hipGetLastError());
    double sc[S_COUNT];
    HIPCHK(c, hipMemcpyAsync(sc, c->scal, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int its = (int)sc[IC_ITS];
    c->ic_k = sc[IC_CONV] != 0.0 ? std::min(IC_MAX_STEPS, its + its / 4 + 4) : IC_TRIAL_STEPS;
    I.coarse_steps = c->ic_k;
  }
  return SFCDD_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the launch shapes.  Each choice depends only on the launch
// shape it serves and is recorded for the process under a key of that shape:
// the substitution kernel's waves (device, precision, local solver and
// order, tile count and size of every subdomain, grid sizes and curves), the SpMV's points per step and window
// (device, grid sizes and curves), the batched factorisation's rows per step
// and column pairing (device, precisions, coarse solver, subdomain sizes and
// coarse sizes; it is timed as a whole setup, since the factorisation shares
// the device with the concurrent coarse setup).
struct TuneRecord {
  int a = 0, b = 0;
  double t = 0.0, t_default = 0.0;
};
std::mutex g_tune_mu;
std::map<uint64_t, TuneRecord> g_tune_trsv, g_tune_spmv, g_tune_setup;

struct KeyMix {
  uint64_t key = 1469598103934665603ull;
  void operator()(uint64_t v) { key = (key ^ v) * 1099511628211ull; }
};

uint64_t key_trsv(const sfcdd_ctx* c, int dev) {
  KeyMix m;
  m((uint64_t)dev);
  m((uint64_t)c->fdtype);
  m((uint64_t)c->local_solver);
  m((uint64_t)c->local_order);
  m((uint64_t)c->coarse_split);
  for (int i = 0; i < c->Ptot; ++i) {
    m((uint64_t)c->nt[i]);
    m((uint64_t)c->Ni[i]);
  }
  // the tile envelopes follow from the grid's geometry and curve
  for (int k = 0; k < c->G; ++k) {
    const GridDesc& g = c->grid[k].desc;
    m((uint64_t)g.curve);
    for (int j = 0; j < g.d; ++j) m((uint64_t)g.n[j]);
  }
  return m.key;
}
uint64_t key_spmv(const sfcdd_ctx* c, int dev) {
  KeyMix m;
  m((uint64_t)dev);
  m((uint64_t)c->G);
  for (int k = 0; k < c->G; ++k) {
    const GridDesc& g = c->grid[k].desc;
    m((uint64_t)g.d);
    m((uint64_t)g.curve);
    for (int j = 0; j < g.d; ++j) m((uint64_t)g.n[j]);
  }
  return m.key;
}
uint64_t key_setup(const sfcdd_ctx* c, int dev) {
  KeyMix m;
  m(key_trsv(c, dev));
  m((uint64_t)c->coarse_iter);
  m((uint64_t)c->coarse_x32);
  m((uint64_t)c->coarse32);
  for (int k = 0; k < c->G; ++k) {
    m((uint64_t)c->grid[k].desc.N0);
    m((uint64_t)c->grid[k].desc.N0d);
  }
  return m.key;
}

// Shapes recorded by earlier tunings of the same launch shapes (applied at
// setup, before the factorisation).
void apply_recorded_shapes(sfcdd_ctx* c) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto t = g_tune_trsv.find(key_trsv(c, dev));
  if (t != g_tune_trsv.end()) {
    c->trsv_waves = t->second.a;
    c->trsv_stream = t->second.b;
  }
  auto v = g_tune_spmv.find(key_spmv(c, dev));
  if (v != g_tune_spmv.end()) {
    c->spmv_u = v->second.a;
    c->spmv_win = v->second.b;
  }
  auto f = g_tune_setup.find(key_setup(c, dev));
  if (f != g_tune_setup.end()) {
    c->factor_rows = f->second.a;
    c->factor_pair = f->second.b;
  }
}

sfcdd_status setup_device(sfcdd_ctx* c);
void local_solves(sfcdd_ctx* c, const double* w, int waves, const int32_t* mask);

sfcdd_status tune_shapes(sfcdd_ctx* c, int32_t repeats, int32_t what, sfcdd_tuning* r) {
  const bool force = repeats < 0;
  repeats = repeats < 0 ? -repeats : (repeats == 0 ? 3 : repeats);
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  const hipStream_t s = c->stream;
  hipEvent_t a, b;
  HIPCHK(c, hipEventCreate(&a));
  HIPCHK(c, hipEventCreate(&b));
  // mean time (ms) of `repeats` runs of f after one warm-up run
  auto timed = [&](auto&& f, double* ms) -> sfcdd_status {
    f();
    HIPCHK(c, hipEventRecord(a, s));
    for (int k = 0; k < repeats; ++k) f();
    HIPCHK(c, hipEventRecord(b, s));
    HIPCHK(c, hipEventSynchronize(b));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, a, b));
    *ms = t / repeats;
    return SFCDD_OK;
  };
  sfcdd_status st = SFCDD_OK;
  r->tuned = 0;
  double* w = c->vec[V_TMP];
  double* y = c->vec[V_Y];
  launch_zero(c->Ntot, w, s);
  // substitution kernel: waves per workgroup
  if (what & SFCDD_TUNE_TRSV) {
    const uint64_t key = key_trsv(c, dev);
    TuneRecord rec;
    bool have = false;
    if (!force) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_trsv.find(key);
      if (it != g_tune_trsv.end()) { rec = it->second; have = true; }
    }
    if (!have) {
      // waves per workgroup, and the non-temporal hint on the factor loads
      // (factors a little larger than the last-level cache can still be
      // re-read from it by the backward sweep)
      const bool chol = c->local_solver == SFCDD_LOCAL_CHOLESKY;
      const int ncand = chol ? 3 : 1;
      // the default first
      const int cand[3] = {c->max_nt <= 8 ? 4 : 16, 8, c->max_nt <= 8 ? 16 : 4};
      const int keep_stream = c->trsv_stream;
      c->trsv_stream = -1;
      const int rule = stream_factors(c) ? 1 : 0;
      rec.a = c->trsv_waves;
      rec.b = -1;
      rec.t = 1e300;
      for (int h = 0; h < (chol ? 2 : 1) && st == SFCDD_OK; ++h) {
        c->trsv_stream = h == 0 ? rule : 1 - rule;
        for (int k = 0; k < ncand && st == SFCDD_OK; ++k) {
          double ms = 0.0;
          st = timed([&] { local_solves(c, w, cand[k], nullptr); }, &ms);
          if (h == 0 && k == 0) rec.t_default = ms;
          if (ms < rec.t) {
            rec.t = ms;
            rec.a = ncand > 1 ? cand[k] : c->trsv_waves;
            rec.b = chol ? c->trsv_stream : -1;
          }
        }
      }
      c->trsv_stream = keep_stream;
      if (st == SFCDD_OK) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_trsv[key] = rec;
      }
      r->tuned |= SFCDD_TUNE_TRSV;
    }
    c->trsv_waves = rec.a;
    c->trsv_stream = rec.b;
    r->trsv_ms = rec.t;
    r->trsv_default_ms = rec.t_default;
  }
  // SpMV: points per thread (and window)
  if (st == SFCDD_OK && (what & SFCDD_TUNE_SPMV)) {
    const uint64_t key = key_spmv(c, dev);
    TuneRecord rec;
    bool have = false;
    if (!force) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_spmv.find(key);
      if (it != g_tune_spmv.end()) { rec = it->second; have = true; }
    }
    if (!have) {
      // points per thread (the window is 256 of them per thread); the
      // default first
      const int us[3] = {2, 1, 4};
      rec.t = 1e300;
      for (int i = 0; i < 3 && st == SFCDD_OK; ++i) {
        Batch B = c->batch();
        B.spmv_u = us[i];
        double ms = 0.0;
        st = timed([&] { launch_spmv(B, 0, c->nbr, w, y, nullptr, nullptr, s); }, &ms);
        if (i == 0) rec.t_default = ms;
        if (ms < rec.t) { rec.t = ms; rec.a = us[i]; rec.b = RED_THREADS * us[i]; }
      }
      if (st == SFCDD_OK) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_spmv[key] = rec;
      }
      r->tuned |= SFCDD_TUNE_SPMV;
    }
    c->spmv_u = rec.a;
    c->spmv_win = rec.b;
    r->spmv_ms = rec.t;
    r->spmv_default_ms = rec.t_default;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != SFCDD_OK) return st;
  // batched factorisation: rows per panel step and column pairing, timed as
  // whole setups of this context (which ends set up with the winner)
  if (what & SFCDD_TUNE_SETUP) {
    const uint64_t key = key_setup(c, dev);
    TuneRecord rec;
    bool have = false;
    if (!force) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_setup.find(key);
      if (it != g_tune_setup.end()) { rec = it->second; have = true; }
    }
    if (!have) {
      const int saved_rows = c->factor_rows, saved_pair = c->factor_pair;
      // the default shape (the rules) first, then every explicit one
      std::vector<std::pair<int, int>> cand{{0, -1}, {1, 0}};
      for (int pr = 0; pr <= 1; ++pr)
        for (int rw = 2; rw <= potrf_full_max_rows(c->fdtype == SFCDD_FP64, pr != 0); ++rw)
          cand.emplace_back(rw, pr);
      rec.t = 1e300;
      int last = -1;
      for (size_t k = 0; k < cand.size(); ++k) {
        c->factor_rows = cand[k].first;
        c->factor_pair = cand[k].second;
        double best_k = 1e300;
        for (int rpt = 0; rpt < std::max(1, std::min(repeats, 2)); ++rpt) {
          if ((st = setup_device(c)) != SFCDD_OK) {
            c->factor_rows = saved_rows;
            c->factor_pair = saved_pair;
            return st;
          }
          best_k = std::min(best_k, c->info.setup_ms[5]);
        }
        last = (int)k;
        if (k == 0) rec.t_default = best_k;
        // the explicit shape of the default is the one setup_device reports
        const int rw = k == 0 ? c->info.factor_rows : cand[k].first;
        const int pr = k == 0 ? c->info.factor_pair : cand[k].second;
        if (best_k < rec.t) { rec.t = best_k; rec.a = rw; rec.b = pr; }
      }
      c->factor_rows = rec.a;
      c->factor_pair = rec.b;
      if (last < 0 || !(cand[last].first == rec.a && cand[last].second == rec.b))
        if ((st = setup_device(c)) != SFCDD_OK) return st;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_setup[key] = rec;
      }
      r->tuned |= SFCDD_TUNE_SETUP;
    } else {
      c->factor_rows = rec.a;
      c->factor_pair = rec.b;
    }
    r->setup_ms = rec.t;
    r->setup_default_ms = rec.t_default;
  }
  r->trsv_waves = c->trsv_waves;
  r->trsv_stream = c->trsv_stream;
  r->spmv_points = c->spmv_u;
  r->spmv_window = c->spmv_win;
  r->factor_rows = c->factor_rows > 0 ? c->factor_rows : c->info.factor_rows;
  r->factor_pair = c->factor_pair >= 0 ? c->factor_pair : c->info.factor_pair;
  c->info.trsv_waves = c->trsv_waves;
  c->info.spmv_points = c->spmv_u;
  c->info.spmv_window = c->spmv_win;
  return SFCDD_OK;
}

// Workspace of the allocation-free setup: one array per device, resident for
// the life of the process.  In host code its name is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SFCDD_NOALLOC_WORKSPACE_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
uint64_t g_noalloc_gen[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's static workspace (looked up on the
// first call on that device) and the generation the new context takes; a
// context of an older generation on the same device is stale.
sfcdd_status noalloc_acquire(int* dev_out, void** ptr_out, uint64_t* gen_out) {
  sfcdd_ctx* none = nullptr;
  int dev = 0;
  HIPCHK(none, hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    FAIL(none, SFCDD_EINVAL, "device %d: the allocation-free setup supports devices 0..%d", dev,
         NOALLOC_MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(none, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) FAIL(none, SFCDD_EDEVICE, "hipGetSymbolAddress returned no address for the static workspace");
    g_noalloc_ptr[dev] = ptr;
  }
  *dev_out = dev;
  *ptr_out = g_noalloc_ptr[dev];
  *gen_out = ++g_noalloc_gen[dev];
  return SFCDD_OK;
}

// EINVAL for an allocation-free context whose workspace a later
// allocation-free setup on the same device has taken over.
bool noalloc_stale(const sfcdd_ctx* c) {
  if (!c->noalloc) return false;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_gen[c->noalloc_dev] != c->noalloc_gen;
}

sfcdd_status setup_common(int G, const sfcdd_params* params, void* workspace_dev, size_t bytes,
                          void* hip_stream, sfcdd_ctx** out, bool noalloc = false) {
  if (!out) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!noalloc && !workspace_dev) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "workspace is NULL");
  sfcdd_ctx* c = new (std::nothrow) sfcdd_ctx();
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_ENOMEM, "host allocation failed");
  sfcdd_status st = plan(c, G, params);
  if (st != SFCDD_OK) {
    g_last_error = c->err;
    delete c;
    return st;
  }
  if (noalloc) {
    if (c->total > SFCDD_NOALLOC_WORKSPACE_BYTES) {
      g_last_error = "the problem needs a workspace of " + std::to_string(c->total) +
                     " bytes; the allocation-free setup has " +
                     std::to_string((unsigned long long)SFCDD_NOALLOC_WORKSPACE_BYTES);
      delete c;
      return SFCDD_ENOMEM;
    }
    st = noalloc_acquire(&c->noalloc_dev, &workspace_dev, &c->noalloc_gen);
    if (st != SFCDD_OK) {
      delete c;
      return st;
    }
    bytes = SFCDD_NOALLOC_WORKSPACE_BYTES;
    c->noalloc = true;
  }
  if (bytes < c->total) {
    g_last_error = "workspace too small: need " + std::to_string(c->total) + " bytes";
    delete c;
    return SFCDD_ENOMEM;
  }
  c->ws = reinterpret_cast<unsigned char*>((reinterpret_cast<uintptr_t>(workspace_dev) + 255) & ~uintptr_t(255));
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  bind(c);
  // the scalars and the flags are consecutive workspace regions: one copy reads both back
  c->rb_flags = c->r_active.off - c->r_scal.off;
  c->rb_bytes = c->rb_flags + 4 * (size_t)G;
  c->hb_off = (c->rb_bytes + 255) & ~size_t(255);
  c->hnd_off = c->hb_off + 4 * (size_t)G + 8 * MAXD + 256;
  const size_t hbytes = c->hnd_off + 16;
  if (c->noalloc) {
    // pageable host image: device-to-host copies into it are waited for with a
    // stream synchronisation (see wait_readback)
    c->host_pageable.assign(hbytes, 0);
    c->host_scal = reinterpret_cast<double*>(c->host_pageable.data());
  } else if (hipHostMalloc((void**)&c->host_scal, hbytes, hipHostMallocDefault) != hipSuccess) {
    g_last_error = "hipHostMalloc failed";
    delete c;
    return SFCDD_EDEVICE;
  }
  if (hipEventCreateWithFlags(&c->ev_rb, hipEventDisableTiming) != hipSuccess) {
    g_last_error = "hipEventCreate failed";
    if (!c->noalloc) (void)hipHostFree(c->host_scal);
    delete c;
    return SFCDD_EDEVICE;
  }
  *out = c;
  apply_recorded_shapes(c);
  return setup_device(c);
}

}  // namespace

extern "C" {

sfcdd_status sfcdd_workspace_size_batch(int32_t ngrids, const sfcdd_params* params, size_t* bytes) {
  if (!bytes) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "bytes is NULL");
  sfcdd_ctx tmp;
  const sfcdd_status st = plan(&tmp, ngrids, params);
  if (st != SFCDD_OK) {
    g_last_error = tmp.err;
    return st;
  }
  *bytes = tmp.total;
  return SFCDD_OK;
}

sfcdd_status sfcdd_workspace_size(const sfcdd_params* params, size_t* bytes) {
  return sfcdd_workspace_size_batch(1, params, bytes);
}

sfcdd_status sfcdd_setup(const sfcdd_params* params, void* workspace_dev, size_t bytes,
                         void* hip_stream, sfcdd_ctx** out) {
  return setup_common(1, params, workspace_dev, bytes, hip_stream, out);
}

sfcdd_status sfcdd_setup_batch(int32_t ngrids, const sfcdd_params* params, void* workspace_dev,
                               size_t bytes, void* hip_stream, sfcdd_ctx** out) {
  return setup_common(ngrids, params, workspace_dev, bytes, hip_stream, out);
}

sfcdd_status sfcdd_setup_noalloc(const sfcdd_params* params, void* hip_stream, sfcdd_ctx** out) {
  return setup_common(1, params, nullptr, 0, hip_stream, out, true);
}

sfcdd_status sfcdd_apply_precond(sfcdd_ctx* c, const double* g, double* h) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (!g || !h || g == h) FAIL(c, SFCDD_EINVAL, "g and h must be distinct non-NULL device vectors");
  const int64_t N = c->Ntot;
  if (c->layout == 1) {
    apply_s(c, g, h);
  } else {
    launch_permute(N, c->sfc_index, g, c->vec[V_IN], 1, c->stream);
    apply_s(c, c->vec[V_IN], c->vec[V_OUT]);
    launch_permute(N, c->sfc_index, c->vec[V_OUT], h, 0, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  return SFCDD_OK;
}

sfcdd_status sfcdd_matvec(sfcdd_ctx* c, const double* x, double* y) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (!x || !y || x == y) FAIL(c, SFCDD_EINVAL, "x and y must be distinct non-NULL device vectors");
  const int64_t N = c->Ntot;
  if (c->layout == 1) {
    spmv(c, 0, x, y, nullptr, nullptr);
  } else {
    launch_permute(N, c->sfc_index, x, c->vec[V_IN], 1, c->stream);
    spmv(c, 0, c->vec[V_IN], c->vec[V_OUT], nullptr, nullptr);
    launch_permute(N, c->sfc_index, c->vec[V_OUT], y, 0, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  return SFCDD_OK;
}

sfcdd_status sfcdd_solve(sfcdd_ctx* c, const double* b_in, double* x_io, double rtol,
                         int32_t max_iter, int32_t method, double xi, sfcdd_solve_info* info) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (!b_in || !x_io || b_in == x_io) FAIL(c, SFCDD_EINVAL, "b and x must be distinct non-NULL device vectors");
  if (!(rtol > 0.0) || max_iter < 0) FAIL(c, SFCDD_EINVAL, "need rtol > 0 and max_iter >= 0");
  c->ic_max_steps = 0;
  c->ic_unconv = 0;
  const bool plain = (method & SFCDD_SOLVE_PLAIN_START) != 0;
  const bool energy = (method & SFCDD_SOLVE_ENERGY) != 0;
  const bool recursive = (method & SFCDD_SOLVE_RECURSIVE) != 0 || energy;
  method &= ~(SFCDD_SOLVE_PLAIN_START | SFCDD_SOLVE_RECURSIVE | SFCDD_SOLVE_ENERGY);
  if (method != SFCDD_PCG && method != SFCDD_FCG && method != SFCDD_RICHARDSON)
    FAIL(c, SFCDD_EINVAL, "method = %d", method);
  // balanced form: coarse-corrected start, then one coarse solve per iteration
  const bool proj = (c->variant == SFCDD_BALANCED || c->variant == SFCDD_DEFLATED) && !plain;
  // preconditioner inside the iteration: grids that are not updating skip
  // their subdomain and coarse solves
  auto precond = [&](const double* g, double* h) {
    if (proj) apply_s_defl(c, g, h, c->active);
    else apply_s(c, g, h, c->active);
  };
  // h = C^{-1} g and the partials of h . db (and h . dc): the deflated
  // operator forms them in its last launch
  auto precond_dot = [&](const double* g, double* h, const double* db, const double* dc) {
    if (proj) {
      apply_s_defl(c, g, h, c->active, db, dc);
    } else {
      apply_s(c, g, h, c->active);
      launch_dot(c->batch(), h, db, dc, c->partials, c->stream);
    }
  };
  const hipStream_t s = c->stream;
  const int64_t N = c->Ntot;
  const int G = c->G;
  const Batch B = c->batch();
  double *x = c->vec[V_X], *r = c->vec[V_R], *z = c->vec[V_Z], *p = c->vec[V_P], *q = c->vec[V_Q],
         *b = c->vec[V_B], *tmp = c->vec[V_TMP];
  if (c->layout == 1) {
    launch_copy(N, b_in, b, s);
    launch_copy(N, x_io, x, s);
  } else {
    launch_permute(N, c->sfc_index, b_in, b, 1, s);
    launch_permute(N, c->sfc_index, x_io, x, 1, s);
  }
  if (proj) {
    // x <- x + F (b - A x), so that R_0 (b - A x) = 0 (balancing start)
    spmv(c, 3, x, tmp, b, nullptr);
    coarse_solve(c, tmp);
    launch_combine(B, COMB_ADD_PROLONG, c->d0, x, nullptr, x, s);
  }
  launch_dot(B, b, b, nullptr, c->partials, s);
  launch_finalize(B, FIN_BB, c->partials, c->scal, nullptr, s);
  sfcdd_status st;
  if ((st = read_scal(c))) return st;
  std::vector<double> tol2(G), bb(G), rr(G, 0.0);
  for (int g = 0; g < G; ++g) {
    bb[g] = hs(c, g, S_BB);
    if (energy && bb[g] != 0.0) FAIL(c, SFCDD_EINVAL, "SFCDD_SOLVE_ENERGY needs b = 0 (grid %d)", g);
    tol2[g] = energy ? rtol * rtol : rtol * rtol * bb[g];
  }
  // the squared norm a grid's stopping test looks at, from the partials of
  // the residual's r . r just formed: that norm, or (energy test) -(x . r)
  // (np: the partials' count per grid, from the SpMV that formed them, or 0)
  auto norm_fin = [&](int rr_mode, int en_mode, int np) {
    if (energy) {
      launch_dot(B, x, r, nullptr, c->partials, s);
      launch_finalize(B, en_mode, c->partials, c->scal, en_mode == FIN_EN ? nullptr : c->active, s);
    } else {
      launch_finalize(B, rr_mode, c->partials, c->scal, rr_mode == FIN_RR ? nullptr : c->active, s, np);
    }
  };
  std::vector<int32_t> flags(G, ACT_RUN), its(G, 0), stagnated(G, 0);
  // true residual at each grid's previous restart (stagnation test)
  std::vector<double> last_trr(G, std::numeric_limits<double>::infinity());
  sfcdd_solve_info inf{};
  int it = 0, restarts = 0;
  auto n_updating = [&]() {
    int n = 0;
    for (int g = 0; g < G; ++g) n += act_updating(flags[g]);
    return n;
  };
  auto read_rr = [&]() -> sfcdd_status {
    sfcdd_status e = read_scal(c);
    if (e) return e;
    for (int g = 0; g < G; ++g) rr[g] = hs(c, g, S_RR);
    return SFCDD_OK;
  };
  // per-grid scalars written by the host (tolerances, Richardson damping):
  // read-modify-write of the device scalar array, which read_scal just copied
  auto upload_scal = [&]() -> sfcdd_status {
    HIPCHK(c, hipMemcpyAsync(c->scal, c->host_scal, sizeof(double) * G * S_COUNT, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SFCDD_OK;
  };
  // Asynchronous copy of the residual norms and flags of the step just
  // enqueued; the host waits for it while the next preconditioner
  // application (enqueued speculatively) runs.
  int32_t* hflags = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(c->host_scal) + c->rb_flags);
  auto enqueue_readback = [&]() -> sfcdd_status {
    HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, c->rb_bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(c->ev_rb, s));
    return SFCDD_OK;
  };
  auto wait_readback = [&]() -> sfcdd_status {
    if (c->noalloc) HIPCHK(c, hipStreamSynchronize(s));  // pageable target: the copy is complete
    else HIPCHK(c, hipEventSynchronize(c->ev_rb));
    c->active_in_flight = false;
    ic_note(c);
    for (int g = 0; g < G; ++g) rr[g] = hs(c, g, S_RR);
    return SFCDD_OK;
  };

  if (method == SFCDD_RICHARDSON) {
    std::vector<double> xig(G, xi);
    if (!(xi > 0.0)) {
      // Lanczos estimate of the extreme eigenvalues of C^{-1}A from CG steps (per grid)
      std::vector<std::vector<double>> al(G), be(G);
      std::vector<int32_t> ok(G, ACT_RUN);
      if ((st = write_active(c, ok))) return st;
      launch_zero(N, z, s);  // z is the iterate of the estimation run (on the residual of x)
      spmv(c, 3, x, r, b, nullptr);
      precond(r, q);
      launch_copy(N, q, p, s);
      launch_dot(B, r, q, nullptr, c->partials, s);
      launch_finalize(B, FIN_RZ_INIT, c->partials, c->scal, c->active, s);
      for (int k = 0; k < 30; ++k) {
        const int np = spmv(c, 1, p, tmp, nullptr, c->partials);
        launch_finalize(B, FIN_PQ_ALPHA, c->partials, c->scal, c->active, s, np);
        launch_update_xr(B, c->scal, c->active, z, r, p, tmp, c->partials, s);
        if ((st = read_scal(c))) return st;
        for (int g = 0; g < G; ++g) {
          const double a_k = hs(c, g, S_ALPHA);
          if (ok[g] && a_k > 0.0 && std::isfinite(a_k)) al[g].push_back(a_k);
          else ok[g] = ACT_DONE;
        }
        if ((st = write_active(c, ok))) return st;
        precond(r, q);
        launch_dot(B, r, q, nullptr, c->partials, s);
        launch_finalize(B, FIN_RZ_NEXT, c->partials, c->scal, c->active, s);
        if ((st = read_scal(c))) return st;
        for (int g = 0; g < G; ++g) {
          const double b_k = hs(c, g, S_BETA);
          if (ok[g] && b_k > 0.0 && std::isfinite(b_k)) be[g].push_back(b_k);
          else ok[g] = ACT_DONE;
        }
        if ((st = write_active(c, ok))) return st;
        int nok = 0;
        for (int g = 0; g < G; ++g) nok += ok[g] != ACT_DONE;
        if (nok == 0) break;
        launch_update_p(B, c->scal, c->active, p, q, s);
      }
      for (int g = 0; g < G; ++g) {
        const int m = (int)std::min(al[g].size(), be[g].size() + 1);
        if (m == 0) FAIL(c, SFCDD_ENOTCONV, "Lanczos estimate failed for grid %d", g);
        std::vector<double> ta(m), tb(m > 1 ? m - 1 : 0);
        for (int k = 0; k < m; ++k) ta[k] = 1.0 / al[g][k] + (k > 0 ? be[g][k - 1] / al[g][k - 1] : 0.0);
        for (int k = 0; k + 1 < m; ++k) tb[k] = std::sqrt(be[g][k]) / al[g][k];
        double lmin, lmax;
        tridiag_extremes(ta, tb, &lmin, &lmax);
        if (g == 0) {
          inf.lambda_min = lmin;
          inf.lambda_max = lmax;
        }
        xig[g] = 2.0 / (lmin + lmax);
      }
    }
    inf.xi = xig[0];
    // r = b - A x and its norm; damping and tolerances to the device
    norm_fin(FIN_RR, FIN_EN, spmv(c, 2, x, r, b, c->partials));
    if ((st = read_rr())) return st;
    for (int g = 0; g < G; ++g) {
      c->host_scal[(size_t)g * S_COUNT + S_XI] = xig[g];
      c->host_scal[(size_t)g * S_COUNT + S_TOL2] = tol2[g];
      flags[g] = rr[g] <= tol2[g] ? ACT_DONE : ACT_RUN;
    }
    if ((st = upload_scal())) return st;
    if ((st = write_active(c, flags))) return st;
    if (n_updating() > 0 && max_iter > 0) {
      precond(r, z);
      for (;;) {
        // x += xi C^{-1} r; r = b - A x; a grid below tolerance stops (DONE)
        const std::vector<int32_t> before = flags;
        launch_axpy_scal(B, c->scal, S_XI, c->active, x, z, s);
        norm_fin(FIN_RR_DONE, FIN_EN_DONE, spmv(c, 2, x, r, b, c->partials));
        if ((st = enqueue_readback())) return st;
        ++it;
        if (it < max_iter) precond(r, z);  // next iteration's, speculatively
        if ((st = wait_readback())) return st;
        for (int g = 0; g < G; ++g) {
          its[g] += act_updating(before[g]);
          flags[g] = hflags[g];
        }
        c->active_shadow = flags;
        if (n_updating() == 0 || it >= max_iter) break;
      }
    }
  } else {
    // an iterative coarse solve varies the preconditioner slightly between
    // applications: the flexible update keeps the directions conjugate
    const bool flex = method == SFCDD_FCG || c->coarse_iter;
    const int fin_rz = flex ? FIN_RZ_NEXT_FLEX : FIN_RZ_NEXT;
    // r = b - A x
    norm_fin(FIN_RR, FIN_EN, spmv(c, 2, x, r, b, c->partials));
    if ((st = read_rr())) return st;
    for (int g = 0; g < G; ++g) {
      c->host_scal[(size_t)g * S_COUNT + S_TOL2] = tol2[g];
      flags[g] = rr[g] <= tol2[g] ? ACT_DONE : ACT_RUN;
    }
    if (n_updating() > 0 && max_iter > 0) {
      if ((st = upload_scal())) return st;
      if ((st = write_active(c, flags))) return st;
      // z = C^{-1} r, p = z
      precond_dot(r, z, r, nullptr);
      launch_finalize(B, FIN_RZ_INIT, c->partials, c->scal, c->active, s);
      launch_copy(N, z, p, s);
      for (;;) {
        // step: x += alpha p, r -= alpha q; a grid whose recursive residual is
        // below tolerance is frozen (CAND) until its true residual is checked
        const std::vector<int32_t> before = flags;
        const int np = spmv(c, 1, p, q, nullptr, c->partials);
        launch_finalize(B, FIN_PQ_ALPHA, c->partials, c->scal, c->active, s, np);
        launch_update_xr(B, c->scal, c->active, x, r, p, q, c->partials, s);
        norm_fin(FIN_RR_CAND, FIN_EN_CAND, 0);
        if ((st = enqueue_readback())) return st;
        ++it;
        if (it < max_iter) {
          // next direction, enqueued before the host has seen the residuals
          precond_dot(r, z, r, flex ? q : nullptr);
          launch_finalize(B, fin_rz, c->partials, c->scal, c->active, s);
          launch_update_p(B, c->scal, c->active, p, z, s);
        }
        if ((st = wait_readback())) return st;
        bool check = false;
        for (int g = 0; g < G; ++g) {
          its[g] += act_updating(before[g]);
          flags[g] = hflags[g];
          if (!std::isfinite(rr[g]) && act_updating(before[g]))
            FAIL(c, SFCDD_ENOTCONV, "residual of grid %d is not finite", g);
          if (flags[g] == ACT_CAND || (it >= max_iter && act_updating(flags[g]))) check = true;
        }
        c->active_shadow = flags;
        if (check && recursive) {
          // the recursive residual decides: candidates are done
          for (int g = 0; g < G; ++g)
            if (flags[g] == ACT_CAND || (it >= max_iter && act_updating(flags[g]))) flags[g] = ACT_DONE;
          if ((st = write_active(c, flags))) return st;
        } else if (check) {
          // confirm on the true residual; a grid whose true residual is still
          // too large restarts from its current x (residual replacement),
          // unless it has not halved since the grid's previous restart
          const int np = spmv(c, 2, x, tmp, b, c->partials);
          launch_finalize(B, FIN_TRR, c->partials, c->scal, nullptr, s, np);
          if ((st = read_scal(c))) return st;
          std::vector<int32_t> pass(G, ACT_SKIP);
          bool any_restart = false;
          for (int g = 0; g < G; ++g) {
            if (flags[g] != ACT_CAND && !(it >= max_iter && act_updating(flags[g]))) continue;
            const double trr = hs(c, g, S_TRR);
            rr[g] = trr;
            if (trr <= tol2[g]) {
              flags[g] = ACT_DONE;
            } else if (flags[g] == ACT_CAND && trr > 0.25 * last_trr[g]) {
              flags[g] = ACT_DONE;  // rounding floor reached
              stagnated[g] = 1;
            } else if (flags[g] == ACT_CAND && it < max_iter && restarts < 8 * G) {
              last_trr[g] = trr;
              const GridDesc& gd = c->grid[g].desc;
              launch_copy(gd.N, tmp + gd.goff, r + gd.goff, s);
              flags[g] = ACT_RESTART;
              pass[g] = ACT_RESTART;
              any_restart = true;
              ++restarts;
            } else {
              flags[g] = ACT_DONE;  // max_iter reached
            }
          }
          if (any_restart) {
            // z = C^{-1} r and p = z for the restarted grids only
            if ((st = write_active(c, pass))) return st;
            precond_dot(r, z, r, flex ? q : nullptr);
            launch_finalize(B, fin_rz, c->partials, c->scal, c->active, s);
            launch_update_p(B, c->scal, c->active, p, z, s);
          }
          if ((st = write_active(c, flags))) return st;
        }
        if (n_updating() == 0 || it >= max_iter) break;
      }
    }
  }
  if (c->layout == 1) launch_copy(N, x, x_io, s);
  else launch_permute(N, c->sfc_index, x, x_io, 0, s);
  HIPCHK(c, hipStreamSynchronize(s));
  prof_collect(c);
  c->last_iters = its;
  c->last_relres.assign(G, 0.0);
  bool conv = true, stag_only = true;
  double worst = 0.0;
  int itmax = 0;
  for (int g = 0; g < G; ++g) {
    const double rel = bb[g] > 0 ? std::sqrt(rr[g] / bb[g]) : std::sqrt(rr[g]);
    c->last_relres[g] = rel;
    worst = std::max(worst, rel);
    itmax = std::max(itmax, its[g]);
    if (rr[g] > tol2[g]) {
      conv = false;
      if (!stagnated[g]) stag_only = false;
    }
  }
  inf.iterations = itmax;
  inf.restarts = restarts;
  inf.rel_residual = worst;
  inf.coarse_steps = c->ic_max_steps;
  inf.coarse_unconverged = c->ic_unconv;
  if (info) *info = inf;
  if (!conv && stag_only)
    FAIL(c, SFCDD_ESTAGNATED, "true residual stagnated at %.3e above rtol %.1e after %d iterations "
         "(the FP64 rounding floor of the grid)", worst, rtol, itmax);
  if (!conv) FAIL(c, SFCDD_ENOTCONV, "not converged after %d iterations (rel. residual %.3e)", itmax, worst);
  return SFCDD_OK;
}

sfcdd_status sfcdd_get_batch_stats(sfcdd_ctx* c, int32_t* iterations, double* rel_residual) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  for (int g = 0; g < c->G; ++g) {
    if (iterations) iterations[g] = g < (int)c->last_iters.size() ? c->last_iters[g] : 0;
    if (rel_residual) rel_residual[g] = g < (int)c->last_relres.size() ? c->last_relres[g] : 0.0;
  }
  return SFCDD_OK;
}

sfcdd_status sfcdd_grad_coeff(sfcdd_ctx* c, const double* lam, const double* u, double* grad_a) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (!lam || !u || !grad_a) FAIL(c, SFCDD_EINVAL, "NULL argument");
  if (c->G != 1) FAIL(c, SFCDD_EINVAL, "the coefficient gradient is defined for a single grid");
  const hipStream_t s = c->stream;
  const int64_t N = c->Ntot;
  const GridDesc& g = c->grid[0].desc;
  const double *L = lam, *U = u;
  if (c->layout == 1) {  // to natural order
    launch_permute(N, c->sfc_index, lam, c->vec[V_IN], 0, s);
    launch_permute(N, c->sfc_index, u, c->vec[V_OUT], 0, s);
    L = c->vec[V_IN];
    U = c->vec[V_OUT];
  }
  launch_grad_coeff(g, L, U, c->partials, s);
  launch_finalize_vec(g.d, c->partials, c->gout, s);
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->gout, 8 * g.d, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int j = 0; j < g.d; ++j) grad_a[j] = -g.inv_h2[j] * c->host_scal[j];
  return SFCDD_OK;
}

sfcdd_status sfcdd_get_partition(sfcdd_ctx* c, int32_t grid, int32_t* sfc_index_host,
                                 int64_t* ta_host, int64_t* Ni_host, double* omega_host,
                                 int32_t* q_out) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (grid < 0 || grid >= c->G) FAIL(c, SFCDD_EINVAL, "grid %d out of range", grid);
  const GridHost& h = c->grid[grid];
  if (sfc_index_host) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(sfc_index_host, c->sfc_index + h.desc.goff, 4 * h.desc.N, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < h.desc.N; ++k) sfc_index_host[k] -= (int32_t)h.desc.goff;
  }
  for (int i = 0; i < h.desc.P; ++i) {
    if (ta_host) ta_host[i] = h.ta[i];
    if (Ni_host) Ni_host[i] = h.Ni[i];
    if (omega_host) omega_host[i] = h.omega[i];
  }
  if (q_out) *q_out = h.desc.q;
  return SFCDD_OK;
}

sfcdd_status sfcdd_partition_host(const sfcdd_params* params, int64_t* ta_host, int64_t* Ni_host,
                                  double* omega_host, int32_t* q_out) {
  GridHost h;
  std::string e;
  const sfcdd_status st = plan_grid(h, params, e);
  if (st != SFCDD_OK) {
    g_last_error = e;
    return st;
  }
  for (int i = 0; i < h.desc.P; ++i) {
    if (ta_host) ta_host[i] = h.ta[i];
    if (Ni_host) Ni_host[i] = h.Ni[i];
    if (omega_host) omega_host[i] = h.omega[i];
  }
  if (q_out) *q_out = h.desc.q;
  return SFCDD_OK;
}

sfcdd_status sfcdd_ct_layout(int32_t d, int32_t L, int32_t phat, int32_t capacity, int32_t* ngrids,
                             int32_t* levels, int32_t* layer, double* weight, int32_t* P) {
  sfcdd_ctx* none = nullptr;
  if (!ngrids) FAIL(none, SFCDD_EINVAL, "ngrids is NULL");
  if (d < 1 || d > MAXD) FAIL(none, SFCDD_EINVAL, "d = %d out of range 1..%d", d, MAXD);
  if (L < 1 || L > 60) FAIL(none, SFCDD_EINVAL, "L = %d out of range 1..60", L);
  if (phat < 1) FAIL(none, SFCDD_EINVAL, "phat = %d must be >= 1", phat);
  // layer i: the level vectors with l_j >= 1 and |l|_1 = L + d - 1 - i, in
  // lexicographic order (first entry slowest)
  std::vector<int32_t> lv;
  std::vector<int32_t> lay;
  std::vector<int32_t> cur(d);
  for (int i = 0; i < d; ++i) {
    const int total = L + d - 1 - i;
    // odometer over the first d - 1 entries; the last takes the rest
    std::function<void(int, int)> rec = [&](int k, int left) {
      if (k == d - 1) {
        if (left >= 1) {
          cur[k] = left;
          lv.insert(lv.end(), cur.begin(), cur.end());
          lay.push_back(i);
        }
        return;
      }
      for (int v = 1; v <= left - (d - 1 - k); ++v) {
        cur[k] = v;
        rec(k + 1, left - v);
      }
    };
    rec(0, total);
  }
  const int64_t n = (int64_t)lay.size();
  if (n > INT32_MAX) FAIL(none, SFCDD_EOVERFLOW, "more than 2^31 grids");
  *ngrids = (int32_t)n;
  if (!levels && !layer && !weight && !P) return SFCDD_OK;
  if (capacity < n) FAIL(none, SFCDD_ENOMEM, "capacity %d < %lld grids", capacity, (long long)n);
  for (int64_t k = 0; k < n; ++k) {
    const int i = lay[k];
    // binom(d - 1, i) exactly, then the sign of the layer
    double b = 1.0;
    for (int t = 1; t <= i; ++t) b = b * (double)(d - t) / (double)t;
    const double w = (i % 2 ? -1.0 : 1.0) * std::round(b);
    // P = phat 2^(d-1-i) (eq. Pchoice), at most the grid's point count
    int64_t Pk = (int64_t)phat << (d - 1 - i);
    int64_t N = 1;
    for (int j = 0; j < d; ++j) {
      const int64_t nj = (int64_t(1) << lv[k * d + j]) - 1;
      N = N > INT64_MAX / nj ? INT64_MAX : N * nj;
    }
    Pk = std::min<int64_t>(std::min<int64_t>(Pk, N), INT32_MAX);
    if (levels) std::memcpy(levels + k * d, lv.data() + k * d, sizeof(int32_t) * d);
    if (layer) layer[k] = i;
    if (weight) weight[k] = w;
    if (P) P[k] = (int32_t)std::max<int64_t>(1, Pk);
  }
  return SFCDD_OK;
}

sfcdd_status sfcdd_autotune(sfcdd_ctx* c, int32_t repeats, double* best_ms) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  sfcdd_tuning r{};
  const sfcdd_status st = tune_shapes(c, repeats, SFCDD_TUNE_TRSV, &r);
  if (st != SFCDD_OK) return st;
  if (best_ms) *best_ms = r.trsv_ms;
  return SFCDD_OK;
}

sfcdd_status sfcdd_tune(sfcdd_ctx* c, int32_t repeats, int32_t what, sfcdd_tuning* report) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (what & ~SFCDD_TUNE_ALL) FAIL(c, SFCDD_EINVAL, "what = %d", what);
  sfcdd_tuning r{};
  const sfcdd_status st = tune_shapes(c, repeats, what, &r);
  if (st != SFCDD_OK) return st;
  if (report) *report = r;
  return SFCDD_OK;
}

sfcdd_status sfcdd_set_profiling(sfcdd_ctx* c, int32_t on) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->ev_used = 0;
  for (int k = 0; k < SFCDD_K_COUNT; ++k) {
    c->k_ms[k] = 0.0;
    c->k_n[k] = 0;
  }
  c->prof = on != 0;
  return SFCDD_OK;
}

sfcdd_status sfcdd_get_kernel_time(sfcdd_ctx* c, int32_t kind, double* total_ms, int64_t* launches) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  if (kind < 0 || kind >= SFCDD_K_COUNT) FAIL(c, SFCDD_EINVAL, "kind = %d", kind);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (total_ms) *total_ms = c->k_ms[kind];
  if (launches) *launches = c->k_n[kind];
  return SFCDD_OK;
}

sfcdd_status sfcdd_get_info(sfcdd_ctx* c, sfcdd_info* info) {
  if (!c || !info) FAIL(c, SFCDD_EINVAL, "NULL argument");
  *info = c->info;
  info->coarse_steps = c->ic_k;
  return SFCDD_OK;
}

sfcdd_status sfcdd_ct_combine(sfcdd_ctx* c, const double* weights, const double* u, const double* x,
                              int64_t M, double* out) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  LIVE(c);
  if (M < 0 || (M > 0 && (!weights || !u || !x || !out))) FAIL(c, SFCDD_EINVAL, "ct_combine: NULL argument");
  const int d = c->grid[0].desc.d;
  for (int g = 1; g < c->G; ++g)
    if (c->grid[g].desc.d != d) FAIL(c, SFCDD_EINVAL, "ct_combine: grids of different dimension");
  if (d > 10) FAIL(c, SFCDD_EINVAL, "ct_combine: d = %d > 10", d);
  if (M == 0) return SFCDD_OK;
  launch_ct_combine(c->batch(), c->layout, c->pos, weights, u, x, M, out, c->stream);
  HIPCHK(c, hipGetLastError());
  return SFCDD_OK;
}

sfcdd_status sfcdd_read_probe(const void* buf, size_t bytes, void* hip_stream, int32_t repeats,
                              double* best_ms) {
  sfcdd_ctx* c = nullptr;
  if (!buf || !best_ms || bytes == 0 || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(buf) & 15) != 0 ||
      repeats < 1)
    FAIL(c, SFCDD_EINVAL, "read probe: need a 16-byte aligned buffer, bytes a positive multiple of 16, repeats >= 1");
  const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  double best = 1e300;
  launch_read_probe(buf, (int64_t)bytes, s);  // warm-up
  for (int r = 0; r < repeats; ++r) {
    (void)hipEventRecord(e0, s);
    launch_read_probe(buf, (int64_t)bytes, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(c, hipGetLastError());
  if (!(best < 1e300)) FAIL(c, SFCDD_EDEVICE, "read probe: timing failed");
  *best_ms = best;
  return SFCDD_OK;
}

sfcdd_status sfcdd_destroy(sfcdd_ctx* c) {
  if (!c) return SFCDD_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->host_scal && !c->noalloc) (void)hipHostFree(c->host_scal);
  if (c->ev_rb) (void)hipEventDestroy(c->ev_rb);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);

  delete c;
  return SFCDD_OK;
}

const char* sfcdd_last_error(const sfcdd_ctx* c) {
  return c ? c->err.c_str() : g_last_error.c_str();
}

}  // extern "C"
