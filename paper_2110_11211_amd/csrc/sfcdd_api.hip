// Host side of the C ABI: validation, the closed-form partition, workspace
// layout, and the orchestration of setup (Alg. 1), operator application
// (Alg. 2, eqs. addSW / balSW) and the outer iterations (Alg. 3, PCG).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

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

}  // namespace

struct sfcdd_ctx {
  // parameters
  int d = 0;
  std::vector<int> levels, npts;
  std::vector<double> coeff;
  int P = 0, q = 0, N0 = 0;
  int64_t gnum = 0, gden = 1;
  int weighting = 1, variant = 1, fdtype = 0, local_solver = 0, layout = 0;
  GridDesc g{};
  PartDesc pd{};
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // internal, default priority: coarse setup overlaps the fine factorisation
  // host partition
  std::vector<int32_t> ta, Ni, nt;
  std::vector<int64_t> off, doff, xoff, poff;
  std::vector<double> omega;
  int max_nt = 0, max_Ni = 0, min_Ni = 0;
  int64_t sum_Ni = 0, tiles = 0, parts = 0, xlen = 0;
  int nt0 = 0;
  // workspace regions
  Region r_sfc, r_pos, r_nbr, r_ta, r_Ni, r_nt, r_off, r_doff, r_xoff, r_poff, r_omega, r_fac,
      r_facX, r_xloc, r_fpart, r_A0, r_X0, r_c0, r_d0, r_cpart, r_cmeta, r_dbuf, r_vec, r_partials,
      r_scal, r_status, r_gout, r_cpartk;
  size_t total = 0;
  unsigned char* ws = nullptr;
  // convenience device pointers
  int32_t *sfc_index = nullptr, *pos = nullptr, *nbr = nullptr;
  int32_t *d_ta = nullptr, *d_Ni = nullptr, *d_nt = nullptr;
  int64_t *d_off = nullptr, *d_doff = nullptr, *d_xoff = nullptr, *d_poff = nullptr;
  double* d_omega = nullptr;
  void *fac = nullptr, *facX = nullptr, *xloc = nullptr, *fpart = nullptr;
  double *A0 = nullptr, *X0 = nullptr, *c0 = nullptr, *d0 = nullptr, *cpart = nullptr;
  double* cpartk = nullptr;  // split-K partial tiles of the coarse factorisation
  int32_t *c_nt = nullptr, *c_n = nullptr;
  int64_t *c_off = nullptr, *c_xoff = nullptr, *c_poff = nullptr, *c_doff = nullptr;
  double* dbuf = nullptr;
  double* vec[NVEC] = {};
  double *partials = nullptr, *scal = nullptr, *gout = nullptr;
  int32_t* status = nullptr;
  double* host_scal = nullptr;  // pinned
  std::string err;
  sfcdd_info info{};
  // per-kernel profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double k_ms[SFCDD_K_COUNT] = {};
  int64_t k_n[SFCDD_K_COUNT] = {};
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

// Parameter validation and the host partition (eqs. dof, sloc, enlarge,
// omegai, restr).  Fills everything in ctx except device pointers.
sfcdd_status plan(sfcdd_ctx* c, const sfcdd_params* p) {
  if (!p) FAIL(c, SFCDD_EINVAL, "params is NULL");
  if (p->d < 1 || p->d > MAXD) FAIL(c, SFCDD_EINVAL, "d = %d out of range 1..%d", p->d, MAXD);
  if ((p->level == nullptr) == (p->npts == nullptr))
    FAIL(c, SFCDD_EINVAL, "give exactly one of level / npts");
  c->d = p->d;
  c->levels.clear();
  c->npts.clear();
  GridDesc& g = c->g;
  memset(&g, 0, sizeof(g));
  g.d = p->d;
  int nres = 0;
  for (int j = 0; j < p->d; ++j) {
    int n;
    if (p->level) {
      const int l = p->level[j];
      if (l < 1 || l > 30) FAIL(c, SFCDD_EINVAL, "level[%d] = %d out of range 1..30", j, l);
      c->levels.push_back(l);
      n = (1 << l) - 1;
      nres = std::max(nres, l);
    } else {
      n = p->npts[j];
      if (n < 1) FAIL(c, SFCDD_EINVAL, "npts[%d] = %d < 1", j, n);
      c->npts.push_back(n);
    }
    g.n[j] = n;
  }
  if (!p->level) {
    int mx = 0;
    for (int j = 0; j < p->d; ++j) mx = std::max(mx, g.n[j]);
    while ((int64_t(1) << nres) < (int64_t)mx + 1) ++nres;
    if (nres < 1) nres = 1;
  }
  if ((int64_t)nres * p->d > 64)
    FAIL(c, SFCDD_EOVERFLOW, "Morton key needs %d bits > 64", nres * p->d);
  g.nres = nres;
  int64_t N = 1;
  for (int j = 0; j < p->d; ++j) {
    g.stride[j] = N;
    N *= g.n[j];
    if (N >= (int64_t(1) << 31)) FAIL(c, SFCDD_EOVERFLOW, "N >= 2^31");
    g.shift[j] = p->level ? nres - p->level[j] : 0;
  }
  g.N = N;
  c->coeff.assign(p->d, 1.0);
  if (p->coeff)
    for (int j = 0; j < p->d; ++j) {
      if (!(p->coeff[j] > 0.0) || !std::isfinite(p->coeff[j]))
        FAIL(c, SFCDD_EINVAL, "coeff[%d] must be positive and finite", j);
      c->coeff[j] = p->coeff[j];
    }
  double diag = 0.0;
  for (int j = 0; j < p->d; ++j) {
    const double ih2 = (double)((int64_t)(g.n[j] + 1) * (g.n[j] + 1));
    g.inv_h2[j] = ih2;
    g.c[j] = c->coeff[j] * ih2;
    diag += 2.0 * g.c[j];
  }
  g.diag = diag;

  if (p->P < 1 || p->P > N) FAIL(c, SFCDD_EINVAL, "P = %d must satisfy 1 <= P <= N = %lld", p->P, (long long)N);
  if (p->gamma_den < 1 || p->gamma_den > (int64_t(1) << 30) || p->gamma_num < 0)
    FAIL(c, SFCDD_EINVAL, "gamma = %lld/%lld must be >= 0 with 1 <= den <= 2^30",
         (long long)p->gamma_num, (long long)p->gamma_den);
  if (p->weighting != SFCDD_WEIGHT_NONE && p->weighting != SFCDD_WEIGHT_OMEGA)
    FAIL(c, SFCDD_EINVAL, "weighting = %d", p->weighting);
  if (p->variant != SFCDD_ADDITIVE && p->variant != SFCDD_BALANCED)
    FAIL(c, SFCDD_EINVAL, "variant = %d", p->variant);
  if (p->factor_dtype != SFCDD_FP64 && p->factor_dtype != SFCDD_FP32)
    FAIL(c, SFCDD_EINVAL, "factor_dtype = %d", p->factor_dtype);
  if (p->local_solver != SFCDD_LOCAL_CHOLESKY && p->local_solver != SFCDD_LOCAL_INVERSE)
    FAIL(c, SFCDD_EINVAL, "local_solver = %d", p->local_solver);
  if (p->layout != 0 && p->layout != 1) FAIL(c, SFCDD_EINVAL, "layout = %d", p->layout);
  c->P = p->P;
  c->gnum = p->gamma_num;
  c->gden = p->gamma_den;
  c->weighting = p->weighting;
  c->variant = p->variant;
  c->fdtype = p->factor_dtype;
  c->local_solver = p->local_solver;
  c->layout = p->layout;

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
    qq = std::min<int64_t>(qq, std::max<int64_t>(1, 16384 / P));
    qq = std::min<int64_t>(qq, base);
    q = (int)std::max<int64_t>(1, qq);
  }
  if (q < 1 || q > base) FAIL(c, SFCDD_EINVAL, "q = %d must satisfy 1 <= q <= floor(N/P) = %lld", q, (long long)base);
  if ((int64_t)q * P > (int64_t(1) << 17))
    FAIL(c, SFCDD_EINVAL, "coarse size qP = %lld exceeds 131072", (long long)q * P);
  c->q = q;
  c->N0 = q * P;
  c->nt0 = (int)ceil_div(c->N0, TS);

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
  c->ta.assign(P, 0);
  c->Ni.assign(P, 0);
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
      c->ta[i] = 0;
      c->Ni[i] = (int32_t)N;
    } else {
      int64_t t = (start_of(i - F) - nl) % N;
      if (t < 0) t += N;
      c->ta[i] = (int32_t)t;
      c->Ni[i] = (int32_t)len;
    }
  }
  // multiplicities and omega_i = 1 / min_{p in Omega_i} m_p (eq. omegai)
  c->omega.assign(P, 1.0);
  if (c->weighting == SFCDD_WEIGHT_OMEGA) {
    std::vector<int32_t> m(N + 1, 0);
    for (int i = 0; i < P; ++i) {
      const int64_t a = c->ta[i], e = a + c->Ni[i];
      if (e <= N) {
        m[a] += 1;
        m[e] -= 1;
      } else {
        m[a] += 1;
        m[N] -= 1;
        m[0] += 1;
        m[e - N] -= 1;
      }
    }
    for (int64_t k = 1; k < N; ++k) m[k] += m[k - 1];
    for (int i = 0; i < P; ++i) {
      int32_t mn = INT32_MAX;
      const int64_t a = c->ta[i];
      for (int64_t s = 0; s < c->Ni[i]; ++s) {
        int64_t q2 = a + s;
        if (q2 >= N) q2 -= N;
        mn = std::min(mn, m[q2]);
      }
      c->omega[i] = 1.0 / (double)mn;
    }
  }
  // tiles and offsets
  c->nt.assign(P, 0);
  c->off.assign(P, 0);
  c->doff.assign(P, 0);
  c->xoff.assign(P, 0);
  c->poff.assign(P, 0);
  int64_t toff = 0, dof = 0, xof = 0, pof = 0;
  c->max_nt = 0;
  c->max_Ni = 0;
  c->min_Ni = INT32_MAX;
  for (int i = 0; i < P; ++i) {
    const int ntb = (int)ceil_div(c->Ni[i], TS);
    c->nt[i] = ntb;
    c->off[i] = toff;
    c->doff[i] = dof;
    c->xoff[i] = xof;
    c->poff[i] = pof;
    toff += (int64_t)ntb * (ntb + 1) / 2;
    dof += c->Ni[i];
    xof += (int64_t)ntb * TS;
    pof += (int64_t)ntb * ntb * TS;
    c->max_nt = std::max(c->max_nt, ntb);
    c->max_Ni = std::max(c->max_Ni, c->Ni[i]);
    c->min_Ni = std::min(c->min_Ni, c->Ni[i]);
  }
  c->tiles = toff;
  c->sum_Ni = dof;
  c->xlen = xof;
  c->parts = pof;
  if (c->max_nt * TS > 8192)
    FAIL(c, SFCDD_EINVAL, "largest subdomain N_i = %d exceeds 8192 points", c->max_Ni);

  PartDesc& pdsc = c->pd;
  pdsc.P = P;
  pdsc.q = q;
  pdsc.N0 = c->N0;
  pdsc.base = base;
  pdsc.rem = rem;
  pdsc.F = (int)std::min<int64_t>(F, P);
  pdsc.ncand = (int)std::min<int64_t>(P, 2 * F + 3);

  // workspace layout
  const size_t es = c->fdtype == SFCDD_FP32 ? 4 : 8;
  const int64_t ct = (int64_t)c->nt0 * (c->nt0 + 1) / 2;
  Planner pl;
  c->r_sfc = pl.take(4 * N);
  c->r_pos = pl.take(4 * N);
  c->r_nbr = pl.take((size_t)8 * p->d * N);
  c->r_ta = pl.take(4 * P);
  c->r_Ni = pl.take(4 * P);
  c->r_nt = pl.take(4 * P);
  c->r_off = pl.take(8 * P);
  c->r_doff = pl.take(8 * P);
  c->r_xoff = pl.take(8 * P);
  c->r_poff = pl.take(8 * P);
  c->r_omega = pl.take(8 * P);
  c->r_fac = pl.take((size_t)c->tiles * TS2 * es);
  const bool inv = c->local_solver == SFCDD_LOCAL_INVERSE;
  c->r_facX = pl.take(inv ? (size_t)c->tiles * TS2 * es : 0);
  c->r_xloc = pl.take(inv ? (size_t)c->xlen * es : 0);
  c->r_fpart = pl.take(inv ? (size_t)c->parts * es : 0);
  c->r_A0 = pl.take((size_t)ct * TS2 * 8);
  c->r_X0 = pl.take((size_t)ct * TS2 * 8);
  c->r_c0 = pl.take((size_t)c->nt0 * TS * 8);
  c->r_d0 = pl.take((size_t)c->nt0 * TS * 8);
  c->r_cpart = pl.take((size_t)c->nt0 * c->nt0 * TS * 8);
  c->r_cmeta = pl.take(64);
  c->r_cpartk = pl.take((size_t)c->nt0 * ((c->nt0 + SPLITK - 1) / SPLITK) * TS2 * 8);
  c->r_dbuf = pl.take((size_t)c->sum_Ni * 8);
  c->r_vec = pl.take((size_t)NVEC * (((size_t)N * 8 + 255) & ~size_t(255)));
  c->r_partials = pl.take((size_t)MAXD * RED_BLOCKS * 8);
  c->r_scal = pl.take(S_COUNT * 8);
  c->r_status = pl.take(64);
  c->r_gout = pl.take(MAXD * 8);
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
  c->d_ta = at<int32_t>(c, c->r_ta);
  c->d_Ni = at<int32_t>(c, c->r_Ni);
  c->d_nt = at<int32_t>(c, c->r_nt);
  c->d_off = at<int64_t>(c, c->r_off);
  c->d_doff = at<int64_t>(c, c->r_doff);
  c->d_xoff = at<int64_t>(c, c->r_xoff);
  c->d_poff = at<int64_t>(c, c->r_poff);
  c->d_omega = at<double>(c, c->r_omega);
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
  unsigned char* cm = c->ws + c->r_cmeta.off;
  c->c_off = reinterpret_cast<int64_t*>(cm);       // 0
  c->c_xoff = reinterpret_cast<int64_t*>(cm + 8);  // 0
  c->c_poff = reinterpret_cast<int64_t*>(cm + 16); // 0
  c->c_doff = reinterpret_cast<int64_t*>(cm + 24); // 0
  c->c_nt = reinterpret_cast<int32_t*>(cm + 32);
  c->c_n = reinterpret_cast<int32_t*>(cm + 36);
  c->dbuf = at<double>(c, c->r_dbuf);
  const size_t vstride = ((size_t)c->g.N * 8 + 255) & ~size_t(255);
  for (int k = 0; k < NVEC; ++k)
    c->vec[k] = reinterpret_cast<double*>(c->ws + c->r_vec.off + k * vstride);
  c->partials = at<double>(c, c->r_partials);
  c->scal = at<double>(c, c->r_scal);
  c->status = at<int32_t>(c, c->r_status);
  c->gout = at<double>(c, c->r_gout);
}

// Batched left-looking tiled Cholesky of nb packed matrices (+ optional
// inversion into M = A^{-1} via X = L^{-1}, M = X^T X).
// Batched left-looking factorisation: each workgroup keeps its output tile in
// registers across the K loop.  A single matrix (part != nullptr) uses the
// split-K form instead, so that every column step runs on many workgroups.
template <typename T>
void factor_batch(int nb, int max_nt, const int32_t* nt, const int64_t* off, T* fac, T* X,
                  bool invert, int32_t* status, T* part, hipStream_t s) {
  const int maxc = (max_nt + SPLITK - 1) / SPLITK;
  for (int J = 0; J < max_nt; ++J) {
    if (part) {
      launch_potrf_partial<T>(J, max_nt, maxc, nt, off, fac, part, s);
      const int np = (J + SPLITK - 1) / SPLITK;
      launch_potrf_diag<T>(J, 0, np, maxc, part, 1, nt, off, fac, status, s);
      launch_potrf_panel<T>(J, 0, np, maxc, part, 1, max_nt, nt, off, fac, s);
    } else {
      launch_potrf_diag<T>(J, 1, 0, 0, (const T*)nullptr, nb, nt, off, fac, status, s);
      launch_potrf_panel<T>(J, 1, 0, 0, (const T*)nullptr, nb, max_nt, nt, off, fac, s);
    }
  }
  if (invert) {
    for (int J = max_nt - 1; J >= 0; --J) {
      if (part) launch_trtri_splitk<T>(J, max_nt, maxc, nt, off, fac, X, part, s);
      else launch_trtri_col<T>(J, nb, max_nt, nt, off, fac, X, s);
    }
    launch_lauum<T>(nb, max_nt, nt, off, X, fac, s);
  }
}

// F v = R_0^T A_0^{-1} R_0 v: restriction into c0, then d0 = A_0^{-1} c0.
void coarse_solve(sfcdd_ctx* c, const double* v) {
  ProfScope ps(c, SFCDD_K_COARSE);
  BatchMeta bm{c->c_nt, c->c_off, c->c_xoff, c->c_poff};
  launch_restrict(c->pd, v, c->c0, c->stream);
  launch_symv_tiles<double>(1, c->nt0, bm, c->A0, c->c0, c->cpart, c->stream);
  launch_symv_reduce<double>(1, c->N0, bm, c->c_n, c->c_doff, c->cpart, c->d0, c->stream);
}

// y = sum_i R_i^T omega_i A_i^{-1} R_i w (eq. w1levprec).
void fine_apply(sfcdd_ctx* c, const double* w, double* y) {
  const hipStream_t s = c->stream;
  {
  ProfScope ps(c, SFCDD_K_LOCAL_SOLVE);
  if (c->local_solver == SFCDD_LOCAL_CHOLESKY) {
    if (c->fdtype == SFCDD_FP32)
      launch_schwarz_trsv<float>(c->P, c->g.N, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_doff,
                                 c->max_nt, (const float*)c->fac, w, c->dbuf, s);
    else
      launch_schwarz_trsv<double>(c->P, c->g.N, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->d_doff,
                                  c->max_nt, (const double*)c->fac, w, c->dbuf, s);
  } else {
    BatchMeta bm{c->d_nt, c->d_off, c->d_xoff, c->d_poff};
    if (c->fdtype == SFCDD_FP32) {
      launch_gather_local<float>(c->P, c->g.N, c->max_nt, bm, c->d_ta, c->d_Ni, w, (float*)c->xloc, s);
      launch_symv_tiles<float>(c->P, c->max_nt, bm, (const float*)c->fac, (const float*)c->xloc,
                               (float*)c->fpart, s);
      launch_symv_reduce<float>(c->P, c->max_Ni, bm, c->d_Ni, c->d_doff, (const float*)c->fpart,
                                c->dbuf, s);
    } else {
      launch_gather_local<double>(c->P, c->g.N, c->max_nt, bm, c->d_ta, c->d_Ni, w, (double*)c->xloc, s);
      launch_symv_tiles<double>(c->P, c->max_nt, bm, (const double*)c->fac, (const double*)c->xloc,
                                (double*)c->fpart, s);
      launch_symv_reduce<double>(c->P, c->max_Ni, bm, c->d_Ni, c->d_doff, (const double*)c->fpart,
                                 c->dbuf, s);
    }
  }
  }
  ProfScope ps(c, SFCDD_K_SCATTER);
  launch_scatter(c->g, c->pd, c->d_ta, c->d_Ni, c->d_doff, c->d_omega, c->dbuf, y, s);
}

void spmv(sfcdd_ctx* c, const double* x, double* y, const double* b, double* partials) {
  ProfScope ps(c, SFCDD_K_SPMV);
  launch_spmv(c->g, c->nbr, x, y, b, partials, nullptr, c->stream);
}

// h = C^{-1} g in curve order (Alg. 2; balanced form eq. balSW).
void apply_s(sfcdd_ctx* c, const double* g, double* h) {
  const hipStream_t s = c->stream;
  if (c->variant == SFCDD_BALANCED) {
    double *t = c->vec[V_T], *w = c->vec[V_W], *y = c->vec[V_Y], *v = c->vec[V_V];
    coarse_solve(c, g);                                               // d0 = A0^{-1} R0 g
    launch_combine(c->g, c->pd, COMB_PROLONG, c->d0, nullptr, nullptr, t, s);  // t = F g
    spmv(c, t, w, g, c->partials);                                    // w = g - A t = G g
    fine_apply(c, w, y);                                              // y = C1^{-1} G g
    spmv(c, y, v, nullptr, nullptr);                                  // v = A y
    coarse_solve(c, v);                                               // d0 = A0^{-1} R0 A y
    launch_combine(c->g, c->pd, COMB_BAL_FINAL, c->d0, y, t, h, s);  // h = y - F A y + F g
  } else {
    coarse_solve(c, g);
    fine_apply(c, g, h);
    launch_combine(c->g, c->pd, COMB_ADD_PROLONG, c->d0, h, nullptr, h, s);
  }
}

sfcdd_status read_scal(sfcdd_ctx* c, int slot, double* out) {
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal + slot, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *out = c->host_scal[0];
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

}  // namespace

extern "C" {

sfcdd_status sfcdd_workspace_size(const sfcdd_params* params, size_t* bytes) {
  if (!bytes) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "bytes is NULL");
  sfcdd_ctx tmp;
  const sfcdd_status st = plan(&tmp, params);
  if (st != SFCDD_OK) {
    g_last_error = tmp.err;
    return st;
  }
  *bytes = tmp.total;
  return SFCDD_OK;
}

sfcdd_status sfcdd_setup(const sfcdd_params* params, void* workspace_dev, size_t bytes,
                         void* hip_stream, sfcdd_ctx** out) {
  if (!out) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!workspace_dev) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "workspace is NULL");
  sfcdd_ctx* c = new (std::nothrow) sfcdd_ctx();
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_ENOMEM, "host allocation failed");
  sfcdd_status st = plan(c, params);
  if (st != SFCDD_OK) {
    g_last_error = c->err;
    delete c;
    return st;
  }
  if (bytes < c->total) {
    g_last_error = "workspace too small: need " + std::to_string(c->total) + " bytes";
    delete c;
    return SFCDD_ENOMEM;
  }
  // align the base
  c->ws = reinterpret_cast<unsigned char*>((reinterpret_cast<uintptr_t>(workspace_dev) + 255) & ~uintptr_t(255));
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  bind(c);
  if (hipHostMalloc((void**)&c->host_scal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    g_last_error = "hipHostMalloc failed";
    delete c;
    return SFCDD_EDEVICE;
  }
  *out = c;
  const hipStream_t s = c->stream;
  const int P = c->P;
  hipEvent_t ev[6];
  for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
  HIPCHK(c, hipEventRecord(ev[0], s));

  // tables
  HIPCHK(c, hipMemcpyAsync(c->d_ta, c->ta.data(), 4 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_Ni, c->Ni.data(), 4 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_nt, c->nt.data(), 4 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_off, c->off.data(), 8 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_doff, c->doff.data(), 8 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_xoff, c->xoff.data(), 8 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_poff, c->poff.data(), 8 * P, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d_omega, c->omega.data(), 8 * P, hipMemcpyHostToDevice, s));
  {
    static thread_local int64_t zeros[4] = {0, 0, 0, 0};
    static thread_local int32_t cm[2];
    cm[0] = c->nt0;
    cm[1] = c->N0;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->r_cmeta.off, zeros, 32, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->c_nt, cm, 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  HIPCHK(c, hipMemsetAsync(c->status, 0, 64, s));

  // curve order and neighbours (Alg. 1: sfc_index, neighbour map)
  HIPCHK(c, hipMemsetAsync(c->sfc_index, 0, 4 * c->g.N, s));
  launch_sfc_rank(c->g, c->pos, c->sfc_index, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(ev[1], s));
  launch_build_nbr(c->g, c->pos, c->sfc_index, c->nbr, s);
  HIPCHK(c, hipEventRecord(ev[2], s));

  // The coarse setup (one matrix, latency-bound right-looking steps) runs on
  // an internal stream forked from the caller's, concurrently with the
  // batched subdomain factorisation; both join before setup returns.
  hipEvent_t fork, join;
  HIPCHK(c, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&join, hipEventDisableTiming));
  if (!c->side) HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIPCHK(c, hipEventRecord(fork, s));
  HIPCHK(c, hipStreamWaitEvent(c->side, fork, 0));
  hipEvent_t cev0, cev1;
  HIPCHK(c, hipEventCreate(&cev0));
  HIPCHK(c, hipEventCreate(&cev1));
  {
    const hipStream_t cs = c->side;
    HIPCHK(c, hipEventRecord(cev0, cs));
    // coarse matrix A_0 = R_0 A R_0^T = sum_j c_j E_j (eq. csm), then A_0^{-1}
    HIPCHK(c, hipMemsetAsync(c->A0, 0, c->r_A0.bytes, cs));
    HIPCHK(c, hipMemsetAsync(c->c0, 0, c->r_c0.bytes, cs));
    const int64_t ctiles_elems = (int64_t)c->nt0 * (c->nt0 + 1) / 2 * TS2;
    for (int j = 0; j < c->d; ++j) {
      HIPCHK(c, hipMemsetAsync(c->X0, 0, (size_t)ctiles_elems * 4, cs));
      launch_coarse_counts(c->g, c->pd, j, c->nbr, (int32_t*)c->X0, cs);
      launch_coarse_accumulate(ctiles_elems, c->g.c[j], (const int32_t*)c->X0, c->A0, cs);
    }
    launch_coarse_pad(c->N0, c->nt0, c->A0, cs);
    factor_batch<double>(1, c->nt0, c->c_nt, c->c_off, c->A0, c->X0, true, c->status + 1,
                         c->cpartk, cs);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(cev1, cs));
    HIPCHK(c, hipEventRecord(join, cs));
  }

  // local matrices A_i = R_i A R_i^T
  HIPCHK(c, hipMemsetAsync(c->fac, 0, c->r_fac.bytes, s));
  if (c->fdtype == SFCDD_FP32)
    launch_assemble_local<float>(c->g, P, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->nbr, c->max_nt,
                                 (float*)c->fac, s);
  else
    launch_assemble_local<double>(c->g, P, c->d_ta, c->d_Ni, c->d_nt, c->d_off, c->nbr, c->max_nt,
                                  (double*)c->fac, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(ev[3], s));

  // factor once (Sec. 3.1)
  const bool inv = c->local_solver == SFCDD_LOCAL_INVERSE;
  if (c->fdtype == SFCDD_FP32)
    factor_batch<float>(P, c->max_nt, c->d_nt, c->d_off, (float*)c->fac, (float*)c->facX, inv,
                        c->status, (float*)nullptr, s);
  else
    factor_batch<double>(P, c->max_nt, c->d_nt, c->d_off, (double*)c->fac, (double*)c->facX, inv,
                         c->status, (double*)nullptr, s);
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
  I.N = c->g.N;
  I.P = c->P;
  I.q = c->q;
  I.N0 = c->N0;
  I.max_Ni = c->max_Ni;
  I.min_Ni = c->min_Ni;
  I.tile = TS;
  I.sum_Ni = c->sum_Ni;
  const int64_t es = c->fdtype == SFCDD_FP32 ? 4 : 8;
  I.factor_bytes = c->tiles * TS2 * es;
  int64_t algo = 0;
  for (int i = 0; i < P; ++i) algo += (int64_t)c->Ni[i] * (c->Ni[i] + 1) / 2;
  I.factor_algo_bytes = algo * es;
  I.coarse_bytes = (int64_t)c->r_A0.bytes;
  for (int k = 0; k < 5; ++k) I.setup_ms[k] = ms[k];
  I.setup_ms[5] = tot;

  int32_t stat[2] = {0, 0};
  HIPCHK(c, hipMemcpy(stat, c->status, 8, hipMemcpyDeviceToHost));
  if (stat[0] != 0) FAIL(c, SFCDD_ENOTSPD, "a local matrix is not positive definite");
  if (stat[1] != 0) FAIL(c, SFCDD_ENOTSPD, "the coarse matrix is not positive definite");
  return SFCDD_OK;
}

sfcdd_status sfcdd_apply_precond(sfcdd_ctx* c, const double* g, double* h) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  if (!g || !h || g == h) FAIL(c, SFCDD_EINVAL, "g and h must be distinct non-NULL device vectors");
  const int64_t N = c->g.N;
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
  if (!x || !y || x == y) FAIL(c, SFCDD_EINVAL, "x and y must be distinct non-NULL device vectors");
  const int64_t N = c->g.N;
  if (c->layout == 1) {
    launch_spmv(c->g, c->nbr, x, y, nullptr, nullptr, nullptr, c->stream);
  } else {
    launch_permute(N, c->sfc_index, x, c->vec[V_IN], 1, c->stream);
    launch_spmv(c->g, c->nbr, c->vec[V_IN], c->vec[V_OUT], nullptr, nullptr, nullptr, c->stream);
    launch_permute(N, c->sfc_index, c->vec[V_OUT], y, 0, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  return SFCDD_OK;
}

sfcdd_status sfcdd_solve(sfcdd_ctx* c, const double* b_in, double* x_io, double rtol,
                         int32_t max_iter, int32_t method, double xi, sfcdd_solve_info* info) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  if (!b_in || !x_io || b_in == x_io) FAIL(c, SFCDD_EINVAL, "b and x must be distinct non-NULL device vectors");
  if (!(rtol > 0.0) || max_iter < 0) FAIL(c, SFCDD_EINVAL, "need rtol > 0 and max_iter >= 0");
  if (method != SFCDD_PCG && method != SFCDD_FCG && method != SFCDD_RICHARDSON)
    FAIL(c, SFCDD_EINVAL, "method = %d", method);
  const hipStream_t s = c->stream;
  const int64_t N = c->g.N;
  double *x = c->vec[V_X], *r = c->vec[V_R], *z = c->vec[V_Z], *p = c->vec[V_P], *q = c->vec[V_Q],
         *b = c->vec[V_B], *tmp = c->vec[V_TMP];
  if (c->layout == 1) {
    launch_copy(N, b_in, b, s);
    launch_copy(N, x_io, x, s);
  } else {
    launch_permute(N, c->sfc_index, b_in, b, 1, s);
    launch_permute(N, c->sfc_index, x_io, x, 1, s);
  }
  launch_dot(N, b, b, nullptr, c->partials, s);
  launch_finalize(FIN_BB, c->partials, c->scal, s);
  double bb;
  sfcdd_status st = read_scal(c, S_BB, &bb);
  if (st) return st;
  const double tol2 = rtol * rtol * bb;
  sfcdd_solve_info inf{};
  int it = 0, restarts = 0;
  bool conv = false;
  double rr = 0.0;

  if (method == SFCDD_RICHARDSON) {
    if (!(xi > 0.0)) {
      // Lanczos estimate of the extreme eigenvalues of C^{-1}A from CG steps
      std::vector<double> al, be;
      launch_zero(N, z, s);  // z used as x of the estimation run
      launch_copy(N, b, r, s);
      apply_s(c, r, q);
      launch_copy(N, q, p, s);
      launch_dot(N, r, q, nullptr, c->partials, s);
      launch_finalize(FIN_RZ_INIT, c->partials, c->scal, s);
      for (int k = 0; k < 30; ++k) {
        spmv(c, p, tmp, nullptr, c->partials);
        launch_finalize(FIN_PQ_ALPHA, c->partials, c->scal, s);
        launch_update_xr(N, c->scal, z, r, p, tmp, c->partials, s);
        double a_k;
        if ((st = read_scal(c, S_ALPHA, &a_k))) return st;
        if (!(a_k > 0.0) || !std::isfinite(a_k)) break;
        al.push_back(a_k);
        apply_s(c, r, q);
        launch_dot(N, r, q, nullptr, c->partials, s);
        launch_finalize(FIN_RZ_NEXT, c->partials, c->scal, s);
        double b_k;
        if ((st = read_scal(c, S_BETA, &b_k))) return st;
        if (!(b_k > 0.0) || !std::isfinite(b_k)) break;
        be.push_back(b_k);
        launch_update_p(N, c->scal, p, q, s);
      }
      const int m = (int)al.size();
      if (m == 0) FAIL(c, SFCDD_ENOTCONV, "Lanczos estimate failed");
      std::vector<double> ta(m), tb(m > 1 ? m - 1 : 0);
      for (int k = 0; k < m; ++k) ta[k] = 1.0 / al[k] + (k > 0 ? be[k - 1] / al[k - 1] : 0.0);
      for (int k = 0; k + 1 < m; ++k) tb[k] = std::sqrt(be[k]) / al[k];
      double lmin, lmax;
      tridiag_extremes(ta, tb, &lmin, &lmax);
      inf.lambda_min = lmin;
      inf.lambda_max = lmax;
      xi = 2.0 / (lmin + lmax);
    }
    inf.xi = xi;
    double* hx = c->host_scal + 8;
    hx[0] = xi;
    HIPCHK(c, hipMemcpyAsync(c->scal + S_XI, hx, 8, hipMemcpyHostToDevice, s));
    for (;;) {
      spmv(c, x, r, b, c->partials);
      launch_finalize(FIN_RR, c->partials, c->scal, s);
      if ((st = read_scal(c, S_RR, &rr))) return st;
      if (rr <= tol2) { conv = true; break; }
      if (it >= max_iter) break;
      apply_s(c, r, z);
      launch_axpy_scal(N, c->scal, S_XI, x, z, s);
      ++it;
    }
  } else {
    const bool flex = method == SFCDD_FCG;
    bool fresh = true;
    while (true) {
      if (fresh) {
        spmv(c, x, r, b, c->partials);
        launch_finalize(FIN_RR, c->partials, c->scal, s);
        if ((st = read_scal(c, S_RR, &rr))) return st;
        if (rr <= tol2) { conv = true; break; }
        if (it >= max_iter) break;
        apply_s(c, r, z);
        launch_dot(N, r, z, nullptr, c->partials, s);
        launch_finalize(FIN_RZ_INIT, c->partials, c->scal, s);
        launch_copy(N, z, p, s);
        fresh = false;
      }
      spmv(c, p, q, nullptr, c->partials);
      launch_finalize(FIN_PQ_ALPHA, c->partials, c->scal, s);
      launch_update_xr(N, c->scal, x, r, p, q, c->partials, s);
      launch_finalize(FIN_RR, c->partials, c->scal, s);
      ++it;
      if ((st = read_scal(c, S_RR, &rr))) return st;
      if (!std::isfinite(rr)) FAIL(c, SFCDD_ENOTCONV, "residual is not finite");
      if (rr <= tol2 || it >= max_iter) {
        // confirm on the true residual; restart from x when they disagree
        spmv(c, x, tmp, b, c->partials);
        launch_finalize(FIN_RR, c->partials, c->scal, s);
        if ((st = read_scal(c, S_RR, &rr))) return st;
        if (rr <= tol2) { conv = true; break; }
        if (it >= max_iter || restarts >= 8) break;
        ++restarts;
        fresh = true;
        continue;
      }
      apply_s(c, r, z);
      launch_dot(N, z, r, flex ? q : nullptr, c->partials, s);
      launch_finalize(flex ? FIN_RZ_NEXT_FLEX : FIN_RZ_NEXT, c->partials, c->scal, s);
      launch_update_p(N, c->scal, p, z, s);
    }
  }
  if (c->layout == 1) launch_copy(N, x, x_io, s);
  else launch_permute(N, c->sfc_index, x, x_io, 0, s);
  HIPCHK(c, hipStreamSynchronize(s));
  prof_collect(c);
  inf.iterations = it;
  inf.restarts = restarts;
  inf.rel_residual = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  if (info) *info = inf;
  if (!conv) FAIL(c, SFCDD_ENOTCONV, "not converged after %d iterations (rel. residual %.3e)", it, inf.rel_residual);
  return SFCDD_OK;
}

sfcdd_status sfcdd_grad_coeff(sfcdd_ctx* c, const double* lam, const double* u, double* grad_a) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  if (!lam || !u || !grad_a) FAIL(c, SFCDD_EINVAL, "NULL argument");
  const hipStream_t s = c->stream;
  const int64_t N = c->g.N;
  const double *L = lam, *U = u;
  if (c->layout == 1) {  // to natural order
    launch_permute(N, c->sfc_index, lam, c->vec[V_IN], 0, s);
    launch_permute(N, c->sfc_index, u, c->vec[V_OUT], 0, s);
    L = c->vec[V_IN];
    U = c->vec[V_OUT];
  }
  launch_grad_coeff(c->g, L, U, c->partials, s);
  launch_finalize_vec(c->d, c->partials, c->gout, s);
  HIPCHK(c, hipMemcpyAsync(c->host_scal + 16, c->gout, 8 * c->d, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int j = 0; j < c->d; ++j) grad_a[j] = -c->g.inv_h2[j] * c->host_scal[16 + j];
  return SFCDD_OK;
}

sfcdd_status sfcdd_get_partition(sfcdd_ctx* c, int32_t* sfc_index_host, int64_t* ta_host,
                                 int64_t* Ni_host, double* omega_host, int32_t* q_out) {
  if (!c) FAIL((sfcdd_ctx*)nullptr, SFCDD_EINVAL, "ctx is NULL");
  if (sfc_index_host) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(sfc_index_host, c->sfc_index, 4 * c->g.N, hipMemcpyDeviceToHost));
  }
  for (int i = 0; i < c->P; ++i) {
    if (ta_host) ta_host[i] = c->ta[i];
    if (Ni_host) Ni_host[i] = c->Ni[i];
    if (omega_host) omega_host[i] = c->omega[i];
  }
  if (q_out) *q_out = c->q;
  return SFCDD_OK;
}

sfcdd_status sfcdd_partition_host(const sfcdd_params* params, int64_t* ta_host, int64_t* Ni_host,
                                  double* omega_host, int32_t* q_out) {
  sfcdd_ctx tmp;
  const sfcdd_status st = plan(&tmp, params);
  if (st != SFCDD_OK) {
    g_last_error = tmp.err;
    return st;
  }
  for (int i = 0; i < tmp.P; ++i) {
    if (ta_host) ta_host[i] = tmp.ta[i];
    if (Ni_host) Ni_host[i] = tmp.Ni[i];
    if (omega_host) omega_host[i] = tmp.omega[i];
  }
  if (q_out) *q_out = tmp.q;
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
  return SFCDD_OK;
}

sfcdd_status sfcdd_destroy(sfcdd_ctx* c) {
  if (!c) return SFCDD_OK;
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
  return SFCDD_OK;
}

const char* sfcdd_last_error(const sfcdd_ctx* c) {
  return c ? c->err.c_str() : g_last_error.c_str();
}

}  // extern "C"
