// Host-callable launchers of the sfcdd device kernels (internal interface).
//
// Every kernel works on a batch of G independent grids (G = 1 for a single
// subproblem): vectors of all grids are concatenated, each grid owning the
// entries [goff, goff + N); subdomains and coarse unknowns are numbered
// globally in grid order.  A kernel finds the grid of an entry through the
// per-entry grid id tables (not read when G == 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfcdd {

constexpr int MAXD = 16;

// Geometry, partition and batch placement of one grid.
struct GridDesc {
  int d;
  int nres;                 // curve resolution bits
  int curve;                // 0 Z-order, 1 Hilbert
  int64_t N;
  int n[MAXD];              // interior points per dimension
  int shift[MAXD];          // coordinate scaling to the finest resolution
  int64_t stride[MAXD];     // natural-order strides (first coordinate fastest)
  double c[MAXD];           // a_j / h_j^2
  double inv_h2[MAXD];      // 1 / h_j^2
  double diag;              // sum_j 2 c_j
  // partition
  int P, q, N0;
  int64_t base, rem;        // piece sizes floor(N/P) (+1 for the first rem)
  int F;                    // floor(gamma)
  int ncand;                // subdomains that may contain a point of a piece
  // placement in the batch
  int64_t goff;             // first vector entry
  int soff;                 // first subdomain
  int64_t c0off;            // first coarse unknown
  int64_t c0pad;            // first entry of the tile-padded coarse vector
  int nt0;                  // coarse tiles per edge
  // dense coarse level: the coarse matrix itself (agg = 1), or, with the
  // iterative coarse solve, its Galerkin aggregation over groups of agg = TS
  // consecutive coarse unknowns (the inner solve's second level)
  int agg;
  int N0d;                  // ceil(N0 / agg) dense unknowns
  int nt0d;                 // dense tiles per edge
};

// Device view of a batch (passed by value).
struct Batch {
  const GridDesc* grids;
  int G;
  int dmax;                 // planes of the neighbour table
  int duni;                 // the dimension of every grid when they all agree, else 0
  int64_t Ntot;             // sum of N
  int Ptot;                 // sum of P
  int64_t N0tot;            // sum of N0
  const uint16_t* gid;      // grid of each vector entry
  const uint16_t* sgid;     // grid of each subdomain
  const uint16_t* cgid;     // grid of each coarse unknown
  const uint16_t* ctgid;    // grid of each coarse tile
  int rbx;                  // reduction blocks per grid
  int spmv_u;               // SpMV launch shape: points per thread (window of 256 u points)
  int64_t maxN;             // points of the largest grid
  const int32_t* cperm;     // position of every coarse block in its grid's coarse numbering
};

__device__ __forceinline__ int grid_of(const Batch& B, const uint16_t* ids, int64_t i) {
  return B.G == 1 ? 0 : (int)ids[i];
}

// Per-matrix offsets of a batch of packed tiled matrices: tile count nt,
// first tile, first element of the padded local vector, first partial.
struct BatchMeta {
  const int32_t* nt;
  const int64_t* off;
  const int64_t* xoff;
  const int64_t* poff;
};

// ---- setup ------------------------------------------------------------
void launch_sfc_rank(const Batch& B, int32_t* pos, int32_t* sfc_index, hipStream_t s);
void launch_build_nbr(const Batch& B, const int32_t* pos, const int32_t* sfc_index, int32_t* nbr,
                      hipStream_t s);
// Local elimination order and tile envelope of every subdomain matrix
// (mode 0: curve order, packed triangle; 1: curve order, envelope; 2:
// diagonal-level order, envelope).  lperm (per local row, at xoff) and
// liperm (per subdomain offset, at doff) map local rows to subdomain offsets
// and back; tlo / trb (per tile row, at xoff / TS) hold the first tile column
// and the packed row base; gtiles[3 g] += tiles stored for grid g's
// subdomains, gtiles[3 g + 1] += factor entries one substitution sweep reads,
// gtiles[3 g + 2] += tile products of their factorisation.  kcap: the
// diagonal key levels a subdomain may span (at most ORDER_MAX_KEYS; wider
// subdomains keep the curve order).
constexpr int ORDER_MAX_KEYS = 16384;
void launch_local_order(const Batch& B, int mode, int kcap, int max_nt, const int32_t* ta, const int32_t* Ni,
                        const int32_t* nt, const int64_t* xoff, const int64_t* doff, const int32_t* sfc_index,
                        const int32_t* nbr, int32_t* lperm, int32_t* liperm, int32_t* tlo, int32_t* trb,
                        unsigned long long* gtiles, hipStream_t s);
// Envelope tiles of the local matrices (cleared and assembled).
template <typename T>
void launch_assemble_local(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                           const int64_t* fac_off, const int64_t* xoff, const int64_t* doff,
                           const int32_t* lperm, const int32_t* liperm, const int32_t* tlo, const int32_t* trb,
                           const int32_t* nbr, int max_nt, T* fac, hipStream_t s);
// Coarse elimination order (see k_coarse_order): ccen scratch of N0tot * dmax
// int32, cperm (N0tot), cfnz (tile-padded coarse rows, initialised to the
// row index).
void launch_coarse_order(const Batch& B, int kcap, int max_n0, const int32_t* sfc_index, int32_t* ccen,
                         int32_t* cperm, int32_t* cfnz, hipStream_t s);
// First nonzero column of every row of the dense coarse matrices (lowers
// cfnz[c0pad + r] over the couplings of every dimension).
void launch_coarse_fnz(const Batch& B, const int32_t* nbr, int32_t* cfnz, hipStream_t s);
// Integer coupling counts of dimension j in the permuted coarse numbering
// (inside the envelope tiles, cleared beforehand).
void launch_coarse_counts(const Batch& B, int j, const int32_t* nbr, const int64_t* ctile_off,
                          int32_t* cnt, hipStream_t s);
// Zero the envelope tiles of the dense coarse matrices and of the counts.
void launch_coarse_zero_env(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, double* A0,
                            int32_t* cnt, hipStream_t s);
// Envelope tables of the dense coarse matrices (per tile row at c0pad / TS):
// first tile column clo (non-decreasing) and packed-triangle row base crb;
// wide[0] (nullable): the envelope width of grid 0's matrix (the most tile
// columns left of the diagonal in a tile row).
void launch_coarse_env(const Batch& B, int max_nt0, const int32_t* cfnz, int32_t* clo, int32_t* crb,
                       int32_t* wide, const int32_t* nd, hipStream_t s);
// One-level dissection of a single grid's coarse matrix (halves of the
// curve, separator last): separator marks (sep cleared beforehand) and the
// dissected order (nd = {ta, tb, ts} tiles, or zeros when it does not pay),
// the previous order kept in backup; its undo; the three chains' row tables.
void launch_nd_order(const Batch& B, const int32_t* nbr, int32_t* sep, int32_t* backup, int32_t* cperm,
                     int32_t* nd, int n0, hipStream_t s);
void launch_nd_undo(const Batch& B, const int32_t* backup, int32_t* cperm, int32_t* cfnz, int32_t* nd,
                    int nrows, hipStream_t s);
void launch_nd_views(const int32_t* nd, const int32_t* clo, int stride, int32_t* vinfo, int32_t* vlo, int32_t* vrb,
                     hipStream_t s);
// A_0 += c_j E_j over the envelope tiles; the counts are cleared as read.
void launch_coarse_accumulate(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, int j,
                              int32_t* cnt, double* A0, hipStream_t s);
void launch_coarse_pad(const Batch& B, int max_nt0, const int64_t* ctile_off, double* A0,
                       hipStream_t s);

// ---- batched tiled Cholesky, inversion ----------------------------------
// The single-matrix kernels (diag, step) take the envelope tables of matrix 0
// (tlo / trb at its first tile row; null: every tile).
template <typename T>
void launch_potrf_diag(int J, int kfrom, int nparts, int maxc, const T* part, int nb,
                       const int32_t* nt, const int64_t* off, T* fac, int32_t* status,
                       hipStream_t s, const int32_t* tlo = nullptr, const int32_t* trb = nullptr,
                       const int32_t* vinfo = nullptr, int vstride = 0);
// Whole factorisation, one workgroup per matrix (pair: two columns per
// step; faster alone, but no room beside it for other workgroups).
// rows: row tiles per step of the panel updates (2 .. potrf_full_max_rows;
// 0 = the default 3 FP32, 2 FP64; 1 = the light kernel for matrices of a
// few tile rows: one row per step, no double-buffered prefetch, 35 KB of LDS
// in FP32; pair is then ignored).
int potrf_full_max_rows(bool fp64, bool pair);
// With tlo / trb (and xoff) the matrices are stored as tile envelopes (see
// launch_local_order); with null tables as packed triangles.
template <typename T>
void launch_potrf_full(int nb, const int32_t* nt, const int64_t* off, const int64_t* xoff, const int32_t* tlo,
                       const int32_t* trb, T* fac, int32_t* status, bool pair, hipStream_t s, int rows = 0);
// Rescales the off-diagonal envelope tiles of factored subdomain matrices to
// U_IJ = L_IJ L_JJ^{-1} (the unit block-lower factor the substitution kernel
// uses).
template <typename T>
void launch_unit_lower(int nb, int max_nt, const int32_t* nt, const int64_t* off, const int64_t* xoff,
                       const int32_t* tlo, const int32_t* trb, T* fac, hipStream_t s);
// Widest envelope (tile columns left of the diagonal, over the tile rows)
// for which the column steps also form the rows of the inverse.
constexpr int XROW_MAXW = 24;
// One matrix: sub-diagonal tiles of column J, the diagonal tile of column
// J + 1, and the split-K partials of column J + 2 (three slots of slot_tiles
// tiles at part, slot C mod 3 for column C).  X (nullable): also row J of
// the inverse X = L^{-1} (packed lower tiles at X + off[0] tiles), whose
// last row launch_xrow forms after the last step, when the device-side
// envelope width *wide is at most XROW_MAXW.  vinfo (nullable): nviews
// chains over the parts of a dissected matrix in the same launches (see
// factor_nd); max_nt is then the most tile rows of a view.
template <typename T>
void launch_potrf_step(int J, int max_nt, int maxc, T* part, int64_t slot_tiles, const int32_t* nt,
                       const int64_t* off, T* fac, int32_t* status, hipStream_t s,
                       const int32_t* tlo = nullptr, const int32_t* trb = nullptr, T* X = nullptr,
                       const int32_t* wide = nullptr, const int32_t* vinfo = nullptr, int vstride = 0,
                       int nviews = 1, T* V = nullptr);
// Row J of X (tile offset xo: local tile (J, C) at (xo + J, xo + C)).
template <typename T>
void launch_xrow(int J, const int64_t* off, const T* fac, T* X, hipStream_t s, const int32_t* tlo,
                 const int32_t* trb, const int32_t* wide, int xo = 0);
// Factor and inverse of a dissected single coarse matrix (launch_nd_order,
// launch_nd_views): the two halves' chains concurrently, then the
// separator.  part: six slots of vstride * maxc tiles; vbuf: ts (ta + tb)
// tiles of V = L_S,half X_half,half.
template <typename T>
void factor_nd(int ta, int tb, int ts, int maxc, T* part, const int64_t* off, T* fac, T* X, int32_t* status,
               const int32_t* nt, const int32_t* clo, const int32_t* vinfo, const int32_t* vlo, const int32_t* vrb,
               int vstride, T* vbuf, hipStream_t s);
template <typename T>
void launch_trtri_col(int J, int nb, int max_nt, const int32_t* nt, const int64_t* off,
                      const T* L, T* X, hipStream_t s);
// xoff / tlo (nullable): envelope of each L (first tile column per tile row
// at xoff[b] / TS); the tile sums skip the zero tiles left of it.  wide
// (nullable): the device-side envelope width of a single matrix; at most
// XROW_MAXW, the column steps formed X and these kernels return at once.
template <typename T>
void launch_trtri_rec(int nb, int max_nt, const int32_t* nt, const int64_t* off, const int64_t* toff,
                      const T* L, T* X, T* Tb, hipStream_t s, const int64_t* xoff = nullptr,
                      const int32_t* tlo = nullptr, const int32_t* wide = nullptr);
template <typename T>
void launch_lauum(int nb, int max_nt, const int32_t* nt, const int64_t* off, const T* X, T* M,
                  hipStream_t s);

// ---- per-iteration operators ---------------------------------------------
// Blocks per grid of the windowed SpMV for grids of up to maxN points.
int spmv_blocks(int64_t maxN, int u);
// mode 0: y = A x;  1: y = A x, per-grid partials of x.y;  2: y = b - A x,
// per-grid partials of y.y;  3: y = b - A x.  Returns the partials written
// per grid (0 for modes 0 and 3), the count launch_finalize then takes.
int launch_spmv(const Batch& B, int mode, const int32_t* nbr, const double* x, double* y,
                 const double* b, double* partials, hipStream_t s);
// active (nullable): per-grid solver flags; subdomains of grids that are not
// updating (flag not RUN or RESTART) are skipped.
// Whether the substitution kernel's LDS (the subdomain's right-hand side and
// the tile-row tables) fits a CU for subdomains of max_nt tile rows at this
// many waves per workgroup.  The launcher lowers the waves until it does.
bool trsv_fits(int max_nt, int elem_bytes, int waves);
// Factors stored as tile envelopes in the local order lperm (see
// launch_local_order), off-diagonal tiles in the unit block-lower form (see
// launch_unit_lower); ztile: a TS x TS tile of zeros.
template <typename T>
void launch_schwarz_trsv(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                         const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                         const int32_t* tlo, const int32_t* trb, int max_nt, int waves, bool stream,
                         const T* fac, const T* ztile, const double* w, double* dbuf, const int32_t* active,
                         hipStream_t s);
template <typename T>
void launch_symv_tiles(int nb, int max_nt, const BatchMeta& bm, const T* M, const T* xloc, T* part,
                       hipStream_t s);
template <typename T>
void launch_symv_reduce(int nb, int max_n, const BatchMeta& bm, const int32_t* n,
                        const int64_t* doff, const T* part, double* out, hipStream_t s);
template <typename T>
void launch_gather_local(const Batch& B, int max_nt, const BatchMeta& bm, const int32_t* ta,
                         const int32_t* Ni, const double* w, T* xloc, hipStream_t s);
// h[p] = sum over the subdomains i containing p of w_i(p) d_i[p - ta_i]:
// w_i = omega_i, or (dweight) 1 / (number of subdomains containing p).
void launch_scatter(const Batch& B, int dweight, const int32_t* ta, const int32_t* Ni,
                    const int64_t* doff, const double* omega, const double* dbuf, double* h,
                    hipStream_t s);
void launch_restrict(const Batch& B, int max_block, const double* v, double* c0, hipStream_t s);
// out = X^T (X v) for packed lower-tiled FP64 X (the coarse operator X = L_0^{-1}):
// v tile-padded at bm.xoff, ytmp the same layout, part the per-(tile, chunk)
// partials at bm.poff, out unpadded at doff (n[b] entries).
template <typename T>
void launch_coarse_apply(int nb, int max_nt, const BatchMeta& bm, const int32_t* n,
                         const int64_t* doff, const T* X, const double* v, double* ytmp,
                         double* part, double* out, const int32_t* active, hipStream_t s,
                         const int32_t* nd = nullptr);
void launch_round_f32(int64_t n, const double* src, float* dst, hipStream_t s);
// Rounds the tiles inside the envelopes of the dense coarse matrices (tile
// row I of grid g: clo[c0pad / TS + I] .. I, packed triangle at off[g]).
void launch_round_env(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, const double* src,
                      float* dst, hipStream_t s);

// ---- iterative coarse solve (single grid) -----------------------------------
void launch_coarse_ell(const Batch& B, int64_t n0, const int32_t* nbr, int kw, int64_t ld, int32_t* deg,
                       int32_t* col, double* val, int32_t* status, hipStream_t s);
void launch_bj_extract(int64_t n0, int64_t ld, const int32_t* deg, const int32_t* col, const double* val,
                       double* tiles, hipStream_t s);
void launch_bj_form(int ntiles, const double* X, float* M, hipStream_t s);
void launch_ic_trial(int64_t n0, int64_t ld, double* b, hipStream_t s);
void launch_ic_begin(const int32_t* outer, int32_t* flag, double* sc, hipStream_t s);
void launch_ic_spmv(int64_t ld, const int32_t* deg, const int32_t* col, const double* val, const double* p,
                    double* q, double* part, const int32_t* flag, hipStream_t s);
void launch_ic_update(int first, int it, int64_t n0, int nt, int nq, const double* qpart, const double* sc,
                      const double* b, double* x, double* r, const double* p, const double* q, const float* M,
                      double* z1, double* cagg, double* part, const int32_t* flag, hipStream_t s);
void launch_ic_dir(int first, int it, int64_t n0, int nt, double tol2, const double* part, const double* cagg,
                   const double* dagg, double* sc, const double* z1, double* p, int32_t* flag, hipStream_t s);
void launch_combine(const Batch& B, int mode, const double* d0, const double* a, const double* b,
                    double* out, hipStream_t s);
// out = a + R_0^T d0 and the partials of out . b (and out . c, c non-null)
// in launch_dot's layout.
void launch_combine_dot(const Batch& B, const double* d0, const double* a, double* out, const double* b,
                        const double* c, double* partials, hipStream_t s);

// ---- BLAS-1 and scalars (per grid) -----------------------------------------
void launch_dot(const Batch& B, const double* a, const double* b, const double* c,
                double* partials, hipStream_t s);
// nparts: partials per grid (0: rbx, the BLAS-1 reductions' count).
void launch_finalize(const Batch& B, int mode, const double* partials, double* scal,
                     int32_t* active, hipStream_t s, int nparts = 0);
void launch_update_xr(const Batch& B, const double* scal, const int32_t* active, double* x,
                      double* r, const double* p, const double* q, double* partials,
                      hipStream_t s);
void launch_update_p(const Batch& B, const double* scal, const int32_t* active, double* p,
                     const double* z, hipStream_t s);
void launch_axpy_scal(const Batch& B, const double* scal, int slot, const int32_t* active,
                      double* x, const double* z, hipStream_t s);
void launch_permute(int64_t n, const int32_t* idx, const double* in, double* out, int gather,
                    hipStream_t s);
void launch_grad_coeff(const GridDesc& g, const double* lam, const double* u, double* partials,
                       hipStream_t s);
void launch_finalize_vec(int nvals, const double* partials, double* out, hipStream_t s);
void launch_copy(int64_t n, const double* a, double* b, hipStream_t s);
void launch_zero(int64_t n, double* a, hipStream_t s);
void launch_read_probe(const void* buf, int64_t bytes, hipStream_t s);
void launch_ct_combine(const Batch& B, int layout, const int32_t* pos, const double* w, const double* u,
                       const double* x, int64_t M, double* out, hipStream_t s);

// Scalar slots of the solver's per-grid device scalars S[g * S_COUNT + slot].
enum {
  S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_RZNEW, S_ZQ, S_BB, S_XI, S_TMP, S_TOL2, S_TRR,
  // inner CG of the iterative coarse solve (single grid): r.z of the last two
  // steps, r.r at the start, steps taken, 1 when converged
  IC_RZ = 16, IC_RR0 = 18, IC_ITS = 19, IC_CONV = 20,
  S_COUNT = 24
};
// Per-grid solver flags (device array `active`).
enum {
  ACT_DONE = 0,      // converged or stopped: no updates
  ACT_RUN = 1,       // iterating
  ACT_RESTART = 2,   // iterating, next direction p = z (becomes RUN at the next step size)
  ACT_CAND = 3,      // recursive residual below tolerance, awaiting the true-residual check
  ACT_SKIP = 4       // excluded from the current pass
};
__host__ __device__ __forceinline__ bool act_updating(int f) { return f == ACT_RUN || f == ACT_RESTART; }
// Finalize modes.  With a flag array, the CG recurrences (PQ_ALPHA, RZ_*) are
// applied to updating grids only.
enum {
  FIN_PQ_ALPHA = 0,   // S_PQ = sum; S_ALPHA = S_RZ / S_PQ; RESTART -> RUN
  FIN_RR,             // S_RR = sum
  FIN_RZ_INIT,        // S_RZ = sum
  FIN_RZ_NEXT,        // rz = sum; S_BETA = rz / S_RZ; S_RZ = rz
  FIN_RZ_NEXT_FLEX,   // rz = sum0, zq = sum1; S_BETA = -S_ALPHA zq / S_RZ; S_RZ = rz
  FIN_BB,             // S_BB = sum
  FIN_RR_CAND,        // S_RR = sum; updating grid with S_RR <= S_TOL2 -> CAND
  FIN_RR_DONE,        // S_RR = sum; updating grid with S_RR <= S_TOL2 -> DONE
  FIN_TRR,            // S_TRR = sum
  FIN_EN,             // S_RR = -sum (sum = x . r with b = 0: x^T A x)
  FIN_EN_CAND,        // S_RR = -sum; updating grid with S_RR <= S_TOL2 -> CAND
  FIN_EN_DONE         // S_RR = -sum; updating grid with S_RR <= S_TOL2 -> DONE
};
// Combine modes of launch_combine.
enum {
  COMB_PROLONG = 0,          // out = R0^T d0
  COMB_ADD_PROLONG,          // out = a + R0^T d0
  COMB_BAL_FINAL             // out = a - R0^T d0 + b      (y - F A y + F g)
};

}  // namespace sfcdd
