// Batched dense Cholesky factorisation of the subdomain matrices and of the
// coarse matrix (factor once, Sec. 3.1), on packed lower 64x64 tiles with
// MFMA tile products, left-looking over tile columns J.  A batch of matrices
// is factored by one persistent workgroup per matrix; a single large matrix
// by two launches per column (the diagonal tile, then its sub-diagonal tiles
// beside the split-K partial update of the next column).  The diagonal tiles
// keep the INVERSE of the diagonal Cholesky block, L_JJ^{-1}, so that both
// the panel update and the substitution sweeps are tile products.
#include <algorithm>
#include <utility>

#include "common.h"
#include "kernels.h"

namespace sfcdd {

// Broadcast of lane `src` (wave-uniform) to every lane through an SGPR.
__device__ __forceinline__ float bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row stride of the LDS buffers of the diagonal-tile factorisation: 16-byte
// aligned rows whose 16-byte chunks fall in distinct bank groups for 8
// consecutive rows (66 doubles, 68 floats).
template <typename T> struct Pstride { static constexpr int v = (sizeof(T) == 8) ? 66 : 68; };

constexpr int DB = 16;         // block edge inside the diagonal tile
constexpr int NDB = TS / DB;   // blocks per tile edge

// 1/sqrt(x) for x > 0: hardware estimate refined by one Newton step.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ float rsqrt_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
}

// Lane K of each row of 16 lanes, to every lane of that row (DPP
// row_newbcast).
template <int K, typename T>
__device__ __forceinline__ T row_bcast(T v) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + K, 0xF, 0xF, false));
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x150 + K, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + K, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}

// Row PK of 16 lanes copied to all four rows (lane 16 p + i receives lane
// 16 PK + i) with the gfx950 permlane swaps: the 16-lane swap pairs rows
// (0, 1) and (2, 3), its first result holding rows (0, 0, 2, 2) and its
// second (1, 1, 3, 3); the 32-lane swap of either gives the lower pair
// (first result) or the upper pair (second) in both halves.
template <int PK>
__device__ __forceinline__ unsigned row_to_all(unsigned v) {
  const auto x = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  const unsigned w = (PK & 1) ? x[1] : x[0];
  const auto z = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return (PK & 2) ? z[1] : z[0];
}
template <int PK>
__device__ __forceinline__ float row_to_all(float v) {
  return __uint_as_float(row_to_all<PK>(__float_as_uint(v)));
}
template <int PK>
__device__ __forceinline__ double row_to_all(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = row_to_all<PK>((unsigned)b), hi = row_to_all<PK>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Pivot K of the DB x DB block held by one wave: lane (p, i) = 16 p + i holds
// w[q] = W[i][p + 4 q] of the working matrix (symmetric, both triangles).
// The factor column is l = W[:, K] / sqrt(W[K][K]): the lane's own l_i sits
// in lane (K mod 4, i) (row_to_all), and l_j for its columns j = p + 4 q is
// row K right of the pivot, in lane K of each 16-lane row (row broadcast).
// The whole block takes W -= l l^T without masks: rows and columns already
// eliminated hold only rounding residues, which the update moves among
// themselves (an active entry W[i][j], i, j >= K, is changed by l_i l_j with
// both from the active part), so no branch or lane mask sits on the
// dependent chain.  The factor column goes to lo[] in the lanes of column K
// (its entries above the diagonal are residues and are dropped when the
// lower triangle is written).  A non-positive pivot is replaced by 1 and
// flagged in bad.
template <typename T, int K>
__device__ __forceinline__ void pivot_step(T (&w)[DB / 4], T (&lo)[DB / 4], T (&rd)[DB], int p, bool& bad) {
  constexpr int pk = K & 3, qk = K >> 2;
  T piv = bcast(w[qk], 16 * pk + K);   // W[K][K] (through an SGPR)
  bad |= !(piv > T(0));
  piv = piv > T(0) ? piv : T(1);
  const T rs = rsqrt_nr(piv);
  rd[K] = rs;
  const T li = row_to_all<pk>(w[qk]) * rs;
  T lj[DB / 4];
#pragma unroll
  for (int q = 0; q < DB / 4; ++q) lj[q] = row_bcast<K>(w[q]) * rs;
#pragma unroll
  for (int q = 0; q < DB / 4; ++q) w[q] = fma(-li, lj[q], w[q]);
  if (p == pk) lo[qk] = li;
}
template <typename T, int... K>
__device__ __forceinline__ void pivots(std::integer_sequence<int, K...>, T (&w)[DB / 4], T (&lo)[DB / 4],
                                       T (&rd)[DB], int p, bool& bad) {
  (pivot_step<T, K>(w, lo, rd, p, bad), ...);
}

// Cholesky factor and inverse of the DB x DB diagonal block at (o, o) of sC,
// by the first wave (pivots as in pivot_step, all 64 lanes).  Writes the
// factor back to the block (upper part zero), its inverse (lower, upper part
// zero) to dinv (row stride ldd).  A non-positive pivot sets *status to -6
// and is replaced by 1.
template <typename T>
__device__ __forceinline__ void factor_block(T* __restrict__ sC, int o, T* __restrict__ dinv, int ldd,
                                             int32_t* status) {
  constexpr int PS = Pstride<T>::v;
  const int lane = threadIdx.x, p = lane >> 4, i = lane & 15;
  T w[DB / 4], lo[DB / 4], rd[DB];
  // the lane's part of the full symmetric row i, from the lower triangle (the
  // stored upper part is not meaningful)
#pragma unroll
  for (int q = 0; q < DB / 4; ++q) {
    const int j = p + 4 * q;
    w[q] = sC[j <= i ? (o + i) * PS + o + j : (o + j) * PS + o + i];
    lo[q] = T(0);
  }
  bool bad = false;
  pivots<T>(std::make_integer_sequence<int, DB>{}, w, lo, rd, p, bad);
  if (bad && lane == 0) atomicExch(status, -6);
#pragma unroll
  for (int q = 0; q < DB / 4; ++q) sC[(o + i) * PS + o + p + 4 * q] = p + 4 * q <= i ? lo[q] : T(0);
  // inverse by forward substitution, lane c < DB owning column c; L_rk read
  // back from the block (same address in every lane), 1/L_rr = rd[r].
  // Column-oriented: once x_k is known it is subtracted from every later
  // row, so the dependent chain is one multiply-add per row (each row's sum
  // still takes its terms in increasing k).
  const bool act = lane < DB;
  T x[DB], sum[DB];
#pragma unroll
  for (int r = 0; r < DB; ++r) sum[r] = (r == lane) ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < DB; ++k) {
    x[k] = sum[k] * rd[k];
#pragma unroll
    for (int r = k + 1; r < DB; ++r) sum[r] -= sC[(o + r) * PS + o + k] * x[k];
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < DB; ++r) dinv[r * ldd + lane] = x[r];
  }
}

// 16x16 blocks on MFMA, one wave: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] per k-step of 4.  Operand fragments of a row-major block X:
// fragment st of lane l is X[l%16][4 st + l/16] (the A operand of X, and the
// B operand of X^T).
template <typename T>
__device__ __forceinline__ void frag_load(T (&f)[DB / 4], const T* X, int ld) {
  const int m = threadIdx.x & 15, kk = (threadIdx.x >> 4) & 3;
#pragma unroll
  for (int st = 0; st < DB / 4; ++st) f[st] = X[m * ld + 4 * st + kk];
}
// B operand of a row-major block Z (B = Z): Z[4 st + l/16][l%16].
template <typename T>
__device__ __forceinline__ void frag_load_b(T (&f)[DB / 4], const T* Z, int ld) {
  const int m = threadIdx.x & 15, kk = (threadIdx.x >> 4) & 3;
#pragma unroll
  for (int st = 0; st < DB / 4; ++st) f[st] = Z[(4 * st + kk) * ld + m];
}
template <typename T>
__device__ __forceinline__ void frag_mma(typename Acc<T>::type& c, const T (&a)[DB / 4],
                                         const T (&b)[DB / 4]) {
#pragma unroll
  for (int st = 0; st < DB / 4; ++st) c = mfma16(a[st], b[st], c);
}
template <typename T>
__device__ __forceinline__ void blk_store(const typename Acc<T>::type& c, T* D, int ld, T sign) {
  const int g = (threadIdx.x >> 4) & 3, n = threadIdx.x & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) D[Acc<T>::row(g, r) * ld + n] = sign * c[r];
}
template <typename T>
__device__ __forceinline__ void blk_load(typename Acc<T>::type& c, const T* D, int ld) {
  const int g = (threadIdx.x >> 4) & 3, n = threadIdx.x & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = D[Acc<T>::row(g, r) * ld + n];
}
template <typename T>
__device__ __forceinline__ typename Acc<T>::type blk_zero() {
  typename Acc<T>::type c;
  c[0] = c[1] = c[2] = c[3] = T(0);
  return c;
}

// One column block bk of the blocked factorisation: the diagonal block by the
// first wave (its pivots are one dependent chain), then the panel
// L_rb,bk = C_rb,bk L_bk,bk^{-T} and the trailing update
// C_rb,cb -= L_rb,bk L_cb,bk^T with their 16x16 block products dealt over
// the four waves.
template <typename T, int bk>
__device__ __forceinline__ void factor_column(T* __restrict__ sC, T* __restrict__ sX, int32_t* status) {
  constexpr int PS = Pstride<T>::v;
  constexpr int o = bk * DB;
  constexpr int nr = NDB - 1 - bk;  // blocks below the diagonal
  typedef typename Acc<T>::type AT;
  const int wv = threadIdx.x >> 6;
  T* dinv = sX + o * PS + o;        // L_bk,bk^{-1} is block (bk, bk) of X
  if (wv == 0) factor_block(sC, o, dinv, PS, status);
  lds_barrier();
  if constexpr (nr > 0) {
    if (wv < nr) {                  // panel block row bk + 1 + wv
      T fd[DB / 4], fc[DB / 4];
      frag_load<T>(fd, dinv, PS);                                   // B = Dinv^T
      T* C = sC + (o + DB + wv * DB) * PS + o;
      frag_load<T>(fc, C, PS);
      AT pc = blk_zero<T>();
      frag_mma<T>(pc, fc, fd);
      blk_store<T>(pc, C, PS, T(1));
    }
    lds_barrier();
    // trailing blocks (bk + 1 + q, bk + 1 + u), u <= q, numbered q (q + 1) / 2 + u
    for (int t = wv; t < nr * (nr + 1) / 2; t += 4) {
      const int q = t >= 3 ? 2 : (t >= 1 ? 1 : 0);
      const int u = t - q * (q + 1) / 2;
      T fq[DB / 4], fu[DB / 4];
      frag_load<T>(fq, sC + (o + DB + q * DB) * PS + o, PS);
      frag_load<T>(fu, sC + (o + DB + u * DB) * PS + o, PS);
      T* D = sC + (o + DB + q * DB) * PS + o + DB + u * DB;
      AT cc;
      blk_load<T>(cc, D, PS);
      AT up = blk_zero<T>();
      frag_mma<T>(up, fq, fu);
      cc -= up;
      blk_store<T>(cc, D, PS, T(1));
    }
    lds_barrier();
  }
}

// Block row I of X = L^{-1}: X_IJ = -L_II^{-1} sum_{K=J}^{I-1} L_IK X_KJ,
// J < I (rows above already complete), one block J per wave.
template <typename T, int I>
__device__ __forceinline__ void inverse_row(const T* __restrict__ sC, T* __restrict__ sX) {
  constexpr int PS = Pstride<T>::v;
  typedef typename Acc<T>::type AT;
  const int J = threadIdx.x >> 6;
  if (J < I) {
    AT t = blk_zero<T>();
    for (int K = J; K < I; ++K) {
      T fa[DB / 4], fb[DB / 4];
      frag_load<T>(fa, sC + (I * DB) * PS + K * DB, PS);         // A = L_IK
      frag_load_b<T>(fb, sX + (K * DB) * PS + J * DB, PS);       // B = X_KJ
      frag_mma<T>(t, fa, fb);
    }
    T fdi[DB / 4];
    frag_load<T>(fdi, sX + (I * DB) * PS + I * DB, PS);          // A = L_II^{-1}
    T* tmp = sX + (J + 1) * DB;                                  // free upper block (0, J + 1)
    blk_store<T>(t, tmp, PS, T(1));
    T fb[DB / 4];
    frag_load_b<T>(fb, tmp, PS);
    AT xij = blk_zero<T>();
    frag_mma<T>(xij, fdi, fb);
    blk_store<T>(xij, sX + (I * DB) * PS + J * DB, PS, T(-1));
  }
  lds_barrier();
}

// Cholesky factorisation and inversion of a TS x TS LDS tile (stride
// Pstride, lower part read), blocked by DB, by the four waves of the
// workgroup (the pivots of each diagonal block by the first).
// On exit sX holds L^{-1} (lower; stride Pstride); sC holds L (lower).  The
// inverted diagonal blocks are formed in place in sX, and the free blocks
// above its diagonal serve as scratch.
template <typename T>
__device__ __forceinline__ void potrf_inv_tile(T* __restrict__ sC, T* __restrict__ sX, int32_t* status) {
  lds_barrier();
  factor_column<T, 0>(sC, sX, status);
  factor_column<T, 1>(sC, sX, status);
  factor_column<T, 2>(sC, sX, status);
  factor_column<T, 3>(sC, sX, status);
  inverse_row<T, 1>(sC, sX);
  inverse_row<T, 2>(sC, sX);
  inverse_row<T, 3>(sC, sX);
}

// LDS of the diagonal-tile factorisation: two Pstride tiles (C, X).  The
// GEMM staging (LdsV tiles, the same size) fits in the same space.
template <typename T>
constexpr size_t diag_lds_bytes() {
  return 2 * (size_t)TS * Pstride<T>::v * sizeof(T);
}

// Tile addressing of a factor: the packed lower triangle (Tri), or the tile
// envelope of a subdomain factor (Env: tile row I holds the tiles J = lo[I]
// .. I at rb[I] + J, lo non-decreasing; every tile left of lo[I] is zero in
// the matrix and in its Cholesky factor).
struct Tri {
  __device__ __forceinline__ int64_t operator()(int I, int J) const { return tri_index(I, J); }
  __device__ __forceinline__ int first(int) const { return 0; }
  __device__ __forceinline__ int last(int, int ntb) const { return ntb - 1; }
};
// Null tables: the packed triangle.
struct Env {
  const int32_t* lo;
  const int32_t* rb;
  __device__ __forceinline__ int64_t operator()(int I, int J) const {
    return rb ? (int64_t)rb[I] + J : tri_index(I, J);
  }
  __device__ __forceinline__ int first(int I) const { return lo ? lo[I] : 0; }
  // last tile row with a tile in column J
  __device__ __forceinline__ int last(int J, int ntb) const {
    if (!lo) return ntb - 1;
    int h = J;
    while (h + 1 < ntb && lo[h + 1] <= J) ++h;
    return h;
  }
};

// Left-looking: the tile first receives -sum_{K<J} L_JK L_JK^T.  The terms
// K = kfrom .. J-1 are formed in this workgroup; the terms K < kfrom (single
// matrix, split-K) were precomputed as nparts partial tiles part[I][c].
// acc += sign * sum_{K = k0}^{k1 - 1} A_K B_K^T for row-major global tiles
// A_K = pa(K), B_K = pb(K) (B = A when SYRK), two LDS buffers of two tiles
// each at lds.  The loads run NPF steps ahead in registers, so a tile has NPF
// tile products' time to arrive from memory.  Every step issues its loads
// unconditionally (past the end they repeat the last tile) and the loop runs
// in whole groups of NPF steps, so the code between a load and its use is
// the same on every path and the wait before each LDS store covers only the
// loads of that stage.  One barrier per step: the store into a buffer at
// step K follows the barrier of step K - 1, which every wave passes only
// after its products of step K - 2 on that buffer.
constexpr int FACTOR_PF = 3;
template <int NPF, bool SYRK, typename T, typename FA, typename FB>
__device__ __forceinline__ void gemm_loop_pf(TileAcc<T>& acc, int k0, int k1, FA pa, FB pb, T* lds, T sign) {
  constexpr int S = LdsV<T>::v;
  if (k0 >= k1) return;
  TileRegs<T> ra[NPF], rb[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    const int Kl = min(k0 + t, k1 - 1);
    ra[t].load(pa(Kl));
    if (!SYRK) rb[t].load(pb(Kl));
  }
  for (int K = k0; K < k1; K += NPF) {
#pragma unroll
    for (int t = 0; t < NPF; ++t) {
      const int Kc = K + t;
      T* buf = lds + ((Kc - k0) & 1) * 2 * TS * S;
      ra[t].store_lds(buf);
      if (!SYRK) rb[t].store_lds(buf + TS * S);
      const int Kl = min(Kc + NPF, k1 - 1);
      ra[t].load(pa(Kl));
      if (!SYRK) rb[t].load(pb(Kl));
      lds_barrier();
      if (Kc < k1) tile_mma<T>(acc, buf, SYRK ? buf : buf + TS * S, sign);
    }
  }
  lds_barrier();
}

template <typename T, bool DBUF = false, typename IX = Tri>
__device__ __forceinline__ void diag_tile(int J, int kfrom, int nparts, int maxc, const T* __restrict__ part,
                                          T* __restrict__ F, int32_t* __restrict__ status,
                                          unsigned char* smem_raw, IX ix = IX()) {
  T* sA = reinterpret_cast<T*>(smem_raw);
  kfrom = max(kfrom, ix.first(J));
  TileAcc<T> acc;
  acc.load(F + ix(J, J) * TS2);
  {
    const int c0 = min(nparts, ix.first(J) / SPLITK);   // chunks left of the envelope were not formed
    sub_tiles(acc, part + ((int64_t)J * maxc + c0) * TS2, TS2, nparts - c0);
  }
  if (DBUF) {
    auto pj = [&](int K) { return F + ix(J, K) * TS2; };
    gemm_loop_pf<FACTOR_PF, true, T>(acc, kfrom, J, pj, pj, sA, T(-1));
  } else {
    TileRegs<T> ra;
    if (kfrom < J) ra.load(F + ix(J, kfrom) * TS2);
    for (int K = kfrom; K < J; ++K) {
      lds_barrier();
      ra.store_lds(sA);
      lds_barrier();
      if (K + 1 < J) ra.load(F + ix(J, K + 1) * TS2);
      tile_mma<T>(acc, sA, sA, T(-1));  // A_JJ -= L_JK L_JK^T
    }
  }
  lds_barrier();
  constexpr int PS = Pstride<T>::v;
  T* sC = reinterpret_cast<T*>(smem_raw);
  T* sX = sC + TS * PS;

  for (int a = 0; a < 2; ++a)
    for (int b2 = 0; b2 < 2; ++b2)
      for (int r = 0; r < 4; ++r) sC[TileAcc<T>::row(a, r) * PS + TileAcc<T>::col(b2)] = acc.c[a][b2][r];
  potrf_inv_tile(sC, sX, status);
  T* D = F + ix(J, J) * TS2;
  for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) {
    const int i = e / TS, j = e % TS;
    D[e] = j <= i ? sX[i * PS + j] : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_diag(int J, int kfrom, int nparts, int maxc,
                                                             const T* __restrict__ part,
                                                             const int32_t* __restrict__ nt,
                                                             const int64_t* __restrict__ off,
                                                             T* __restrict__ fac,
                                                             int32_t* __restrict__ status,
                                                             const int32_t* __restrict__ tlo,
                                                             const int32_t* __restrict__ trb,
                                                             const int32_t* __restrict__ vinfo, int vstride) {
  __builtin_amdgcn_s_setprio(3);  // head of the same chain as k_potrf_step
  const int b = vinfo ? 0 : blockIdx.x;
  if (vinfo) {  // views of a dissected matrix (see k_potrf_step), view blockIdx.x
    const int v = blockIdx.x;
    if (J >= vinfo[3 * v + 1]) return;
    tlo += v * vstride;
    trb += v * vstride;
  } else if (J >= nt[b]) {
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  diag_tile<T, false, Env>(J, kfrom, nparts, maxc, part, fac + off[b] * TS2, status, smem_raw, Env{tlo, trb});
}

// Sub-diagonal tile (I, J): A_IJ - sum_{K<J} L_IK L_JK^T (terms K >= kfrom
// here, the others from nparts partial tiles), times L_JJ^{-T}.  Row I takes
// the terms K >= max(lo[I], lo[J]) only (and the partial chunks from lo[I] /
// SPLITK); lo[J] <= lo[I] unless the envelope is non-decreasing only within
// parts (a dissected coarse matrix, whose separator rows reach further left
// than the rows above them).
template <typename T, bool DBUF = false, typename IX = Tri>
__device__ __forceinline__ void panel_tile(int J, int I, int kfrom, int nparts, int maxc, const T* __restrict__ part,
                           T* __restrict__ F, T* sA, T* sB, IX ix = IX()) {
  kfrom = max(kfrom, max(ix.first(I), ix.first(J)));
  TileAcc<T> acc;
  acc.load(F + ix(I, J) * TS2);
  {
    const int c0 = min(nparts, ix.first(I) / SPLITK);
    sub_tiles(acc, part + ((int64_t)I * maxc + c0) * TS2, TS2, nparts - c0);
  }
  if (DBUF) {   // sA: four LDS tiles
    gemm_loop_pf<FACTOR_PF, false, T>(acc, kfrom, J, [&](int K) { return F + ix(I, K) * TS2; },
                                      [&](int K) { return F + ix(J, K) * TS2; }, sA, T(-1));
  } else {
    TileRegs<T> ra, rb;
    if (kfrom < J) {
      ra.load(F + ix(I, kfrom) * TS2);
      rb.load(F + ix(J, kfrom) * TS2);
    }
    for (int K = kfrom; K < J; ++K) {
      lds_barrier();
      ra.store_lds(sA);
      rb.store_lds(sB);
      lds_barrier();
      if (K + 1 < J) {
        ra.load(F + ix(I, K + 1) * TS2);
        rb.load(F + ix(J, K + 1) * TS2);
      }
      tile_mma<T>(acc, sA, sB, T(-1));  // A_IJ -= L_IK L_JK^T
    }
  }
  lds_barrier();
  acc.store_lds(sA);
  stage_tile(sB, F + ix(J, J) * TS2);      // L_JJ^{-1}
  lds_barrier();
  TileAcc<T> out;
  out.zero();
  tile_mma<T>(out, sA, sB, T(1));     // L_IJ = A_IJ L_JJ^{-T}
  out.store(F + ix(I, J) * TS2);
}

// Partial update of column Jn: part[I][c] = sum_{K = k0}^{k1 - 1} L_IK L_JnK^T
// (zero when the range is empty).
template <typename T, typename IX = Tri>
__device__ __forceinline__ void partial_tile(int Jn, int I, int c, int k0, int k1, int maxc, const T* __restrict__ F,
                             T* __restrict__ part, T* sA, T* sB, IX ix = IX()) {
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  if (k0 < k1) {
    ra.load(F + ix(I, k0) * TS2);
    rb.load(F + ix(Jn, k0) * TS2);
  }
  for (int K = k0; K < k1; ++K) {
    lds_barrier();
    ra.store_lds(sA);
    rb.store_lds(sB);
    lds_barrier();
    if (K + 1 < k1) {
      ra.load(F + ix(I, K + 1) * TS2);
      rb.load(F + ix(Jn, K + 1) * TS2);
    }
    tile_mma<T>(acc, sA, sB, T(1));
  }
  acc.store(part + ((int64_t)I * maxc + c) * TS2);
}

// Rows per step of the batched panel update: every step loads the L_JK tile
// once for R row tiles L_IK, so the tile products of one step cover the load
// latency of the next and the L_JK tile is read once per R rows.  R = 3 for
// FP32 (about 300 registers per lane) is the default shape; R = 4 is faster
// alone but leaves less room on a SIMD for the concurrent coarse setup.
template <typename T> struct PanelRows { static constexpr int v = sizeof(T) == 4 ? 3 : 2; };

// acc[r] += sign * A_r B^T for r < nr (LDS tiles A_r at sA + r TS S, B at
// sBt, k-contiguous): tile_mma with the B fragments loaded once per k group.
template <typename T, int R>
__device__ __forceinline__ void tile_mma_rows(TileAcc<T> (&acc)[R], int nr, const T* __restrict__ sA,
                                              const T* __restrict__ sBt, T sign) {
  constexpr int S = LdsV<T>::v;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = 32 * (w >> 1), j0 = 32 * (w & 1);
  const int li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < TS / 16; ++t) {
    const int kb = 16 * t + 4 * lk;
    T b[2][4];
#pragma unroll
    for (int n = 0; n < 2; ++n) load4(b[n], sBt + (j0 + 16 * n + li) * S + kb);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r < nr) {
        T a[2][4];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          load4(a[m], sA + r * TS * S + (i0 + 16 * m + li) * S + kb);
#pragma unroll
          for (int u = 0; u < 4; ++u) a[m][u] *= sign;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[r].c[m][n] = mfma16(a[m][u], b[n][u], acc[r].c[m][n]);
      }
    }
  }
}

// Rows r < R (of nr) whose first tile column lo[I0 + r] is at most K: a
// prefix, since lo does not decrease.
template <int R>
__device__ __forceinline__ int rows_upto(const int (&lor)[R], int nr, int K) {
  int n = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) n += (r < nr && lor[r] <= K) ? 1 : 0;
  return n;
}

// Sub-diagonal tiles (I0 + r, J), r < nr <= R, of one matrix: A_IJ minus
// sum_{kfrom<=K<J} L_IK L_JK^T, times L_JJ^{-T}.  Row I takes the terms
// K >= lo[I] only (its tiles left of that are zero).  LDS: R + 1 tiles at lds.
template <typename T, int R, typename IX>
__device__ __forceinline__ void panel_rows(int J, int kfrom, int I0, int nr, T* __restrict__ F, T* lds, IX ix) {
  constexpr int S = LdsV<T>::v;
  T* sB = lds + R * TS * S;
  int lor[R];
#pragma unroll
  for (int r = 0; r < R; ++r) lor[r] = r < nr ? ix.first(I0 + r) : J;
  TileAcc<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) acc[r].load(F + ix(I0 + r, J) * TS2);
  const int k0 = max(kfrom, lor[0]);
  TileRegs<T> ra[R], rb;
  if (k0 < J) {
    const int n1 = rows_upto<R>(lor, nr, k0);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < n1) ra[r].load(F + ix(I0 + r, k0) * TS2);
    rb.load(F + ix(J, k0) * TS2);
  }
  for (int K = k0; K < J; ++K) {
    const int nk = rows_upto<R>(lor, nr, K);
    lds_barrier();  // the products of step K - 1 have read the tiles
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nk) ra[r].store_lds(lds + r * TS * S);
    rb.store_lds(sB);
    lds_barrier();
    if (K + 1 < J) {
      const int n1 = rows_upto<R>(lor, nr, K + 1);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < n1) ra[r].load(F + ix(I0 + r, K + 1) * TS2);
      rb.load(F + ix(J, K + 1) * TS2);
    }
    tile_mma_rows<T, R>(acc, nk, lds, sB, T(-1));  // A_IJ -= L_IK L_JK^T
  }
  lds_barrier();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) acc[r].store_lds(lds + r * TS * S);
  stage_tile(sB, F + ix(J, J) * TS2);  // L_JJ^{-1}
  lds_barrier();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < nr) {
      TileAcc<T> out;
      out.zero();
      tile_mma<T>(out, lds + r * TS * S, sB, T(1));  // L_IJ = A_IJ L_JJ^{-T}
      out.store(F + ix(I0 + r, J) * TS2);
    }
  }
  __syncthreads();
}

// acc0[r] += sign A_r B0^T and, where r >= r1, acc1[r] += sign A_r B1^T
// (LDS tiles A_r at sA + r TS S; B0, B1 k-contiguous): the A fragments are
// loaded once for both columns.
template <typename T, int R>
__device__ __forceinline__ void tile_mma_pair(TileAcc<T> (&acc0)[R], TileAcc<T> (&acc1)[R], int nr, int r1,
                                              const T* __restrict__ sA, const T* __restrict__ sB0,
                                              const T* __restrict__ sB1, T sign) {
  constexpr int S = LdsV<T>::v;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = 32 * (w >> 1), j0 = 32 * (w & 1);
  const int li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < TS / 16; ++t) {
    const int kb = 16 * t + 4 * lk;
    T b0[2][4], b1[2][4];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      load4(b0[n], sB0 + (j0 + 16 * n + li) * S + kb);
      load4(b1[n], sB1 + (j0 + 16 * n + li) * S + kb);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r < nr) {
        T a[2][4];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          load4(a[m], sA + r * TS * S + (i0 + 16 * m + li) * S + kb);
#pragma unroll
          for (int u = 0; u < 4; ++u) a[m][u] *= sign;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc0[r].c[m][n] = mfma16(a[m][u], b0[n][u], acc0[r].c[m][n]);
        if (r >= r1) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
              for (int n = 0; n < 2; ++n) acc1[r].c[m][n] = mfma16(a[m][u], b1[n][u], acc1[r].c[m][n]);
        }
      }
    }
  }
}

// Columns J and J + 1 of rows I0 + r, r < nr <= R (I0 >= J), updated by
// the columns K < J: A_IJ -= sum L_IK L_JK^T and, for I > J, A_I,J+1 -=
// sum L_IK L_J+1,K^T, with each row tile L_IK loaded once for both columns;
// the updated tiles are written back in place.  Row I takes the terms
// K >= lo[I]; a row with lo[I] > J has no tile in column J.  LDS: R + 2
// tiles at lds.
template <typename T, int R, typename IX>
__device__ __forceinline__ void pair_rows(int J, int I0, int nr, T* __restrict__ F, T* lds, IX ix) {
  constexpr int S = LdsV<T>::v;
  T* sB0 = lds + R * TS * S;
  T* sB1 = sB0 + TS * S;
  int lor[R];
#pragma unroll
  for (int r = 0; r < R; ++r) lor[r] = r < nr ? ix.first(I0 + r) : J;
  const int k0 = lor[0];
  if (k0 >= J) return;  // no row of the group has a term K < J
  const int r1 = I0 > J ? 0 : 1;  // row J has no tile in column J + 1
  const int lo1 = ix.first(J + 1);
  TileAcc<T> acc0[R], acc1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < nr) {
      if (lor[r] <= J) acc0[r].load(F + ix(I0 + r, J) * TS2);
      if (r >= r1) acc1[r].load(F + ix(I0 + r, J + 1) * TS2);
    }
  }
  TileRegs<T> ra[R], rb0, rb1;
  {
    const int n1 = rows_upto<R>(lor, nr, k0);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < n1) ra[r].load(F + ix(I0 + r, k0) * TS2);
    rb0.load(F + ix(J, k0) * TS2);
    if (k0 >= lo1) rb1.load(F + ix(J + 1, k0) * TS2);
  }
  for (int K = k0; K < J; ++K) {
    const int nk = rows_upto<R>(lor, nr, K);
    lds_barrier();  // the products of step K - 1 have read the tiles
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nk) ra[r].store_lds(lds + r * TS * S);
    rb0.store_lds(sB0);
    if (K >= lo1) rb1.store_lds(sB1);
    lds_barrier();
    if (K + 1 < J) {
      const int n1 = rows_upto<R>(lor, nr, K + 1);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < n1) ra[r].load(F + ix(I0 + r, K + 1) * TS2);
      rb0.load(F + ix(J, K + 1) * TS2);
      if (K + 1 >= lo1) rb1.load(F + ix(J + 1, K + 1) * TS2);
    }
    // an active row r >= r1 has lo <= K, and lo[J + 1] <= lo of that row, so
    // the tile L_J+1,K it takes is one that was loaded
    tile_mma_pair<T, R>(acc0, acc1, nk, r1, lds, sB0, sB1, T(-1));
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < nr) {
      if (lor[r] <= J) acc0[r].store(F + ix(I0 + r, J) * TS2);
      if (r >= r1) acc1[r].store(F + ix(I0 + r, J + 1) * TS2);
    }
  }
  __syncthreads();
}

// Whole left-looking factorisation of one matrix per workgroup (batches of
// many small matrices): the diagonal tile and then the sub-diagonal tiles of
// each column, all in this workgroup.  Tiles written here are read back in
// later columns only by this workgroup, whose waves share one CU and its
// vector L1: the workgroup-scope release/acquire of the barrier makes the
// stores visible.
// PAIR: columns J and J + 1 together (the update by the columns K < J loads
// each row tile once for both; the two columns are then finished in turn,
// column J + 1 still taking the term K = J).  About 8% faster alone, at
// about 380 registers per lane (FP32); the caller weighs that against the
// room the concurrent coarse setup needs on the SIMDs.
// R: row tiles per step of the panel and pair updates (the autotuner picks
// it per launch shape; PanelRows by default).
template <typename T, bool PAIR, int R, bool DBUF = true>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_full(const int32_t* __restrict__ nt,
                                                             const int64_t* __restrict__ off,
                                                             const int64_t* __restrict__ xoff,
                                                             const int32_t* __restrict__ tlo,
                                                             const int32_t* __restrict__ trb,
                                                             T* __restrict__ fac,
                                                             int32_t* __restrict__ status) {
  const int b = blockIdx.x;
  const int ntb = nt[b];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* F = fac + off[b] * TS2;
  const int64_t trow = tlo ? xoff[b] / TS : 0;
  const Env ix{tlo ? tlo + trow : nullptr, tlo ? trb + trow : nullptr};
  int J = 0;
  if (!PAIR) {
    for (; J < ntb; ++J) {
      diag_tile<T, DBUF>(J, 0, 0, 0, (const T*)nullptr, F, status, smem_raw, ix);
      __syncthreads();
      const int h = ix.last(J, ntb);
      for (int I = J + 1; I <= h; I += R) panel_rows<T, R>(J, 0, I, min(R, h + 1 - I), F, sA, ix);
      __syncthreads();
    }
    return;
  }
  for (; J + 1 < ntb; J += 2) {
    const int h0 = ix.last(J, ntb), h1 = ix.last(J + 1, ntb);
    if (J > 0)
      for (int I = J; I <= h1; I += R) pair_rows<T, R>(J, I, min(R, h1 + 1 - I), F, sA, ix);
    diag_tile<T, DBUF>(J, J, 0, 0, (const T*)nullptr, F, status, smem_raw, ix);
    __syncthreads();
    for (int I = J + 1; I <= h0; I += R) panel_rows<T, R>(J, J, I, min(R, h0 + 1 - I), F, sA, ix);
    diag_tile<T, DBUF>(J + 1, J, 0, 0, (const T*)nullptr, F, status, smem_raw, ix);
    __syncthreads();
    for (int I = J + 2; I <= h1; I += R) panel_rows<T, R>(J + 1, J, I, min(R, h1 + 1 - I), F, sA, ix);
  }
  if (J < ntb) {  // odd tile count: the last column alone
    diag_tile<T, DBUF>(J, 0, 0, 0, (const T*)nullptr, F, status, smem_raw, ix);
    __syncthreads();
  }
}

// One matrix (batch of one), step J after the diagonal tile of column J,
// with the split-K partial sums two columns ahead.  Slot C mod 3 of `part`
// holds the partials of column C: part[I][c] = sum of L_IK L_CK^T over the
// chunk K in [c SPLITK, (c + 1) SPLITK) of K <= C - 3, formed in step C - 2.
// Workgroups of step J:
//  - 0: the tile (J + 1, J) (its partials, the direct terms K = J - 2, J - 1,
//    times L_JJ^{-T}), then in the same workgroup the diagonal tile of
//    column J + 1 (its partials, K = J - 1 and the tile just formed);
//  - 1 .. m - 1: the tiles (I, J), I = J + 2 .. ntb - 1, the same way;
//  - the rest: the partials of column J + 2 over K <= J - 1, rows J + 2 ..
//    ntb - 1, one chunk each.
// So the chain from one diagonal tile to the next holds no chunk sums and no
// cross-workgroup handshake: five tile products and a diagonal
// factorisation.
// Head of the column step J of a single matrix (FP32): the tile (I, J), I =
// J + 1, and the diagonal tile I, fused so that every input comes from
// memory in one round.  Both tiles' operands other than L_IJ itself are
// final when the step starts: A_IJ and A_II, their split-K partials over K
// <= J - 3 and K <= J - 2 (slots of columns J and I), the direct terms'
// tiles L_I,J-2, L_J,J-2, L_I,J-1, L_J,J-1 and L_JJ^{-1}.  Then
//   L_IJ = (A_IJ - sum_K L_IK L_JK^T) L_JJ^{-T}
//   A_II - sum_{K < J} L_IK L_IK^T - L_IJ L_IJ^T -> factor and inverse,
// with L_IJ handed to the diagonal update through LDS.  Rows take the
// terms K >= lo[I] only (a row whose envelope starts right of J has no tile
// (I, J)), the panel's terms K >= lo[J] too.
template <typename IX>
__device__ __forceinline__ void chain_head(int J, int maxc, const float* __restrict__ partJ,
                                           const float* __restrict__ partI, float* __restrict__ F,
                                           int32_t* __restrict__ status, unsigned char* smem_raw, IX ix) {
  typedef float T;
  constexpr int S = LdsV<T>::v;
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * S;
  const int I = J + 1;
  const int lo = ix.first(I);
  const bool hasp = lo <= J;
  const int kp0 = max(J - 2, max(lo, ix.first(J)));  // direct terms of the panel tile: K = kp0 .. J - 1
  const int kd0 = max(J - 1, lo);      // direct terms of the diagonal tile from memory: K = kd0 .. J - 1
  TileRegs<T> rI[2], rJ[2], rD;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int K = J - 2 + t;
    if (K >= 0 && K >= lo) {
      rI[t].load(F + ix(I, K) * TS2);
      if (K >= kp0) rJ[t].load(F + ix(J, K) * TS2);
    }
  }
  if (hasp) rD.load(F + ix(J, J) * TS2);
  TileAcc<T> ap, ad;
  if (hasp) ap.load(F + ix(I, J) * TS2);
  ad.load(F + ix(I, I) * TS2);
  if (hasp) {
    const int nc = J >= 3 ? (J - 2 + SPLITK - 1) / SPLITK : 0;
    const int c0 = min(nc, lo / SPLITK);
    sub_tiles(ap, partJ + ((int64_t)I * maxc + c0) * TS2, TS2, nc - c0);
  }
  {
    const int nc = J >= 2 ? (J - 1 + SPLITK - 1) / SPLITK : 0;
    const int c0 = min(nc, lo / SPLITK);
    sub_tiles(ad, partI + ((int64_t)I * maxc + c0) * TS2, TS2, nc - c0);
  }
  if (hasp) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int K = J - 2 + t;
      if (K < kp0) continue;
      lds_barrier();
      rI[t].store_lds(sA);
      rJ[t].store_lds(sB);
      lds_barrier();
      tile_mma<T>(ap, sA, sB, T(-1));    // A_IJ -= L_IK L_JK^T
      if (K >= kd0) tile_mma<T>(ad, sA, sA, T(-1));  // A_II -= L_IK L_IK^T (K = J - 1)
    }
    lds_barrier();
    ap.store_lds(sA);
    rD.store_lds(sB);                     // L_JJ^{-1}
    lds_barrier();
    TileAcc<T> out;
    out.zero();
    tile_mma<T>(out, sA, sB, T(1));       // L_IJ = A_IJ L_JJ^{-T}
    out.store(F + ix(I, J) * TS2);
    lds_barrier();
    out.store_lds(sA);
    lds_barrier();
    tile_mma<T>(ad, sA, sA, T(-1));       // A_II -= L_IJ L_IJ^T
  }
  lds_barrier();
  constexpr int PS = Pstride<T>::v;
  T* sC = reinterpret_cast<T*>(smem_raw);
  T* sX = sC + TS * PS;
  for (int a = 0; a < 2; ++a)
    for (int b2 = 0; b2 < 2; ++b2)
      for (int r = 0; r < 4; ++r) sC[TileAcc<T>::row(a, r) * PS + TileAcc<T>::col(b2)] = ad.c[a][b2][r];
  potrf_inv_tile(sC, sX, status);
  T* D = F + ix(I, I) * TS2;
  for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) {
    const int i = e / TS, j = e % TS;
    D[e] = j <= i ? sX[i * PS + j] : T(0);
  }
}

// Tile (J, C), C <= J, of X = L^{-1} for a single matrix, formed row by row
// as the factorisation proceeds (L X = I):
//   X_JJ = L_JJ^{-1},  X_JC = -L_JJ^{-1} sum_{max(C, lo[J]) <= K < J} L_JK X_KC.
// Row J of L is complete once column J - 1 is factored, and the rows of X
// above it were formed earlier, so row J of X is formed by extra workgroups
// of the column step J (the chain itself does not wait for them), and the
// inversion no longer follows the factorisation on the setup's critical
// path.  X is a packed lower-triangular tile matrix at X (a chain over one
// part of a dissected matrix writes its local tile (J, C) at (xo + J, xo +
// C)).  A row takes up to
// (row width of the envelope) tile products in one workgroup: for envelopes
// wider than XROW_MAXW tiles (the device-side width *wide) the rows would
// outlast the column steps, and the recursive inversion after the
// factorisation (whose kernels skip otherwise) is used instead.
template <typename T, typename IX>
__device__ __forceinline__ void xrow_tile(int J, int C, const T* __restrict__ F, T* __restrict__ X, T* sA,
                                          T* sB, IX ix, int xo = 0) {
  T* XD = X + tri_index(xo + J, xo + C) * TS2;
  if (C == J) {
    typedef typename Vec16<T>::type V;
    const V* src = reinterpret_cast<const V*>(F + ix(J, J) * TS2);
    V* dst = reinterpret_cast<V*>(XD);
    for (int e = threadIdx.x; e < TS2 / Vec16<T>::n; e += TILE_THREADS) dst[e] = src[e];
    return;
  }
  const int k0 = max(C, ix.first(J));
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  if (k0 < J) {
    ra.load(F + ix(J, k0) * TS2);
    rb.load(X + tri_index(xo + k0, xo + C) * TS2);
  }
  for (int K = k0; K < J; ++K) {
    lds_barrier();
    ra.store_lds(sA);
    rb.store_lds_t(sB);
    lds_barrier();
    if (K + 1 < J) {
      ra.load(F + ix(J, K + 1) * TS2);
      rb.load(X + tri_index(xo + K + 1, xo + C) * TS2);
    }
    tile_mma<T>(acc, sA, sB, T(1));  // sum L_JK X_KC
  }
  lds_barrier();
  acc.store_lds_t(sB);
  stage_tile(sA, F + ix(J, J) * TS2);  // L_JJ^{-1}
  lds_barrier();
  TileAcc<T> out;
  out.zero();
  tile_mma<T>(out, sA, sB, T(-1));
  out.store(XD);
}

// The last row of X (after the last column step).
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_xrow(int J, const int64_t* __restrict__ off,
                                                       const T* __restrict__ fac, T* __restrict__ X,
                                                       const int32_t* __restrict__ tlo,
                                                       const int32_t* __restrict__ trb,
                                                       const int32_t* __restrict__ wide, int xo) {
  if (wide && *wide > XROW_MAXW) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  xrow_tile<T, Env>(J, (int)blockIdx.x, fac + off[0] * TS2, X + off[0] * TS2, sA, sB, Env{tlo, trb}, xo);
}

// One term of V_IC = sum_K L_IK X_KC for the separator rows of a view (local
// rows nc .. ntb - 1; the separator's row i at V + (i s0 + xo + C) tiles):
// V_IC += L_IK X_KC for every such row I whose envelope reaches column K.
template <typename T, typename IX>
__device__ __forceinline__ void nd_vterm(int K, int C, int nc, int ntb, int xo, int s0, const T* __restrict__ F,
                                         const T* __restrict__ X, T* __restrict__ V, T* sA, T* sB, IX ix) {
  TileRegs<T> ra, rb;
  rb.load(X + tri_index(xo + K, xo + C) * TS2);
  rb.store_lds_t(sB);   // X_KC^T
  for (int I = nc; I < ntb; ++I) {
    if (ix.first(I) > K) continue;
    T* Vt = V + ((int64_t)(I - nc) * s0 + xo + C) * TS2;
    TileAcc<T> acc;
    acc.load(Vt);
    ra.load(F + ix(I, K) * TS2);
    lds_barrier();
    ra.store_lds(sA);
    lds_barrier();
    tile_mma<T>(acc, sA, sB, T(1));
    acc.store(Vt);
  }
}

// Column step J of one chain.  Views (vinfo non-null; the chains of a
// dissected coarse matrix, view blockIdx.y): vinfo[3 v ..] = {tile rows,
// columns the chain factors, X tile offset}, row tables at tlo / trb + v *
// vstride, split-K slots at part + 3 v slot_tiles tiles.  The chain of view
// v factors its first nc columns only: its last step forms the tiles below
// them (the separator's rows) but neither the next diagonal tile nor
// partials of columns >= nc.  V (nullable, views): the step also adds the
// term K = J - 1 of the separator rows' V = L_S,half X_half,half (row J - 1
// of X and column J - 1 of L are final by then; s0 = vinfo[9]), J
// workgroups after the rows of X; that code is in the VT instantiation only
// (present in the other one, it slowed the large grid's setup by 6 ms beside
// the batched factorisation although never executed).
template <typename T, bool VT>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_step(int J, int maxc, T* __restrict__ part,
                                                             int64_t slot_tiles,
                                                             const int32_t* __restrict__ nt,
                                                             const int64_t* __restrict__ off,
                                                             T* __restrict__ fac,
                                                             int32_t* __restrict__ status,
                                                             const int32_t* __restrict__ tlo,
                                                             const int32_t* __restrict__ trb,
                                                             T* __restrict__ X,
                                                             const int32_t* __restrict__ wide,
                                                             const int32_t* __restrict__ vinfo, int vstride,
                                                             T* __restrict__ V) {
  // The steps form a chain of dependent launches that runs beside the
  // throughput-bound batched factorisation of the subdomains; the highest
  // wave priority lets its instructions issue first on the shared SIMDs
  // (the 127 steps of the 8192-unknown coarse matrix: 10.4 -> 8.5 ms beside
  // it, the batched factorisation 9.9 -> 10.5 ms).
  int ntb = nt[0], ncol = ntb, xo = 0;
  if (vinfo) {
    const int v = blockIdx.y;
    ntb = vinfo[3 * v];
    ncol = vinfo[3 * v + 1];
    xo = vinfo[3 * v + 2];
    tlo += v * vstride;
    trb += v * vstride;
    part += 3 * v * slot_tiles * TS2;
  }
  const int m = ntb - 1 - J;  // tiles below the diagonal in column J
  if (m <= 0 || J >= ncol) return;
  const int ncj = (J + SPLITK - 1) / SPLITK;   // chunks of column J + 2
  const int nwg = m + (m > 1 ? (m - 1) * ncj : 0);
  const Env ix{tlo, trb};
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  T* F = fac + off[0] * TS2;
  const int x = blockIdx.x;
  if (x >= nwg) {  // row J of the inverse, terms of V (normal priority: off the chain)
    if (!X) return;
    const int xr = x - nwg;
    if (xr <= J) {
      if (!(wide && *wide > XROW_MAXW)) xrow_tile<T, Env>(J, xr, F, X + off[0] * TS2, sA, sB, ix, xo);
      return;
    }
    if constexpr (VT) {
      if (xr - (J + 1) < J)
        nd_vterm<T, Env>(J - 1, xr - (J + 1), ncol, ntb, xo, vinfo[9], F, X + off[0] * TS2, V, sA, sB, ix);
    }
    return;
  }
  __builtin_amdgcn_s_setprio(3);
  auto slot = [&](int C) { return part + (int64_t)(C % 3) * slot_tiles * TS2; };
  const bool next = J + 1 < ncol;   // the chain factors column J + 1
  // column J: partials over K <= J - 3, direct terms from K = max(0, J - 2)
  const int kd = J >= 2 ? J - 2 : 0;
  const int nc_j = J >= 3 ? (J - 2 + SPLITK - 1) / SPLITK : 0;
  if (x < m) {
    if constexpr (sizeof(T) == 4) {
      if (x == 0 && next) {
        chain_head<Env>(J, maxc, slot(J), slot(J + 1), F, status, smem_raw, ix);
        return;
      }
    }
    const int I = J + 1 + x;
    // rows whose envelope starts right of column J have no tile in it
    if (ix.first(I) <= J) panel_tile<T, false, Env>(J, I, kd, nc_j, maxc, slot(J), F, sA, sB, ix);
    if (x > 0 || !next) return;
    __syncthreads();
    // diagonal tile J + 1: partials over K <= J - 2, direct K = J - 1, J
    const int nc_d = J >= 2 ? (J - 1 + SPLITK - 1) / SPLITK : 0;
    diag_tile<T, false, Env>(J + 1, J >= 1 ? J - 1 : 0, nc_d, maxc, slot(J + 1), F, status, smem_raw, ix);
    return;
  }
  // partials of column J + 2 over K = 0 .. J - 1, rows J + 2 .. ntb - 1; a
  // row takes the chunks from lo[I] / SPLITK on (its terms K >= lo[I] and
  // K >= lo[J + 2]), and rows with no tile in column J + 2 none
  if (J + 2 >= ncol) return;
  const int y = x - m, mr = m - 1;
  const int I = J + 2 + y % mr, c = y / mr;
  const int lo = ix.first(I);
  if (lo > J + 2 || c < lo / SPLITK) return;
  partial_tile<T, Env>(J + 2, I, c, max(c * SPLITK, max(lo, ix.first(J + 2))), min(J, (c + 1) * SPLITK), maxc, F,
                       slot(J + 2), sA, sB, ix);
}

// The FP64 tile kernels stage two 64x65 double tiles (66.5 KB of LDS), above
// the default 64 KB dynamic limit: raise it once per kernel.
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Off-diagonal tiles of the subdomain factors rescaled to the unit
// block-lower form U_IJ = L_IJ L_JJ^{-1}: with Delta the diagonal blocks of
// the Cholesky factor L, A = U Delta Delta^T U^T, so the substitution sweeps
// take the diagonal blocks off their dependent chain (forward and backward
// with the unit factor U, the block-diagonal solve in between).  Run after
// the factorisation is complete; the diagonal tiles (holding L_JJ^{-1}) are
// read, not changed.  One workgroup per tile row.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_unit_lower(const int32_t* __restrict__ nt,
                                                             const int64_t* __restrict__ off,
                                                             const int64_t* __restrict__ xoff,
                                                             const int32_t* __restrict__ tlo,
                                                             const int32_t* __restrict__ trb,
                                                             T* __restrict__ fac) {
  const int b = blockIdx.y, I = blockIdx.x;
  if (I >= nt[b]) return;
  constexpr int S = LdsV<T>::v;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * S;
  const int64_t trow = xoff[b] / TS;
  const Env ix{tlo + trow, trb + trow};
  T* F = fac + off[b] * TS2;
  for (int J = ix.first(I); J < I; ++J) {
    lds_barrier();
    stage_tile(sA, F + ix(I, J) * TS2);      // L_IJ
    stage_tile_t(sB, F + ix(J, J) * TS2);    // (L_JJ^{-1})^T
    lds_barrier();
    TileAcc<T> out;
    out.zero();
    tile_mma<T>(out, sA, sB, T(1));          // L_IJ L_JJ^{-1}
    out.store(F + ix(I, J) * TS2);
  }
}

template <typename T>
void launch_unit_lower(int nb, int max_nt, const int32_t* nt, const int64_t* off, const int64_t* xoff,
                       const int32_t* tlo, const int32_t* trb, T* fac, hipStream_t s) {
  const size_t sh = 2 * (size_t)TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_unit_lower<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_unit_lower<T>, dim3(max_nt, nb), dim3(TILE_THREADS), sh, s, nt, off, xoff, tlo, trb, fac);
}

template <typename T>
void launch_potrf_diag(int J, int kfrom, int nparts, int maxc, const T* part, int nb,
                       const int32_t* nt, const int64_t* off, T* fac, int32_t* status,
                       hipStream_t s, const int32_t* tlo, const int32_t* trb, const int32_t* vinfo,
                       int vstride) {
  const size_t sh = diag_lds_bytes<T>();
  static bool once = (allow_lds(k_potrf_diag<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_potrf_diag<T>, dim3(nb), dim3(TILE_THREADS), sh, s, J, kfrom, nparts, maxc,
                     part, nt, off, fac, status, tlo, trb, vinfo, vstride);
}
template <typename T, bool PAIR, int R>
static void potrf_full_rows(int nb, const int32_t* nt, const int64_t* off, const int64_t* xoff, const int32_t* tlo,
                            const int32_t* trb, T* fac, int32_t* status, hipStream_t s) {
  const size_t sh = std::max(diag_lds_bytes<T>(), (size_t)std::max(4, R + (PAIR ? 2 : 1)) * TS * LdsV<T>::v * sizeof(T));
  static bool once = (allow_lds(k_potrf_full<T, PAIR, R>, sh), true);
  (void)once;
  hipLaunchKernelGGL((k_potrf_full<T, PAIR, R>), dim3(nb), dim3(TILE_THREADS), sh, s, nt, off, xoff, tlo, trb, fac,
                     status);
}

// Small matrices (a few tile rows): the diagonal update without the
// double-buffered prefetch and one row per panel step, so that the staging
// (35 KB FP32) lets four workgroups share a CU.
template <typename T>
static void potrf_full_light(int nb, const int32_t* nt, const int64_t* off, const int64_t* xoff, const int32_t* tlo,
                             const int32_t* trb, T* fac, int32_t* status, hipStream_t s) {
  const size_t sh = std::max(diag_lds_bytes<T>(), (size_t)2 * TS * LdsV<T>::v * sizeof(T));
  static bool once = (allow_lds(k_potrf_full<T, false, 1, false>, sh), true);
  (void)once;
  hipLaunchKernelGGL((k_potrf_full<T, false, 1, false>), dim3(nb), dim3(TILE_THREADS), sh, s, nt, off, xoff, tlo, trb,
                     fac, status);
}

// Largest row count whose LDS staging (rows + 1 or + 2 tiles, at least four)
// fits the 160 KB of a CU: 4 FP32; FP64 3 for one column, 2 for pairs.
int potrf_full_max_rows(bool fp64, bool pair) { return fp64 ? (pair ? 2 : 3) : 4; }

template <typename T>
void launch_potrf_full(int nb, const int32_t* nt, const int64_t* off, const int64_t* xoff, const int32_t* tlo,
                       const int32_t* trb, T* fac, int32_t* status, bool pair,
                       hipStream_t s, int rows) {
  if (rows == 1) {
    potrf_full_light<T>(nb, nt, off, xoff, tlo, trb, fac, status, s);
    return;
  }
  if (rows <= 0) rows = PanelRows<T>::v;
  rows = std::max(2, std::min(rows, potrf_full_max_rows(sizeof(T) == 8, pair)));
  if (pair) {
    if (rows == 2) potrf_full_rows<T, true, 2>(nb, nt, off, xoff, tlo, trb, fac, status, s);
    else if (rows == 3) potrf_full_rows<T, true, 3>(nb, nt, off, xoff, tlo, trb, fac, status, s);
    else if constexpr (sizeof(T) == 4) potrf_full_rows<T, true, 4>(nb, nt, off, xoff, tlo, trb, fac, status, s);
  } else {
    if (rows == 2) potrf_full_rows<T, false, 2>(nb, nt, off, xoff, tlo, trb, fac, status, s);
    else if (rows == 3) potrf_full_rows<T, false, 3>(nb, nt, off, xoff, tlo, trb, fac, status, s);
    else if constexpr (sizeof(T) == 4) potrf_full_rows<T, false, 4>(nb, nt, off, xoff, tlo, trb, fac, status, s);
  }
}
template <typename T>
void launch_potrf_step(int J, int max_nt, int maxc, T* part, int64_t slot_tiles, const int32_t* nt,
                       const int64_t* off, T* fac, int32_t* status, hipStream_t s, const int32_t* tlo,
                       const int32_t* trb, T* X, const int32_t* wide, const int32_t* vinfo, int vstride,
                       int nviews, T* V) {
  const int m = max_nt - 1 - J;
  if (m <= 0) return;
  const int nc = (J + SPLITK - 1) / SPLITK;   // chunks of column J + 2
  const int nwg = m + (m > 1 ? (m - 1) * nc : 0);
  const size_t sh = std::max(2 * TS * LdsV<T>::v * sizeof(T), diag_lds_bytes<T>());
  static bool once = (allow_lds(k_potrf_step<T, false>, sh), allow_lds(k_potrf_step<T, true>, sh), true);
  (void)once;
  const dim3 grid(nwg + (X ? J + 1 : 0) + (X && V ? J : 0), nviews);
  if (X && V)
    hipLaunchKernelGGL((k_potrf_step<T, true>), grid, dim3(TILE_THREADS), sh, s, J, maxc, part, slot_tiles, nt, off,
                       fac, status, tlo, trb, X, wide, vinfo, vstride, V);
  else
    hipLaunchKernelGGL((k_potrf_step<T, false>), grid, dim3(TILE_THREADS), sh, s, J, maxc, part, slot_tiles, nt, off,
                       fac, status, tlo, trb, X, wide, vinfo, vstride, (T*)nullptr);
}

template <typename T>
void launch_xrow(int J, const int64_t* off, const T* fac, T* X, hipStream_t s, const int32_t* tlo,
                 const int32_t* trb, const int32_t* wide, int xo) {
  const size_t sh = 2 * TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_xrow<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_xrow<T>, dim3(J + 1), dim3(TILE_THREADS), sh, s, J, off, fac, X, tlo, trb, wide, xo);
}

// Column J of X = L^{-1} from the columns right of it (X L = I):
// X_JJ = L_JJ^{-1};  X_IJ = -(sum_{K=J+1..I} X_IK L_KJ) L_JJ^{-1}, I > J.
// L holds off-diagonal factor tiles and inverted diagonal tiles, so
// X_II L_IJ uses the stored diagonal tile of row I directly.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_col(int J, const int32_t* __restrict__ nt,
                                                            const int64_t* __restrict__ off,
                                                            const T* __restrict__ L,
                                                            T* __restrict__ X) {
  const int b = blockIdx.y;
  const int I = J + blockIdx.x;
  if (I >= nt[b]) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  const T* Lb = L + off[b] * TS2;
  T* Xb = X + off[b] * TS2;
  if (I == J) {
    const T* src = Lb + tri_index(J, J) * TS2;
    T* dst = Xb + tri_index(J, J) * TS2;
    for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) dst[e] = src[e];
    return;
  }
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(Xb + tri_index(I, J + 1) * TS2);
  rb.load(Lb + tri_index(J + 1, J) * TS2);
  for (int K = J + 1; K <= I; ++K) {
    lds_barrier();
    ra.store_lds(sA);
    rb.store_lds_t(sB);
    lds_barrier();
    if (K + 1 <= I) {
      ra.load(Xb + tri_index(I, K + 1) * TS2);
      rb.load(Lb + tri_index(K + 1, J) * TS2);
    }
    tile_mma<T>(acc, sA, sB, T(1));                // acc += X_IK L_KJ
  }
  lds_barrier();
  acc.store_lds(sA);
  stage_tile_t(sB, Lb + tri_index(J, J) * TS2);
  lds_barrier();
  TileAcc<T> out;
  out.zero();
  tile_mma<T>(out, sA, sB, T(-1));                 // X_IJ = -acc L_JJ^{-1}
  out.store(Xb + tri_index(I, J) * TS2);
}

template <typename T>
void launch_trtri_col(int J, int nb, int max_nt, const int32_t* nt, const int64_t* off,
                      const T* L, T* X, hipStream_t s) {
  const size_t sh = 2 * TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_trtri_col<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_trtri_col<T>, dim3(max_nt - J, nb), dim3(TILE_THREADS), sh, s, J, nt, off, L,
                     X);
}

// Recursive (level-by-level) triangular inversion X = L^{-1} for a batch of
// matrices.  With the tile columns split into blocks of s tiles and the
// blocks paired as (A, B) = ([2ps, 2ps+s), [2ps+s, 2ps+2s)), the block of X
// below a pair's diagonal is X_BA = -X_BB L_BA X_AA, where X_AA and X_BB were
// completed at the previous level (s/2).  Starting from the inverted diagonal
// tiles (s = 1) and doubling s, every level is two independent batched tile
// products: T = L_BA X_AA, then X_BA = -X_BB T.  log2(nt) levels instead of
// nt dependent column steps.  T of matrix b occupies tiles toff[b] ..
// toff[b] + ceil(nt^2 / 4): tile (ii, jj) of pair p is p s^2 + ii s + jj.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_diag_copy(const int32_t* __restrict__ nt,
                                                                  const int64_t* __restrict__ off,
                                                                  const T* __restrict__ L,
                                                                  T* __restrict__ X,
                                                                  const int32_t* __restrict__ wide) {
  if (wide && *wide <= XROW_MAXW) return;
  const int b = blockIdx.y, k = blockIdx.x;
  if (k >= nt[b]) return;
  typedef typename Vec16<T>::type V;
  constexpr int VEC = Vec16<T>::n;
  const V* src = reinterpret_cast<const V*>(L + (off[b] + tri_index(k, k)) * TS2);
  V* dst = reinterpret_cast<V*>(X + (off[b] + tri_index(k, k)) * TS2);
  for (int e = threadIdx.x; e < TS2 / VEC; e += TILE_THREADS) dst[e] = src[e];
}

// Rows of B per workgroup in the inversion products: the R row tiles share
// the loads of the other operand (1 + 1/R tile loads per product instead of
// 2), and at about 110 registers per lane (FP32) a workgroup still fits on a
// SIMD beside the two-column batched factorisation.
constexpr int TRTRI_ROWS = 2;

// T_ij = sum_{k = j}^{B0 - 1} L_ik X_kj for i in B, j in A: workgroup (jj, g)
// forms the R tiles i = B0 + g R + r of column j = A0 + jj (one X_kj per
// step for all of them).  Workgroups with the longest sums (small jj) are
// dispatched first.  With an envelope (tlo), row i takes the terms
// k >= lo[i] only; rows whose envelope starts in B get T_ij = 0.
template <typename T, int R>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_rec_t(int s, const int32_t* __restrict__ nt,
                                                              const int64_t* __restrict__ off,
                                                              const int64_t* __restrict__ toff,
                                                              const T* __restrict__ L,
                                                              const T* __restrict__ X,
                                                              T* __restrict__ Tb,
                                                              const int64_t* __restrict__ xoff,
                                                              const int32_t* __restrict__ tlo,
                                                              const int32_t* __restrict__ wide) {
  if (wide && *wide <= XROW_MAXW) return;  // inverted beside the factorisation
  constexpr int S = LdsV<T>::v;
  const int b = blockIdx.z, p = blockIdx.y;
  const int ng = (s + R - 1) / R;
  const int jj = blockIdx.x / ng, g = blockIdx.x % ng;
  const int A0 = 2 * p * s, B0 = A0 + s;
  const int j = A0 + jj, i0 = B0 + g * R;
  const int nr = min(R, min(B0 + s, nt[b]) - i0);
  if (nr <= 0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* sB = lds + R * TS * S;
  const T* Lb = L + off[b] * TS2;
  const T* Xb = X + off[b] * TS2;
  const int32_t* lo = tlo ? tlo + xoff[b] / TS : nullptr;
  int lor[R];
#pragma unroll
  for (int r = 0; r < R; ++r) lor[r] = r < nr && lo ? lo[i0 + r] : 0;
  const int k0 = max(j, lor[0]);
  TileAcc<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r].zero();
  TileRegs<T> ra[R], rb;
  if (k0 < B0) {
    const int n1 = rows_upto<R>(lor, nr, k0);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < n1) ra[r].load(Lb + tri_index(i0 + r, k0) * TS2);
    rb.load(Xb + tri_index(k0, j) * TS2);
  }
  for (int k = k0; k < B0; ++k) {
    const int nk = rows_upto<R>(lor, nr, k);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nk) ra[r].store_lds(lds + r * TS * S);
    rb.store_lds_t(sB);
    lds_barrier();
    if (k + 1 < B0) {
      const int n1 = rows_upto<R>(lor, nr, k + 1);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < n1) ra[r].load(Lb + tri_index(i0 + r, k + 1) * TS2);
      rb.load(Xb + tri_index(k + 1, j) * TS2);
    }
    tile_mma_rows<T, R>(acc, nk, lds, sB, T(1));   // T_ij += L_ik X_kj
  }
  T* Tp = Tb + (toff[b] + (int64_t)p * s * s + (int64_t)(g * R) * s + jj) * TS2;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) acc[r].store(Tp + (int64_t)r * s * TS2);
}

// X_ij = -sum_{k = B0}^{i} X_ik T_kj for i in B, j in A: workgroup (g, jj)
// forms the R tiles i = i0, i0 - 1, .. (from the top of B down) of column
// j; row i0 - r leaves the sum after k = i0 - r, so the rows still summing
// are always the first ones.  Longest sums (large i) first.  With an
// envelope (tlo), T_kj = 0 for the rows k of B past the last one whose
// envelope reaches into A, and the sums stop there.
template <typename T, int R>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_rec_x(int s, const int32_t* __restrict__ nt,
                                                              const int64_t* __restrict__ off,
                                                              const int64_t* __restrict__ toff,
                                                              const T* __restrict__ Tb,
                                                              T* __restrict__ X,
                                                              const int64_t* __restrict__ xoff,
                                                              const int32_t* __restrict__ tlo,
                                                              const int32_t* __restrict__ wide) {
  if (wide && *wide <= XROW_MAXW) return;  // inverted beside the factorisation
  constexpr int S = LdsV<T>::v;
  const int b = blockIdx.z, p = blockIdx.y;
  const int g = blockIdx.x / s, jj = blockIdx.x % s;
  const int A0 = 2 * p * s, B0 = A0 + s;
  const int top = min(B0 + s, nt[b]) - 1 - B0 - g * R;   // row of B (0-based) of the group's first tile
  if (top < 0) return;
  const int nrows = min(R, top + 1);
  const int i0 = B0 + top, j = A0 + jj;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* sB = lds + R * TS * S;
  T* Xb = X + off[b] * TS2;
  const T* Tp = Tb + (toff[b] + (int64_t)p * s * s + jj) * TS2;  // T_kj at Tp + (k - B0) s TS2
  // last row of B with nonzero T (its envelope reaches into A)
  int kend = i0;
  if (tlo) {
    const int32_t* lo = tlo + xoff[b] / TS;
    const int bend = min(B0 + s, nt[b]);
    int kz = B0 - 1;
    while (kz + 1 < bend && lo[kz + 1] < B0) ++kz;
    kend = min(i0, kz);
  }
  TileAcc<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r].zero();
  TileRegs<T> ra[R], rb;
  if (B0 <= kend) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nrows) ra[r].load(Xb + tri_index(i0 - r, B0) * TS2);
    rb.load(Tp);
  }
  for (int k = B0; k <= kend; ++k) {
    const int nr = min(nrows, i0 - k + 1);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nr) ra[r].store_lds(lds + r * TS * S);
    rb.store_lds_t(sB);
    lds_barrier();
    if (k + 1 <= kend) {
      const int nr1 = min(nrows, i0 - k);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < nr1) ra[r].load(Xb + tri_index(i0 - r, k + 1) * TS2);
      rb.load(Tp + (int64_t)(k + 1 - B0) * s * TS2);
    }
    tile_mma_rows<T, R>(acc, nr, lds, sB, T(-1));  // X_ij -= X_ik T_kj
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nrows) acc[r].store(Xb + tri_index(i0 - r, j) * TS2);
}

template <typename T>
void launch_trtri_rec(int nb, int max_nt, const int32_t* nt, const int64_t* off, const int64_t* toff,
                      const T* L, T* X, T* Tb, hipStream_t st, const int64_t* xoff, const int32_t* tlo,
                      const int32_t* wide) {
  constexpr int R = TRTRI_ROWS;
  const size_t sh = (R + 1) * TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_trtri_rec_t<T, R>, sh), allow_lds(k_trtri_rec_x<T, R>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_trtri_diag_copy<T>, dim3(max_nt, nb), dim3(TILE_THREADS), 0, st, nt, off, L, X, wide);
  for (int s = 1; s < max_nt; s *= 2) {
    const int npairs = (max_nt + 2 * s - 1) / (2 * s);
    const dim3 grid(s * ((s + R - 1) / R), npairs, nb);
    hipLaunchKernelGGL((k_trtri_rec_t<T, R>), grid, dim3(TILE_THREADS), sh, st, s, nt, off, toff, L, X, Tb, xoff,
                       tlo, wide);
    hipLaunchKernelGGL((k_trtri_rec_x<T, R>), grid, dim3(TILE_THREADS), sh, st, s, nt, off, toff, Tb, X, xoff, tlo,
                       wide);
  }
}

// M = X^T X = A^{-1} from X = L^{-1}:  M_IJ = sum_{K >= I} X_KI^T X_KJ, I >= J.
// Diagonal tiles are written in full (both triangles).
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_lauum(const int32_t* __restrict__ nt,
                                                        const int64_t* __restrict__ off,
                                                        const T* __restrict__ X,
                                                        T* __restrict__ M) {
  const int b = blockIdx.y;
  const int ntb = nt[b];
  const int64_t t = blockIdx.x;
  if (t >= (int64_t)ntb * (ntb + 1) / 2) return;
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
  while ((int64_t)I * (I + 1) / 2 > t) --I;
  const int J = (int)(t - (int64_t)I * (I + 1) / 2);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  const T* Xb = X + off[b] * TS2;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(Xb + tri_index(I, I) * TS2);
  rb.load(Xb + tri_index(I, J) * TS2);
  for (int K = I; K < ntb; ++K) {
    lds_barrier();
    ra.store_lds_t(sA);
    rb.store_lds_t(sB);
    lds_barrier();
    if (K + 1 < ntb) {
      ra.load(Xb + tri_index(K + 1, I) * TS2);
      rb.load(Xb + tri_index(K + 1, J) * TS2);
    }
    tile_mma<T>(acc, sA, sB, T(1));                // M_IJ += X_KI^T X_KJ
  }
  acc.store(M + off[b] * TS2 + tri_index(I, J) * TS2);
}

template <typename T>
void launch_lauum(int nb, int max_nt, const int32_t* nt, const int64_t* off, const T* X, T* M,
                  hipStream_t s) {
  const size_t sh = 2 * TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_lauum<T>, sh), true);
  (void)once;
  const int ntiles = max_nt * (max_nt + 1) / 2;
  hipLaunchKernelGGL(k_lauum<T>, dim3(ntiles, nb), dim3(TILE_THREADS), sh, s, nt, off, X, M);
}

// ---------------------------------------------------------------------------
// The separator of a dissected coarse matrix (tile rows s0 = ta + tb .. nt - 1
// of the packed triangle; the first half's rows 0 .. ta - 1, the second
// half's ta .. s0 - 1, with no tiles coupling the halves).  Once the chains
// of both halves have formed the separator's tiles L_IK, K < s0, and the
// rows of X = L^{-1} of both halves, the block form of L X = I gives
//   S = A_SS - L_S,half L_S,half^T (both halves)  ->  L_SS, X_SS = L_SS^{-1}
//   X_S,half = -X_SS L_S,half X_half,half,
// formed as V_IC = sum_{K in C's half, K >= max(C, lo[I])} L_IK X_KC for
// every separator row I and column C < s0 (the column step K + 1 of C's
// half adds term K, one product per tile beside the chain), then
// X_IC = -sum_{s0 <= I' <= I} X_II' V_I'C.

// Blocks [0, npair nck): split-K partials of the Schur complement, tile pair
// p = i (i + 1) / 2 + j (j <= i, separator-local) and chunk c of K < s0,
// spart[p nck + c] = sum_K L_IK L_JK^T; then one block per column C < s0
// adding the last term of V_IC (vbuf[i s0 + C], the other terms added by the
// column steps) for every separator row i.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_nd_sv(int ta, int tb, int ts, const int64_t* __restrict__ off,
                                                        const T* __restrict__ fac, const T* __restrict__ X,
                                                        const int32_t* __restrict__ clo, T* __restrict__ spart,
                                                        T* __restrict__ vbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  const int s0 = ta + tb, nck = (s0 + SPLITK - 1) / SPLITK;
  const int nsp = ts * (ts + 1) / 2 * nck;
  const T* F = fac + off[0] * TS2;
  const T* Xb = X + off[0] * TS2;
  const int x = blockIdx.x;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  if (x < nsp) {
    const int p = x / nck, c = x % nck;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    const int I = s0 + i, J = s0 + (p - i * (i + 1) / 2);
    const int k0 = max(c * SPLITK, max(clo[I], clo[J])), k1 = min((c + 1) * SPLITK, s0);
    if (k0 < k1) {
      ra.load(F + tri_index(I, k0) * TS2);
      rb.load(F + tri_index(J, k0) * TS2);
    }
    for (int K = k0; K < k1; ++K) {
      lds_barrier();
      ra.store_lds(sA);
      rb.store_lds(sB);
      lds_barrier();
      if (K + 1 < k1) {
        ra.load(F + tri_index(I, K + 1) * TS2);
        rb.load(F + tri_index(J, K + 1) * TS2);
      }
      tile_mma<T>(acc, sA, sB, T(1));   // L_IK L_JK^T
    }
    acc.store(spart + (int64_t)x * TS2);
    return;
  }
  // the last term of V (K = the last column of C's half), whose row of X the
  // chain's last step formed
  const int C = x - nsp;
  if (C >= s0) return;
  const int K = C < ta ? ta - 1 : s0 - 1;
  rb.load(Xb + tri_index(K, C) * TS2);
  rb.store_lds_t(sB);   // X_KC^T
  for (int i = 0; i < ts; ++i) {
    const int I = s0 + i;
    if (clo[I] > K) continue;
    T* Vt = vbuf + ((int64_t)i * s0 + C) * TS2;
    TileAcc<T> v;
    v.load(Vt);
    ra.load(F + tri_index(I, K) * TS2);
    lds_barrier();
    ra.store_lds(sA);
    lds_barrier();
    tile_mma<T>(v, sA, sB, T(1));      // V_IC += L_IK X_KC
    v.store(Vt);
  }
}

// The Schur complement into the separator's tiles of the factor storage (a
// tile left of the row's envelope starts from zero: it was never assembled).
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_nd_schur(int ta, int tb, const int64_t* __restrict__ off,
                                                           T* __restrict__ fac, const int32_t* __restrict__ clo,
                                                           const T* __restrict__ spart) {
  const int s0 = ta + tb, nck = (s0 + SPLITK - 1) / SPLITK;
  const int p = blockIdx.x;
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int I = s0 + i, J = s0 + (p - i * (i + 1) / 2);
  T* D = fac + (off[0] + tri_index(I, J)) * TS2;
  TileAcc<T> acc;
  if (J >= clo[I]) acc.load(D);
  else acc.zero();
  sub_tiles(acc, spart + (int64_t)p * nck * TS2, TS2, nck);
  acc.store(D);
}

// X_IC = -sum_{s0 <= I' <= I} X_II' V_I'C for the separator's rows, C < s0.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_nd_xs(int ta, int tb, const int64_t* __restrict__ off,
                                                        T* __restrict__ X, const T* __restrict__ vbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LdsV<T>::v;
  const int s0 = ta + tb;
  const int i = blockIdx.x / s0, C = blockIdx.x % s0;
  const int I = s0 + i;
  T* Xb = X + off[0] * TS2;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(Xb + tri_index(I, s0) * TS2);
  rb.load(vbuf + (int64_t)C * TS2);
  for (int u = 0; u <= i; ++u) {
    lds_barrier();
    ra.store_lds(sA);
    rb.store_lds_t(sB);
    lds_barrier();
    if (u < i) {
      ra.load(Xb + tri_index(I, s0 + u + 1) * TS2);
      rb.load(vbuf + ((int64_t)(u + 1) * s0 + C) * TS2);
    }
    tile_mma<T>(acc, sA, sB, T(-1));    // -X_II' V_I'C
  }
  acc.store(Xb + tri_index(I, C) * TS2);
}

// Factorisation and inverse X = L^{-1} of a dissected coarse matrix (single
// grid; nd tiles ta, tb, ts; views from launch_nd_views with vstride entries
// per view): the chains of the two halves in the same launches (views 0 and
// 1, the rows of X formed beside the steps), the separator's Schur
// complement and the last terms of V, the separator's chain (view 2, whose
// split-K slots reuse view 0's, free by then), X_SS's last row, then
// X_S,half.  part holds six slots of vstride * maxc tiles; vbuf ts * s0
// tiles (cleared here).
template <typename T>
void factor_nd(int ta, int tb, int ts, int maxc, T* part, const int64_t* off, T* fac, T* X, int32_t* status,
               const int32_t* nt, const int32_t* clo, const int32_t* vinfo, const int32_t* vlo, const int32_t* vrb,
               int vstride, T* vbuf, hipStream_t s) {
  const int s0 = ta + tb;
  const int64_t slot_tiles = (int64_t)vstride * maxc;
  (void)hipMemsetAsync(vbuf, 0, (size_t)ts * s0 * TS2 * sizeof(T), s);
  launch_potrf_diag<T>(0, 0, 0, maxc, part, 2, nt, off, fac, status, s, vlo, vrb, vinfo, vstride);
  for (int J = 0; J < std::max(ta, tb); ++J)
    launch_potrf_step<T>(J, std::max(ta, tb) + ts, maxc, part, slot_tiles, nt, off, fac, status, s, vlo, vrb, X,
                         nullptr, vinfo, vstride, 2, vbuf);
  const int nck = (s0 + SPLITK - 1) / SPLITK;
  const int npair = ts * (ts + 1) / 2;
  const size_t sh = 2 * TS * LdsV<T>::v * sizeof(T);
  static bool once = (allow_lds(k_nd_sv<T>, sh), allow_lds(k_nd_xs<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_nd_sv<T>, dim3(npair * nck + s0), dim3(TILE_THREADS), sh, s, ta, tb, ts, off, fac, X,
                     clo, part, vbuf);
  hipLaunchKernelGGL(k_nd_schur<T>, dim3(npair), dim3(TILE_THREADS), 0, s, ta, tb, off, fac, clo, part);
  const int32_t* slo = vlo + 2 * vstride;
  const int32_t* srb = vrb + 2 * vstride;
  launch_potrf_diag<T>(0, 0, 0, maxc, part, 1, nt, off, fac, status, s, slo, srb, vinfo + 6, vstride);
  for (int J = 0; J + 1 < ts; ++J)
    launch_potrf_step<T>(J, ts, maxc, part, slot_tiles, nt, off, fac, status, s, slo, srb, X, nullptr, vinfo + 6,
                         vstride, 1);
  launch_xrow<T>(ts - 1, off, fac, X, s, slo, srb, nullptr, s0);
  hipLaunchKernelGGL(k_nd_xs<T>, dim3(ts * s0), dim3(TILE_THREADS), sh, s, ta, tb, off, X, vbuf);
}

#define INST(T)                                                                                    \
  template void launch_unit_lower<T>(int, int, const int32_t*, const int64_t*, const int64_t*,     \
                                     const int32_t*, const int32_t*, T*, hipStream_t);              \
  template void launch_potrf_diag<T>(int, int, int, int, const T*, int, const int32_t*,            \
                                     const int64_t*, T*, int32_t*, hipStream_t, const int32_t*,    \
                                     const int32_t*, const int32_t*, int);                         \
  template void launch_potrf_full<T>(int, const int32_t*, const int64_t*, const int64_t*,          \
                                     const int32_t*, const int32_t*, T*, int32_t*, bool,           \
                                     hipStream_t, int);                                            \
  template void launch_potrf_step<T>(int, int, int, T*, int64_t, const int32_t*, const int64_t*,    \
                                     T*, int32_t*, hipStream_t, const int32_t*, const int32_t*, T*, \
                                     const int32_t*, const int32_t*, int, int, T*);                \
  template void launch_xrow<T>(int, const int64_t*, const T*, T*, hipStream_t, const int32_t*,     \
                               const int32_t*, const int32_t*, int);                               \
  template void factor_nd<T>(int, int, int, int, T*, const int64_t*, T*, T*, int32_t*,             \
                             const int32_t*, const int32_t*, const int32_t*, const int32_t*,       \
                             const int32_t*, int, T*, hipStream_t);                                \
  template void launch_trtri_col<T>(int, int, int, const int32_t*, const int64_t*, const T*, T*,   \
                                    hipStream_t);                                                  \
  template void launch_lauum<T>(int, int, const int32_t*, const int64_t*, const T*, T*, hipStream_t); \
  template void launch_trtri_rec<T>(int, int, const int32_t*, const int64_t*, const int64_t*,     \
                                    const T*, T*, T*, hipStream_t, const int64_t*, const int32_t*,  \
                                    const int32_t*);
INST(float)
INST(double)
#undef INST

}  // namespace sfcdd
