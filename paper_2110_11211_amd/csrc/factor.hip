// Batched dense Cholesky factorisation of the subdomain matrices and of the
// coarse matrix (factor once, Sec. 3.1), on packed lower 64x64 tiles with
// MFMA tile products.  Left-looking over tile columns J: one launch factors
// the diagonal tiles (J, J) of every matrix of the batch, a second one
// finishes the sub-diagonal tiles (I, J), I > J.  The diagonal tiles keep the
// INVERSE of the diagonal Cholesky block, L_JJ^{-1}, so that both the panel
// update and the substitution sweeps are tile products.
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

// Cholesky factor and inverse of one DB x DB diagonal block at (o, o) of sC,
// by lanes 0..DB-1 of the first wave alone (one wave issues its LDS
// operations in program order, so no barrier is needed inside):
// factoring, lane i owns block row i; inverting, lane c owns column c of the
// inverse, written to dinv (row-major DB x DB, lower).
template <typename T>
__device__ void factor_block(T* __restrict__ sC, int o, T* __restrict__ dinv,
                             T* __restrict__ colbuf, int32_t* status) {
  constexpr int PS = Pstride<T>::v;
  const int i = threadIdx.x;
  if (i >= DB) return;
  for (int k = 0; k < DB; ++k) {
    T piv = sC[(o + k) * PS + o + k];
    if (!(piv > T(0))) {
      if (i == k) atomicExch(status, -6);
      piv = T(1);
    }
    const T dk = sqrt(piv);
    const T rdk = T(1) / dk;
    const T l = (i > k) ? sC[(o + i) * PS + o + k] * rdk : (i == k ? dk : T(0));
    if (i >= k) sC[(o + i) * PS + o + k] = l;
    colbuf[i] = (i > k) ? l : T(0);
#pragma unroll
    for (int j = 0; j < DB; ++j)
      if (j > k) sC[(o + i) * PS + o + j] -= l * colbuf[j];
  }
  // inverse of the DB x DB lower factor, column c per lane
  const int c = i;
  T x[DB];
#pragma unroll
  for (int r = 0; r < DB; ++r) x[r] = (r == c) ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < DB; ++k) {
    x[k] = x[k] / sC[(o + k) * PS + o + k];
#pragma unroll
    for (int r = k + 1; r < DB; ++r) x[r] -= sC[(o + r) * PS + o + k] * x[k];
  }
#pragma unroll
  for (int r = 0; r < DB; ++r) dinv[r * DB + c] = x[r];
}

// Cholesky factorisation and inversion of a TS x TS LDS tile (stride
// Pstride, lower part read), blocked by DB: the DB x DB diagonal blocks are
// factored and inverted by one wave, the panels, trailing updates and the
// off-diagonal blocks of the inverse by the whole workgroup.
// On exit sX holds L^{-1} (lower; stride Pstride); sC holds L (lower).
// A non-positive pivot sets *status to -6 and is replaced by 1.
template <typename T>
__device__ void potrf_inv_tile(T* __restrict__ sC, T* __restrict__ sX, T* __restrict__ dinv,
                               T* __restrict__ colbuf, int32_t* status) {
  constexpr int PS = Pstride<T>::v;
  const int tid = threadIdx.x;
  __syncthreads();
  for (int bk = 0; bk < NDB; ++bk) {
    const int o = bk * DB;
    factor_block(sC, o, dinv + bk * DB * DB, colbuf, status);
    __syncthreads();
    // panel: L[r][o..o+DB) = C[r][o..o+DB) Dinv^T for rows below the block
    const int nrow = TS - o - DB;
    T pv[(TS - DB) * DB / TILE_THREADS];
    const T* Di = dinv + bk * DB * DB;
#pragma unroll
    for (int q = 0; q < (TS - DB) * DB / TILE_THREADS; ++q) {
      const int t = tid + q * TILE_THREADS;
      pv[q] = T(0);
      if (t < nrow * DB) {
        const int r = o + DB + t / DB, cc = t % DB;
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < DB; ++m) acc += sC[r * PS + o + m] * Di[cc * DB + m];
        pv[q] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (TS - DB) * DB / TILE_THREADS; ++q) {
      const int t = tid + q * TILE_THREADS;
      if (t < nrow * DB) sC[(o + DB + t / DB) * PS + o + t % DB] = pv[q];
    }
    __syncthreads();
    // trailing update of the lower part below and right of the block:
    // C[i][j] -= sum_m L[i][o+m] L[j][o+m] for o+DB <= j <= i
    const int m0 = o + DB;
    const int span = TS - m0;
    for (int e = tid; e < span * span; e += TILE_THREADS) {
      const int i = m0 + e / span, j = m0 + e % span;
      if (j > i) continue;
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < DB; ++m) acc += sC[i * PS + o + m] * sC[j * PS + o + m];
      sC[i * PS + j] -= acc;
    }
    __syncthreads();
  }
  // X = L^{-1} by block rows: X_II = Dinv_I,
  // X_IJ = -Dinv_I sum_{K=J}^{I-1} L_IK X_KJ for J < I.
  for (int e = tid; e < TS * TS; e += TILE_THREADS) {
    const int r = e / TS, cc = e % TS;
    const int I = r / DB, J = cc / DB;
    sX[r * PS + cc] = (I == J) ? dinv[I * DB * DB + (r % DB) * DB + (cc % DB)] : T(0);
  }
  __syncthreads();
  T* tmp = sC;  // upper part of sC is free: tmp block (I, J) stored at rows of J, columns of I
  for (int I = 1; I < NDB; ++I) {
    // T_IJ = sum_{K=J}^{I-1} L_IK X_KJ for J < I, one element per thread
    for (int e = tid; e < I * DB * DB; e += TILE_THREADS) {
      const int J = e / (DB * DB), r = (e / DB) % DB, cc = e % DB;
      T acc = T(0);
      for (int K = J; K < I; ++K) {
#pragma unroll
        for (int m = 0; m < DB; ++m)
          acc += sC[(I * DB + r) * PS + K * DB + m] * sX[(K * DB + m) * PS + J * DB + cc];
      }
      tmp[(J * DB + cc) * PS + I * DB + r] = acc;  // transposed into the free upper part
    }
    __syncthreads();
    for (int e = tid; e < I * DB * DB; e += TILE_THREADS) {
      const int J = e / (DB * DB), r = (e / DB) % DB, cc = e % DB;
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < DB; ++m)
        acc += dinv[I * DB * DB + r * DB + m] * tmp[(J * DB + cc) * PS + I * DB + m];
      sX[(I * DB + r) * PS + J * DB + cc] = -acc;
    }
    __syncthreads();
  }
}

// LDS of the diagonal kernel: two Pstride tiles (C, X), the DB x DB block
// inverses and a column buffer.  The GEMM staging (two LDS_S tiles) fits in
// the same space.
template <typename T>
constexpr size_t diag_lds_bytes() {
  return (2 * (size_t)TS * Pstride<T>::v + NDB * DB * DB + TS) * sizeof(T);
}

// left != 0: left-looking, the tile first receives -sum_{K<J} L_JK L_JK^T
// in this workgroup.  nparts > 0 (single matrix, split-K): that update was
// precomputed as nparts partial tiles part[I][c] by k_potrf_partial.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_diag(int J, int left, int nparts, int maxc,
                                                             const T* __restrict__ part,
                                                             const int32_t* __restrict__ nt,
                                                             const int64_t* __restrict__ off,
                                                             T* __restrict__ fac,
                                                             int32_t* __restrict__ status) {
  const int b = blockIdx.x;
  if (J >= nt[b]) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* F = fac + off[b] * TS2;
  TileAcc<T> acc;
  acc.load(F + tri_index(J, J) * TS2);
  for (int c = 0; c < nparts; ++c) acc.sub(part + ((int64_t)J * maxc + c) * TS2);
  const int nk = left ? J : 0;
  TileRegs<T> ra;
  if (nk > 0) ra.load(F + tri_index(J, 0) * TS2);
  for (int K = 0; K < nk; ++K) {
    __syncthreads();
    ra.store_lds(sA);
    __syncthreads();
    if (K + 1 < nk) ra.load(F + tri_index(J, K + 1) * TS2);
    tile_mma<T, false, true>(acc, sA, sA, T(-1));  // A_JJ -= L_JK L_JK^T
  }
  __syncthreads();
  constexpr int PS = Pstride<T>::v;
  T* sC = reinterpret_cast<T*>(smem_raw);
  T* sX = sC + TS * PS;
  T* dinv = sX + TS * PS;
  T* colbuf = dinv + NDB * DB * DB;
  for (int a = 0; a < 2; ++a)
    for (int b2 = 0; b2 < 2; ++b2)
      for (int r = 0; r < 4; ++r) sC[TileAcc<T>::row(a, r) * PS + TileAcc<T>::col(b2)] = acc.c[a][b2][r];
  potrf_inv_tile(sC, sX, dinv, colbuf, status);
  T* D = F + tri_index(J, J) * TS2;
  for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) {
    const int i = e / TS, j = e % TS;
    D[e] = j <= i ? sX[i * PS + j] : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_panel(int J, int left, int nparts, int maxc,
                                                              const T* __restrict__ part,
                                                              const int32_t* __restrict__ nt,
                                                              const int64_t* __restrict__ off,
                                                              T* __restrict__ fac) {
  const int b = blockIdx.y;
  const int I = J + 1 + blockIdx.x;
  if (I >= nt[b]) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LDS_S;
  T* F = fac + off[b] * TS2;
  TileAcc<T> acc;
  acc.load(F + tri_index(I, J) * TS2);
  for (int c = 0; c < nparts; ++c) acc.sub(part + ((int64_t)I * maxc + c) * TS2);
  const int nk = left ? J : 0;
  TileRegs<T> ra, rb;
  if (nk > 0) {
    ra.load(F + tri_index(I, 0) * TS2);
    rb.load(F + tri_index(J, 0) * TS2);
  }
  for (int K = 0; K < nk; ++K) {
    __syncthreads();
    ra.store_lds(sA);
    rb.store_lds(sB);
    __syncthreads();
    if (K + 1 < nk) {
      ra.load(F + tri_index(I, K + 1) * TS2);
      rb.load(F + tri_index(J, K + 1) * TS2);
    }
    tile_mma<T, false, true>(acc, sA, sB, T(-1));  // A_IJ -= L_IK L_JK^T
  }
  __syncthreads();
  acc.store_lds(sA);
  stage_tile(sB, F + tri_index(J, J) * TS2);      // L_JJ^{-1}
  __syncthreads();
  TileAcc<T> out;
  out.zero();
  tile_mma<T, false, true>(out, sA, sB, T(1));     // L_IJ = A_IJ L_JJ^{-T}
  out.store(F + tri_index(I, J) * TS2);
}

// The FP64 tile kernels stage two 64x65 double tiles (66.5 KB of LDS), above
// the default 64 KB dynamic limit: raise it once per kernel.
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
void launch_potrf_diag(int J, int left, int nparts, int maxc, const T* part, int nb,
                       const int32_t* nt, const int64_t* off, T* fac, int32_t* status,
                       hipStream_t s) {
  const size_t sh = diag_lds_bytes<T>();
  static bool once = (allow_lds(k_potrf_diag<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_potrf_diag<T>, dim3(nb), dim3(TILE_THREADS), sh, s, J, left, nparts, maxc,
                     part, nt, off, fac, status);
}
template <typename T>
void launch_potrf_panel(int J, int left, int nparts, int maxc, const T* part, int nb, int max_nt,
                        const int32_t* nt, const int64_t* off, T* fac, hipStream_t s) {
  if (max_nt - 1 - J <= 0) return;
  const size_t sh = 2 * TS * LDS_S * sizeof(T);
  static bool once = (allow_lds(k_potrf_panel<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_potrf_panel<T>, dim3(max_nt - 1 - J, nb), dim3(TILE_THREADS), sh, s, J, left,
                     nparts, maxc, part, nt, off, fac);
}

// Split-K update of column J of one matrix (batch 1): workgroup (x, c)
// computes part[I][c] = sum_{K in chunk c} L_IK L_JK^T for I = J + x, chunk
// c = [c SPLITK, (c + 1) SPLITK) intersected with [0, J).  Many workgroups per
// column instead of one long K loop per tile.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_potrf_partial(int J, int maxc,
                                                                const int32_t* __restrict__ nt,
                                                                const int64_t* __restrict__ off,
                                                                const T* __restrict__ fac,
                                                                T* __restrict__ part) {
  const int I = J + blockIdx.x;
  const int c = blockIdx.y;
  if (I >= nt[0]) return;
  const int k0 = c * SPLITK, k1 = min(J, k0 + SPLITK);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LDS_S;
  const T* F = fac + off[0] * TS2;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(F + tri_index(I, k0) * TS2);
  rb.load(F + tri_index(J, k0) * TS2);
  for (int K = k0; K < k1; ++K) {
    __syncthreads();
    ra.store_lds(sA);
    rb.store_lds(sB);
    __syncthreads();
    if (K + 1 < k1) {
      ra.load(F + tri_index(I, K + 1) * TS2);
      rb.load(F + tri_index(J, K + 1) * TS2);
    }
    tile_mma<T, false, true>(acc, sA, sB, T(1));
  }
  acc.store(part + ((int64_t)I * maxc + c) * TS2);
}

template <typename T>
void launch_potrf_partial(int J, int max_nt, int maxc, const int32_t* nt, const int64_t* off,
                          const T* fac, T* part, hipStream_t s) {
  const int nc = (J + SPLITK - 1) / SPLITK;
  if (nc == 0) return;
  const size_t sh = 2 * TS * LDS_S * sizeof(T);
  static bool once = (allow_lds(k_potrf_partial<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_potrf_partial<T>, dim3(max_nt - J, nc), dim3(TILE_THREADS), sh, s, J, maxc,
                     nt, off, fac, part);
  (void)maxc;
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
  T* sB = sA + TS * LDS_S;
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
    __syncthreads();
    ra.store_lds(sA);
    rb.store_lds(sB);
    __syncthreads();
    if (K + 1 <= I) {
      ra.load(Xb + tri_index(I, K + 1) * TS2);
      rb.load(Lb + tri_index(K + 1, J) * TS2);
    }
    tile_mma<T, false, false>(acc, sA, sB, T(1));
  }
  __syncthreads();
  acc.store_lds(sA);
  stage_tile(sB, Lb + tri_index(J, J) * TS2);
  __syncthreads();
  TileAcc<T> out;
  out.zero();
  tile_mma<T, false, false>(out, sA, sB, T(-1));
  out.store(Xb + tri_index(I, J) * TS2);
}

template <typename T>
void launch_trtri_col(int J, int nb, int max_nt, const int32_t* nt, const int64_t* off,
                      const T* L, T* X, hipStream_t s) {
  const size_t sh = 2 * TS * LDS_S * sizeof(T);
  static bool once = (allow_lds(k_trtri_col<T>, sh), true);
  (void)once;
  hipLaunchKernelGGL(k_trtri_col<T>, dim3(max_nt - J, nb), dim3(TILE_THREADS), sh, s, J, nt, off, L,
                     X);
}

// Split-K form of the column step above for one matrix (batch 1):
// k_trtri_partial computes part[I][c] = sum_{K in chunk c} X_IK L_KJ over the
// chunks c of [J+1, I]; k_trtri_finish sums them and applies -L_JJ^{-1}.
template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_partial(int J, int maxc,
                                                                const int32_t* __restrict__ nt,
                                                                const int64_t* __restrict__ off,
                                                                const T* __restrict__ L,
                                                                const T* __restrict__ X,
                                                                T* __restrict__ part) {
  const int I = J + 1 + blockIdx.x;
  const int c = blockIdx.y;
  const int k0 = J + 1 + c * SPLITK;
  if (I >= nt[0] || k0 > I) return;
  const int k1 = min(I + 1, k0 + SPLITK);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LDS_S;
  const T* Lb = L + off[0] * TS2;
  const T* Xb = X + off[0] * TS2;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(Xb + tri_index(I, k0) * TS2);
  rb.load(Lb + tri_index(k0, J) * TS2);
  for (int K = k0; K < k1; ++K) {
    __syncthreads();
    ra.store_lds(sA);
    rb.store_lds(sB);
    __syncthreads();
    if (K + 1 < k1) {
      ra.load(Xb + tri_index(I, K + 1) * TS2);
      rb.load(Lb + tri_index(K + 1, J) * TS2);
    }
    tile_mma<T, false, false>(acc, sA, sB, T(1));
  }
  acc.store(part + ((int64_t)I * maxc + c) * TS2);
}

template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_trtri_finish(int J, int maxc,
                                                               const int32_t* __restrict__ nt,
                                                               const int64_t* __restrict__ off,
                                                               const T* __restrict__ L,
                                                               T* __restrict__ X,
                                                               const T* __restrict__ part) {
  const int I = J + blockIdx.x;
  if (I >= nt[0]) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sA = reinterpret_cast<T*>(smem_raw);
  T* sB = sA + TS * LDS_S;
  const T* Lb = L + off[0] * TS2;
  T* Xb = X + off[0] * TS2;
  if (I == J) {
    const T* src = Lb + tri_index(J, J) * TS2;
    T* dst = Xb + tri_index(J, J) * TS2;
    for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) dst[e] = src[e];
    return;
  }
  TileAcc<T> acc;
  acc.zero();
  const int np = (I - J + SPLITK - 1) / SPLITK;
  for (int c = 0; c < np; ++c) acc.sub(part + ((int64_t)I * maxc + c) * TS2);  // acc = -sum
  acc.store_lds(sA);
  stage_tile(sB, Lb + tri_index(J, J) * TS2);
  __syncthreads();
  TileAcc<T> out;
  out.zero();
  tile_mma<T, false, false>(out, sA, sB, T(1));
  out.store(Xb + tri_index(I, J) * TS2);
}

template <typename T>
void launch_trtri_splitk(int J, int max_nt, int maxc, const int32_t* nt, const int64_t* off,
                         const T* L, T* X, T* part, hipStream_t s) {
  const size_t sh = 2 * TS * LDS_S * sizeof(T);
  static bool once = (allow_lds(k_trtri_partial<T>, sh), allow_lds(k_trtri_finish<T>, sh), true);
  (void)once;
  const int m = max_nt - 1 - J;
  if (m > 0)
    hipLaunchKernelGGL(k_trtri_partial<T>, dim3(m, (m + SPLITK - 1) / SPLITK), dim3(TILE_THREADS), sh,
                       s, J, maxc, nt, off, L, X, part);
  hipLaunchKernelGGL(k_trtri_finish<T>, dim3(max_nt - J), dim3(TILE_THREADS), sh, s, J, maxc, nt, off,
                     L, X, part);
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
  T* sB = sA + TS * LDS_S;
  const T* Xb = X + off[b] * TS2;
  TileAcc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  ra.load(Xb + tri_index(I, I) * TS2);
  rb.load(Xb + tri_index(I, J) * TS2);
  for (int K = I; K < ntb; ++K) {
    __syncthreads();
    ra.store_lds(sA);
    rb.store_lds(sB);
    __syncthreads();
    if (K + 1 < ntb) {
      ra.load(Xb + tri_index(K + 1, I) * TS2);
      rb.load(Xb + tri_index(K + 1, J) * TS2);
    }
    tile_mma<T, true, false>(acc, sA, sB, T(1));
  }
  acc.store(M + off[b] * TS2 + tri_index(I, J) * TS2);
}

template <typename T>
void launch_lauum(int nb, int max_nt, const int32_t* nt, const int64_t* off, const T* X, T* M,
                  hipStream_t s) {
  const size_t sh = 2 * TS * LDS_S * sizeof(T);
  static bool once = (allow_lds(k_lauum<T>, sh), true);
  (void)once;
  const int ntiles = max_nt * (max_nt + 1) / 2;
  hipLaunchKernelGGL(k_lauum<T>, dim3(ntiles, nb), dim3(TILE_THREADS), sh, s, nt, off, X, M);
}

#define INST(T)                                                                                    \
  template void launch_potrf_diag<T>(int, int, int, int, const T*, int, const int32_t*,            \
                                     const int64_t*, T*, int32_t*, hipStream_t);                   \
  template void launch_potrf_panel<T>(int, int, int, int, const T*, int, int, const int32_t*,      \
                                      const int64_t*, T*, hipStream_t);                            \
  template void launch_potrf_partial<T>(int, int, int, const int32_t*, const int64_t*, const T*,  \
                                        T*, hipStream_t);                                          \
  template void launch_trtri_splitk<T>(int, int, int, const int32_t*, const int64_t*, const T*,   \
                                       T*, T*, hipStream_t);                                       \
  template void launch_trtri_col<T>(int, int, int, const int32_t*, const int64_t*, const T*, T*,   \
                                    hipStream_t);                                                  \
  template void launch_lauum<T>(int, int, const int32_t*, const int64_t*, const T*, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace sfcdd
