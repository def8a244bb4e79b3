// Local elimination order and tile envelope of the subdomain matrices.
//
// The subdomain problems are solved directly: factor once, then forward and
// backward substitution (Sec. 3.1).  Any symmetric reordering of A_i gives
// the same A_i^{-1}, and the Cholesky factor of a matrix has no entries left
// of the first nonzero of each row of its lower triangle (the envelope is
// preserved by the elimination).  Ordering the points of a subdomain by
// level sets of a coordinate diagonal keeps the first nonzero of every row
// close to the diagonal, so only a narrow band of the 64 x 64 tiles of the
// factor is ever stored, factored or streamed.
//
// One workgroup per subdomain:
//  1. coordinates of its points (curve position -> natural index), bounding
//     box;
//  2. the key sum_j s_j (x_j - box_j), s_j = +-1 (s_0 = +1), for each sign
//     pattern (at most 64); the pattern whose largest key level holds the
//     fewest points wins (first pattern on ties);
//  3. stable counting sort of the points by that key (ties in curve order):
//     lperm[t] = subdomain offset of local row t, liperm the inverse;
//  4. first nonzero column of every local row from the stencil neighbours,
//     the first tile column lo[I] of every tile row (made non-decreasing),
//     and the packed row bases rb[I]: tile (I, J), lo[I] <= J <= I, is tile
//     rb[I] + J of the subdomain's factor; gtiles[3 g .. 3 g + 2] of its grid
//     g accumulate the tiles stored, the factor entries one substitution
//     sweep reads (the off-diagonal tiles and the lower triangles of the
//     diagonal tiles, padding rows excluded) and the tile products of the
//     factorisation.
// mode 0 keeps the curve order and every tile (lo = 0: the packed triangle),
// mode 1 the curve order with its envelope, mode 2 the diagonal order with
// its envelope (curve order when d = 1, for subdomains of one tile row, or
// when the key range exceeds kcap).
#include "common.h"
#include "kernels.h"
#include "coarse_blocks.h"

namespace sfcdd {

constexpr int ORDER_THREADS = 256;
constexpr size_t ORDER_LDS_BYTES = 144 * 1024;   // dynamic LDS the ordering kernels may take
constexpr int ORDER_MAX_PATTERNS = 64;

// Ascending sort of the np (a power of two) values at srt by the whole
// workgroup (bitonic network; np / 2 compare-exchanges per stage).
__device__ void bitonic_sort(uint32_t* srt, int np) {
  for (int k = 2; k <= np; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const uint32_t a = srt[i], b = srt[l];
          if ((a > b) == ((i & k) == 0)) {
            srt[i] = b;
            srt[l] = a;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Bits of an index below np (a power of two).
__device__ __forceinline__ int index_bits(int np) { return 31 - __clz(np); }

__device__ __forceinline__ int64_t sub_pos(const GridDesc& g, int64_t t0, int s) {
  int64_t p = t0 + s;
  if (p >= g.N) p -= g.N;
  return g.goff + p;
}

// Key of offset s under sign pattern sg (bit j - 1 set: s_j = -1).
__device__ __forceinline__ int order_key(const GridDesc& g, int nat, const int* bmin, const int* bmax,
                                         int sg) {
  int key = 0;
  for (int j = 0; j < g.d; ++j) {
    const int x = nat / (int)g.stride[j] % g.n[j];
    key += (j > 0 && ((sg >> (j - 1)) & 1)) ? bmax[j] - x : x - bmin[j];
  }
  return key;
}

__global__ __launch_bounds__(ORDER_THREADS) void k_local_order(
    Batch B, int mode, int kcap, int npmax, const int32_t* __restrict__ ta, const int32_t* __restrict__ Ni,
    const int32_t* __restrict__ nt, const int64_t* __restrict__ xoff, const int64_t* __restrict__ doff,
    const int32_t* __restrict__ sfc_index, const int32_t* __restrict__ nbr, int32_t* __restrict__ lperm,
    int32_t* __restrict__ liperm, int32_t* __restrict__ tlo, int32_t* __restrict__ trb,
    unsigned long long* __restrict__ gtiles) {
  const int b = blockIdx.x;
  const int gi = grid_of(B, B.sgid, b);
  const GridDesc& g = B.grids[gi];
  const int n = Ni[b], ntb = nt[b];
  const int64_t t0 = ta[b];
  const int64_t rbase = xoff[b];        // first local row in the row tables
  const int64_t trow = rbase / TS;      // first tile row
  int32_t* perm = lperm + rbase;
  int32_t* iperm = liperm + doff[b];
  const int tid = threadIdx.x, lane = tid & 63;
  __shared__ int bmin[MAXD], bmax[MAXD];
  __shared__ int s_best, s_bestw, s_range, s_red[ORDER_THREADS / 64];
  extern __shared__ int hist[];         // kcap level counters, npmax sort keys, ntb tile-row minima
  uint32_t* srt = reinterpret_cast<uint32_t*>(hist + kcap);
  int* tmin = reinterpret_cast<int*>(srt + npmax);

  // a subdomain of one tile row has nothing to gain from reordering
  bool diag = mode == 2 && g.d >= 2 && ntb > 1;
  if (diag) {
    if (tid < g.d) {
      bmin[tid] = INT32_MAX;
      bmax[tid] = -1;
    }
    __syncthreads();
    for (int j = 0; j < g.d; ++j) {
      int lo = INT32_MAX, hi = -1;
      for (int s = tid; s < n; s += ORDER_THREADS) {
        const int x = (int)(sfc_index[sub_pos(g, t0, s)] - g.goff) / (int)g.stride[j] % g.n[j];
        lo = min(lo, x);
        hi = max(hi, x);
      }
      lo = wave_min(lo);
      hi = wave_max(hi);
      if (lane == 0) {
        atomicMin(&bmin[j], lo);
        atomicMax(&bmax[j], hi);
      }
    }
    __syncthreads();
    if (tid == 0) {
      int r = 1;
      for (int j = 0; j < g.d; ++j) r += bmax[j] - bmin[j];
      s_range = r;
      s_best = 0;
      s_bestw = INT32_MAX;
    }
    __syncthreads();
    diag = s_range <= kcap;
  }
  if (diag) {
    const int R = s_range;
    const int npat = g.d - 1 >= 6 ? ORDER_MAX_PATTERNS : 1 << (g.d - 1);
    // the sign pattern with the narrowest widest level
    for (int sg = 0; sg < npat; ++sg) {
      for (int k = tid; k < R; k += ORDER_THREADS) hist[k] = 0;
      __syncthreads();
      for (int s = tid; s < n; s += ORDER_THREADS)
        atomicAdd(&hist[order_key(g, (int)(sfc_index[sub_pos(g, t0, s)] - g.goff), bmin, bmax, sg)], 1);
      __syncthreads();
      int m = 0;
      for (int k = tid; k < R; k += ORDER_THREADS) m = max(m, hist[k]);
      for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
      if (lane == 0) s_red[tid >> 6] = m;
      __syncthreads();
      if (tid == 0) {
        int w = 0;
        for (int q = 0; q < ORDER_THREADS / 64; ++q) w = max(w, s_red[q]);
        if (w < s_bestw) {
          s_bestw = w;
          s_best = sg;
        }
      }
      __syncthreads();
    }
    const int sg = s_best;
    if (npmax > 0) {
      // sort of the unique values key << IB | s: by key, ties in curve order
      int np = 1;
      while (np < n) np <<= 1;
      const int IB = index_bits(np);
      for (int s = tid; s < np; s += ORDER_THREADS)
        srt[s] = s < n ? ((uint32_t)order_key(g, (int)(sfc_index[sub_pos(g, t0, s)] - g.goff), bmin, bmax, sg) << IB) |
                             (uint32_t)s
                       : 0xFFFFFFFFu;
      __syncthreads();
      bitonic_sort(srt, np);
      for (int t = tid; t < n; t += ORDER_THREADS) {
        const int s = (int)(srt[t] & ((1u << IB) - 1u));
        perm[t] = s;
        iperm[s] = t;
      }
    } else {
    for (int k = tid; k < R; k += ORDER_THREADS) hist[k] = 0;
    __syncthreads();
    for (int s = tid; s < n; s += ORDER_THREADS)
      atomicAdd(&hist[order_key(g, (int)(sfc_index[sub_pos(g, t0, s)] - g.goff), bmin, bmax, sg)], 1);
    __syncthreads();
    // exclusive scan of the level sizes: the first row of every level
    if (tid == 0) {
      int run = 0;
      for (int k = 0; k < R; ++k) {
        const int c = hist[k];
        hist[k] = run;
        run += c;
      }
    }
    __syncthreads();
    // stable placement, 64 offsets at a time by the first wave: the lanes of
    // one key take consecutive rows in lane order
    if (tid < 64) {
      for (int s0 = 0; s0 < n; s0 += 64) {
        const int s = s0 + lane;
        const bool v = s < n;
        const int key = v ? order_key(g, (int)(sfc_index[sub_pos(g, t0, s)] - g.goff), bmin, bmax, sg) : -1;
        uint64_t rem = __ballot(v);
        int t = 0;
        while (rem) {
          const int leader = __ffsll((unsigned long long)rem) - 1;
          const int kk = __shfl(key, leader, 64);
          const uint64_t m = __ballot(v && key == kk);
          if (v && key == kk) t = hist[kk] + __popcll(m & ((1ull << lane) - 1ull));
          if (lane == leader) hist[kk] += __popcll(m);
          rem &= ~m;
        }
        if (v) {
          perm[t] = s;
          iperm[s] = t;
        }
      }
    }
    }
  } else {
    for (int s = tid; s < n; s += ORDER_THREADS) {
      perm[s] = s;
      iperm[s] = s;
    }
  }
  for (int t = n + tid; t < ntb * TS; t += ORDER_THREADS) perm[t] = -1;
  // the stores of perm / iperm are read below by other threads of this workgroup
  __syncthreads();

  // first tile column of every tile row
  for (int I = tid; I < ntb; I += ORDER_THREADS) tmin[I] = mode == 0 ? 0 : I;
  __syncthreads();
  if (mode != 0) {
    for (int t = tid; t < n; t += ORDER_THREADS) {
      const int64_t p = sub_pos(g, t0, perm[t]);
      int f = t;
      for (int j = 0; j < g.d; ++j)
        for (int side = 0; side < 2; ++side) {
          const int64_t q = nbr[(2 * j + side) * B.Ntot + p];
          if (q < 0) continue;
          int64_t u = q - g.goff - t0;
          if (u < 0) u += g.N;
          if (u < n) f = min(f, iperm[u]);
        }
      atomicMin(&tmin[t / TS], f / TS);
    }
    __syncthreads();
  }
  if (tid == 0) {
    // non-decreasing lo (a row may reach no further left than the rows below
    // it), then the packed row bases
    int lo = ntb;
    for (int I = ntb - 1; I >= 0; --I) {
      lo = min(lo, tmin[I]);
      tmin[I] = lo;
    }
    int64_t start = 0, entries = 0, products = 0;
    for (int I = 0; I < ntb; ++I) {
      tlo[trow + I] = tmin[I];
      trb[trow + I] = (int32_t)(start - tmin[I]);
      start += I - tmin[I] + 1;
      const int64_t rows = min(TS, n - I * TS);   // rows of the tile row that are not padding
      entries += rows * TS * (I - tmin[I]) + rows * (rows + 1) / 2;
      // tile products of the left-looking factorisation: the diagonal tile
      // takes I - lo[I] updates; a tile (I, J) takes J - lo[I] updates and
      // the product with L_JJ^{-T}
      products += I - tmin[I];
      for (int J = tmin[I]; J < I; ++J) products += J - tmin[I] + 1;
    }
    atomicAdd(&gtiles[3 * gi], (unsigned long long)start);
    atomicAdd(&gtiles[3 * gi + 1], (unsigned long long)entries);
    atomicAdd(&gtiles[3 * gi + 2], (unsigned long long)products);
  }
}

// Elimination order of the dense coarse matrices (agg = 1; the iterative
// coarse solve's aggregated level keeps its order).  A_0 couples the coarse
// blocks of neighbouring curve segments; in block (curve) order its
// Cholesky factor is nearly full, while ordered by level sets of a
// coordinate diagonal of the blocks' centroids it is banded (at the (7,6,5)
// workload about a fifth of the 64 x 64 tiles), which shortens the
// factorisation's columns and the inversion's sums.  The centroids (4 x the
// mean coordinate, rounded) come from k_coarse_centroid; then one workgroup
// per grid: sign pattern
// with the narrowest widest level (as for the subdomains), stable counting
// sort of the blocks by key (ties in block order).  cperm[c0off + k] = the
// position of block k; cfnz[c0pad + r] = r for every row of the padded
// matrix (the first-nonzero columns k_coarse_counts lowers).  Keys spanning
// more than kcap levels keep the block order.
// 4 x the mean coordinate of every coarse block (rounded), for all blocks of
// the batch: ccen[Ig * dmax + j].
__global__ void k_coarse_centroid(Batch B, const int32_t* __restrict__ sfc_index, int32_t* __restrict__ ccen) {
  const int64_t Ig = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (Ig >= B.N0tot) return;
  const GridDesc& g = B.grids[grid_of(B, B.cgid, Ig)];
  int64_t st, sz;
  block_range((int)(Ig - g.c0off), g, &st, &sz);
  int64_t sum[MAXD];
  for (int j = 0; j < g.d; ++j) sum[j] = 0;
  for (int64_t e = 0; e < sz; ++e) {
    const int nat = (int)(sfc_index[g.goff + st + e] - g.goff);
    for (int j = 0; j < g.d; ++j) sum[j] += nat / (int)g.stride[j] % g.n[j];
  }
  for (int j = 0; j < g.d; ++j) ccen[Ig * B.dmax + j] = (int32_t)((4 * sum[j] + sz / 2) / sz);
}

__device__ __forceinline__ int centroid_key(const GridDesc& g, const int32_t* __restrict__ cen, const int* cmin,
                                            const int* cmax, int sg) {
  int key = 0;
  for (int j = 0; j < g.d; ++j) {
    const int c = cen[j];
    key += (j > 0 && ((sg >> (j - 1)) & 1)) ? cmax[j] - c : c - cmin[j];
  }
  return key;
}

constexpr int CORDER_THREADS = 1024;
__global__ __launch_bounds__(CORDER_THREADS) void k_coarse_order(Batch B, int kcap, int npmax, int hcap,
                                                                const int32_t* __restrict__ ccen,
                                                                int32_t* __restrict__ cperm,
                                                                int32_t* __restrict__ cfnz) {
  const GridDesc& g = B.grids[blockIdx.x];
  const int n = g.N0, tid = threadIdx.x, lane = tid & 63;
  int32_t* perm = cperm + g.c0off;
  for (int r = tid; r < g.nt0d * TS; r += CORDER_THREADS) cfnz[g.c0pad + r] = r;
  __shared__ int cmin[MAXD], cmax[MAXD];
  __shared__ int s_best, s_bestw, s_range, s_red[CORDER_THREADS / 64];
  extern __shared__ int hist[];
  bool diag = g.agg == 1 && g.d >= 2 && g.nt0d > 1;
  if (diag) {
    if (tid < g.d) {
      cmin[tid] = INT32_MAX;
      cmax[tid] = -1;
    }
    __syncthreads();
    for (int j = 0; j < g.d; ++j) {
      int lo = INT32_MAX, hi = -1;
      for (int k = tid; k < n; k += CORDER_THREADS) {
        const int c = ccen[(g.c0off + k) * B.dmax + j];
        lo = min(lo, c);
        hi = max(hi, c);
      }
      lo = wave_min(lo);
      hi = wave_max(hi);
      if (lane == 0) {
        atomicMin(&cmin[j], lo);
        atomicMax(&cmax[j], hi);
      }
    }
    __syncthreads();
    if (tid == 0) {
      int r = 1;
      for (int j = 0; j < g.d; ++j) r += cmax[j] - cmin[j];
      s_range = r;
      s_best = 0;
      s_bestw = INT32_MAX;
    }
    __syncthreads();
    diag = s_range <= kcap;
  }
  if (!diag) {
    for (int k = tid; k < n; k += CORDER_THREADS) perm[k] = k;
    return;
  }
  const int R = s_range;
  const int npat = g.d - 1 >= 6 ? ORDER_MAX_PATTERNS : 1 << (g.d - 1);
  if (npat * R <= hcap) {
    // every pattern's level sizes in one pass over the blocks
    for (int k = tid; k < npat * R; k += CORDER_THREADS) hist[k] = 0;
    __syncthreads();
    for (int k = tid; k < n; k += CORDER_THREADS)
      for (int sg = 0; sg < npat; ++sg)
        atomicAdd(&hist[sg * R + centroid_key(g, ccen + (g.c0off + k) * B.dmax, cmin, cmax, sg)], 1);
    __syncthreads();
    for (int sg = 0; sg < npat; ++sg) {
      int m = 0;
      for (int k = tid; k < R; k += CORDER_THREADS) m = max(m, hist[sg * R + k]);
      m = wave_max(m);
      if (lane == 0) s_red[tid >> 6] = m;
      __syncthreads();
      if (tid == 0) {
        int w = 0;
        for (int q = 0; q < CORDER_THREADS / 64; ++q) w = max(w, s_red[q]);
        if (w < s_bestw) {
          s_bestw = w;
          s_best = sg;
        }
      }
      __syncthreads();
    }
  } else
  for (int sg = 0; sg < npat; ++sg) {
    for (int k = tid; k < R; k += CORDER_THREADS) hist[k] = 0;
    __syncthreads();
    for (int k = tid; k < n; k += CORDER_THREADS) atomicAdd(&hist[centroid_key(g, ccen + (g.c0off + k) * B.dmax, cmin, cmax, sg)], 1);
    __syncthreads();
    int m = 0;
    for (int k = tid; k < R; k += CORDER_THREADS) m = max(m, hist[k]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if (lane == 0) s_red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      int w = 0;
      for (int q = 0; q < CORDER_THREADS / 64; ++q) w = max(w, s_red[q]);
      if (w < s_bestw) {
        s_bestw = w;
        s_best = sg;
      }
    }
    __syncthreads();
  }
  const int sg = s_best;
  if (npmax >= n) {
    // sort of the unique values key << IB | k: by key, ties in block order
    uint32_t* srt = reinterpret_cast<uint32_t*>(hist + hcap);
    int np = 1;
    while (np < n) np <<= 1;
    const int IB = index_bits(np);
    for (int k = tid; k < np; k += CORDER_THREADS)
      srt[k] = k < n ? ((uint32_t)centroid_key(g, ccen + (g.c0off + k) * B.dmax, cmin, cmax, sg) << IB) | (uint32_t)k
                     : 0xFFFFFFFFu;
    __syncthreads();
    bitonic_sort(srt, np);
    for (int t = tid; t < n; t += CORDER_THREADS) perm[srt[t] & ((1u << IB) - 1u)] = t;
    return;
  }
  for (int k = tid; k < R; k += CORDER_THREADS) hist[k] = 0;
  __syncthreads();
  for (int k = tid; k < n; k += CORDER_THREADS) atomicAdd(&hist[centroid_key(g, ccen + (g.c0off + k) * B.dmax, cmin, cmax, sg)], 1);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int k = 0; k < R; ++k) {
      const int c = hist[k];
      hist[k] = run;
      run += c;
    }
  }
  __syncthreads();
  if (tid < 64) {
    for (int k0 = 0; k0 < n; k0 += 64) {
      const int k = k0 + lane;
      const bool v = k < n;
      const int key = v ? centroid_key(g, ccen + (g.c0off + k) * B.dmax, cmin, cmax, sg) : -1;
      uint64_t rem = __ballot(v);
      int t = 0;
      while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int kk = __shfl(key, leader, 64);
        const uint64_t mk = __ballot(v && key == kk);
        if (v && key == kk) t = hist[kk] + __popcll(mk & ((1ull << lane) - 1ull));
        if (lane == leader) hist[kk] += __popcll(mk);
        rem &= ~mk;
      }
      if (v) perm[k] = t;
    }
  }
}

void launch_coarse_order(const Batch& B, int kcap, int max_n0, const int32_t* sfc_index, int32_t* ccen,
                         int32_t* cperm, int32_t* cfnz, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_centroid, dim3((unsigned)((B.N0tot + 255) / 256)), dim3(256), 0, s, B, sfc_index, ccen);
  // sort keys in LDS when they fit (else the wave-serial placement)
  int npmax = 1;
  while (npmax < max_n0) npmax <<= 1;
  if (((size_t)kcap + (size_t)npmax) * sizeof(int) > ORDER_LDS_BYTES) npmax = 0;
  // level counters: every sign pattern at once when they fit beside the sort keys
  const int npat = B.dmax - 1 >= 6 ? ORDER_MAX_PATTERNS : 1 << (B.dmax > 0 ? B.dmax - 1 : 0);
  int hcap = kcap;
  if (((size_t)npat * kcap + (size_t)npmax) * sizeof(int) <= ORDER_LDS_BYTES) hcap = npat * kcap;
  const size_t sh = ((size_t)hcap + (size_t)npmax) * sizeof(int);
  if (sh > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_coarse_order),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_coarse_order, dim3(B.G), dim3(CORDER_THREADS), sh, s, B, kcap, npmax, hcap, ccen, cperm,
                     cfnz);
}

// First tile column of every tile row of the (permuted) dense coarse
// matrices from the rows' first nonzero columns, made non-decreasing, and the
// row bases of the packed triangle (the matrices stay stored as full packed
// triangles; only the factorisation and inversion skip the zero tiles).  One
// workgroup per grid.  With the one-level dissection of a single grid (nd =
// {ta, tb, ts}, ts > 0: tile rows [0, ta) of the first half, [ta, ta + tb) of
// the second, the separator after them) lo is non-decreasing within each of
// the three parts only: the rows of the second half start right of the first
// half, which the separator's rows reach.  wide = the largest I - lo[I] over
// the rows whose inverse rows the column steps form (all rows, or the two
// halves with the dissection).
__global__ __launch_bounds__(ORDER_THREADS) void k_coarse_env(Batch B, const int32_t* __restrict__ cfnz,
                                                              int32_t* __restrict__ clo,
                                                              int32_t* __restrict__ crb,
                                                              int32_t* __restrict__ wide,
                                                              const int32_t* __restrict__ nd) {
  const GridDesc& g = B.grids[blockIdx.x];
  const int nt = g.nt0d;
  const int64_t trow = g.c0pad / TS;
  extern __shared__ int tmin[];
  for (int I = threadIdx.x; I < nt; I += ORDER_THREADS) tmin[I] = I;
  __syncthreads();
  for (int r = threadIdx.x; r < nt * TS; r += ORDER_THREADS) atomicMin(&tmin[r / TS], cfnz[g.c0pad + r] / TS);
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool split = nd && nd[2] > 0;
    const int ta = split ? nd[0] : 0, tab = split ? nd[0] + nd[1] : nt;
    int lo = nt, w = 0;
    for (int I = nt - 1; I >= 0; --I) {
      if (split && (I == tab - 1 || I == ta - 1)) lo = nt;   // the part below is another one
      lo = min(lo, tmin[I]);
      clo[trow + I] = lo;
      crb[trow + I] = I * (I + 1) / 2;
      if (I < tab) w = max(w, I - lo);
    }
    if (wide && blockIdx.x == 0) wide[0] = w;
  }
}

void launch_coarse_env(const Batch& B, int max_nt0, const int32_t* cfnz, int32_t* clo, int32_t* crb,
                       int32_t* wide, const int32_t* nd, hipStream_t s) {
  const size_t sh = (size_t)max_nt0 * sizeof(int);
  hipLaunchKernelGGL(k_coarse_env, dim3(B.G), dim3(ORDER_THREADS), sh, s, B, cfnz, clo, crb, wide, nd);
}

// ---------------------------------------------------------------------------
// One-level nested dissection of a single grid's coarse matrix.
//
// The coarse blocks of the first half of the curve (block index < N0 / 2) and
// those of the second half couple only through the blocks of the first half
// that have a stencil neighbour in the second (the separator).  The curve's
// midpoint splits the grid along a plane (both curves halve the bounding
// box there); a split elsewhere leaves a ragged interface and a larger
// separator, so the first half's chain is the shorter one.  Ordered as
// [first half | second half | separator], the Cholesky factor has no tiles
// coupling the halves, so the two halves factor as independent chains of
// column steps, and the separator's rows follow: about half the dependent
// steps of one chain over the whole matrix.  X_0 = L_0^{-1} keeps the block
// structure (no tiles in the rows of the second half left of it), so the
// coarse solves read only the nonzero tiles.  Within each part the blocks
// keep the centroid-diagonal order.  The halves are trimmed to whole tiles:
// the blocks past the last whole tile of a half go to the separator.

// sep[k] = 1 for every block k of the first half with a neighbour in the
// second (sep cleared beforehand).  Every writer stores the same value.
__global__ __launch_bounds__(256) void k_nd_mark(Batch B, const int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ sep) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= B.Ntot) return;
  const GridDesc& g = B.grids[0];
  const int half = g.N0 / 2;
  const int k = coarse_block(p - g.goff, g);
  if (k >= half) return;
  for (int j = 0; j < g.d; ++j)
    for (int side = 0; side < 2; ++side) {
      const int64_t q = nbr[(2 * j + side) * B.Ntot + p];
      if (q >= 0 && coarse_block(q - g.goff, g) >= half) {
        sep[k] = 1;
        return;
      }
    }
}

// The dissected order from the centroid-diagonal one (cperm): each part in
// that order, the halves' remainders (past their last whole tile) ahead of
// the separator's own blocks.  nd = {ta, tb, ts} tiles of the two halves and
// the separator, or {0, 0, 0} (order unchanged) unless both halves have at
// least two tiles and the separator at most an eighth of the tile rows.
// backup[k] keeps the previous position of block k.  One workgroup; LDS:
// the inverse permutation (N0 ints).
constexpr int ND_THREADS = 1024;
__global__ __launch_bounds__(ND_THREADS) void k_nd_order(Batch B, int32_t* __restrict__ cperm,
                                                         const int32_t* __restrict__ sep,
                                                         int32_t* __restrict__ backup, int32_t* __restrict__ nd) {
  const GridDesc& g = B.grids[0];
  const int n0 = g.N0, nt = g.nt0d, half = n0 / 2;
  extern __shared__ int inv[];
  __shared__ int wsum[3][ND_THREADS / 64 + 1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int k = t; k < n0; k += ND_THREADS) inv[cperm[g.c0off + k]] = k;
  __syncthreads();
  auto part = [&](int k) { return sep[k] ? 2 : (k < half ? 0 : 1); };
  const int seg = (n0 + ND_THREADS - 1) / ND_THREADS;
  const int p0 = min(n0, t * seg), p1 = min(n0, p0 + seg);
  int c[3] = {0, 0, 0};
  for (int pos = p0; pos < p1; ++pos) ++c[part(inv[pos])];
  // exclusive prefix of the segment counts over the threads (wave scans,
  // then the wave totals)
  int x[3];
  for (int q = 0; q < 3; ++q) {
    int v = c[q];
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o, 64);
      if (lane >= o) v += u;
    }
    x[q] = v - c[q];
    if (lane == 63) wsum[q][wv + 1] = v;
  }
  __syncthreads();
  if (t < 3) {
    wsum[t][0] = 0;
    for (int u = 1; u <= ND_THREADS / 64; ++u) wsum[t][u] += wsum[t][u - 1];
  }
  __syncthreads();
  for (int q = 0; q < 3; ++q) x[q] += wsum[q][wv];
  const int na = wsum[0][ND_THREADS / 64], nb = wsum[1][ND_THREADS / 64];
  const int ta = na / TS, tb = nb / TS, ra = na % TS, rb = nb % TS;
  const int ts = nt - ta - tb;
  const bool ok = ta >= 2 && tb >= 2 && ts >= 1 && 8 * ts <= nt;
  if (t == 0) {
    nd[0] = ok ? ta : 0;
    nd[1] = ok ? tb : 0;
    nd[2] = ok ? ts : 0;
  }
  if (!ok) return;
  const int sa = TS * ta, sb = TS * tb, s0 = sa + sb;
  int r[3] = {x[0], x[1], x[2]};
  for (int pos = p0; pos < p1; ++pos) {
    const int k = inv[pos];
    const int q = part(k);
    const int rk = r[q]++;
    int np;
    if (q == 0) np = rk < sa ? rk : s0 + (rk - sa);
    else if (q == 1) np = rk < sb ? sa + rk : s0 + ra + (rk - sb);
    else np = s0 + ra + rb + rk;
    backup[k] = pos;
    cperm[g.c0off + k] = np;
  }
}

// Back to the order before the dissection (its halves' envelopes turned out
// too wide for the inverse rows beside the column steps), with the
// first-nonzero columns reset for k_coarse_fnz.
__global__ __launch_bounds__(256) void k_nd_undo(Batch B, const int32_t* __restrict__ backup,
                                                 int32_t* __restrict__ cperm, int32_t* __restrict__ cfnz,
                                                 int32_t* __restrict__ nd) {
  const GridDesc& g = B.grids[0];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < g.N0) cperm[g.c0off + i] = backup[i];
  if (i < g.nt0d * TS) cfnz[g.c0pad + i] = i;
  if (i < 3) nd[i] = 0;
}

void launch_nd_order(const Batch& B, const int32_t* nbr, int32_t* sep, int32_t* backup, int32_t* cperm,
                     int32_t* nd, int n0, hipStream_t s) {
  hipLaunchKernelGGL(k_nd_mark, dim3((unsigned)((B.Ntot + 255) / 256)), dim3(256), 0, s, B, nbr, sep);
  const size_t sh = (size_t)n0 * sizeof(int);
  if (sh > 32768)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_nd_order),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_nd_order, dim3(1), dim3(ND_THREADS), sh, s, B, cperm, sep, backup, nd);
}

void launch_nd_undo(const Batch& B, const int32_t* backup, int32_t* cperm, int32_t* cfnz, int32_t* nd,
                    int nrows, hipStream_t s) {
  hipLaunchKernelGGL(k_nd_undo, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s, B, backup, cperm, cfnz, nd);
}

// Row tables of the three chains of a dissected coarse matrix (views): view 0
// the first half's tile rows then the separator's, view 1 the second half's
// then the separator's, view 2 the separator's alone.  Per view v:
// vinfo[3 v ..] = {rows, columns factored by its chain, first tile column},
// vinfo[9] = ta + tb,
// and for its local tile row i: vlo[v * stride + i] = first local tile column
// (the separator's own chain treats its block as dense), vrb[v * stride + i]
// = packed index of global tile (row, first column), so that local tile
// (i, j) is packed tile vrb[i] + j.
__global__ __launch_bounds__(256) void k_nd_views(const int32_t* __restrict__ nd, const int32_t* __restrict__ clo,
                                                  int stride, int32_t* __restrict__ vinfo,
                                                  int32_t* __restrict__ vlo, int32_t* __restrict__ vrb) {
  const int ta = nd[0], tb = nd[1], ts = nd[2], s0 = ta + tb;
  if (threadIdx.x == 0) {
    vinfo[0] = ta + ts; vinfo[1] = ta; vinfo[2] = 0;
    vinfo[3] = tb + ts; vinfo[4] = tb; vinfo[5] = ta;
    vinfo[6] = ts;      vinfo[7] = ts; vinfo[8] = s0;
    vinfo[9] = s0;      // columns of the two halves
  }
  for (int i = threadIdx.x; i < ta + ts; i += 256) {
    const int I = i < ta ? i : s0 + (i - ta);
    vlo[i] = clo[I];
    vrb[i] = I * (I + 1) / 2;
  }
  for (int i = threadIdx.x; i < tb + ts; i += 256) {
    const int I = i < tb ? ta + i : s0 + (i - tb);
    vlo[stride + i] = max(clo[I] - ta, 0);
    vrb[stride + i] = I * (I + 1) / 2 + ta;
  }
  for (int i = threadIdx.x; i < ts; i += 256) {
    const int I = s0 + i;
    vlo[2 * stride + i] = 0;
    vrb[2 * stride + i] = I * (I + 1) / 2 + s0;
  }
}

void launch_nd_views(const int32_t* nd, const int32_t* clo, int stride, int32_t* vinfo, int32_t* vlo, int32_t* vrb,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_nd_views, dim3(1), dim3(256), 0, s, nd, clo, stride, vinfo, vlo, vrb);
}

void launch_local_order(const Batch& B, int mode, int kcap, int max_nt, const int32_t* ta, const int32_t* Ni,
                        const int32_t* nt, const int64_t* xoff, const int64_t* doff, const int32_t* sfc_index,
                        const int32_t* nbr, int32_t* lperm, int32_t* liperm, int32_t* tlo, int32_t* trb,
                        unsigned long long* gtiles, hipStream_t s) {
  // sort keys in LDS when they fit (else the wave-serial placement)
  int npmax = 1;
  while (npmax < max_nt * TS) npmax <<= 1;
  if (((size_t)kcap + (size_t)npmax + (size_t)max_nt) * sizeof(int) > ORDER_LDS_BYTES) npmax = 0;
  const size_t sh = ((size_t)kcap + (size_t)npmax + (size_t)max_nt) * sizeof(int);
  if (sh > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_local_order),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_local_order, dim3(B.Ptot), dim3(ORDER_THREADS), sh, s, B, mode, kcap, npmax, ta, Ni, nt, xoff,
                     doff, sfc_index, nbr, lperm, liperm, tlo, trb, gtiles);
}

}  // namespace sfcdd
