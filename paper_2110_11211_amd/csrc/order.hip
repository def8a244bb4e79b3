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

namespace sfcdd {

constexpr int ORDER_THREADS = 256;
constexpr int ORDER_MAX_PATTERNS = 64;

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
    Batch B, int mode, int kcap, const int32_t* __restrict__ ta, const int32_t* __restrict__ Ni,
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
  extern __shared__ int hist[];         // kcap level counters, then ntb tile-row minima
  int* tmin = hist + kcap;

  // a subdomain of one tile row has nothing to gain from reordering
  bool diag = mode == 2 && g.d >= 2 && ntb > 1;
  if (diag) {
    if (tid < g.d) {
      bmin[tid] = INT32_MAX;
      bmax[tid] = -1;
    }
    __syncthreads();
    for (int s = tid; s < n; s += ORDER_THREADS) {
      const int nat = (int)(sfc_index[sub_pos(g, t0, s)] - g.goff);
      for (int j = 0; j < g.d; ++j) {
        const int x = nat / (int)g.stride[j] % g.n[j];
        atomicMin(&bmin[j], x);
        atomicMax(&bmax[j], x);
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

void launch_local_order(const Batch& B, int mode, int kcap, int max_nt, const int32_t* ta, const int32_t* Ni,
                        const int32_t* nt, const int64_t* xoff, const int64_t* doff, const int32_t* sfc_index,
                        const int32_t* nbr, int32_t* lperm, int32_t* liperm, int32_t* tlo, int32_t* trb,
                        unsigned long long* gtiles, hipStream_t s) {
  const size_t sh = ((size_t)kcap + (size_t)max_nt) * sizeof(int);
  if (sh > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_local_order),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_local_order, dim3(B.Ptot), dim3(ORDER_THREADS), sh, s, B, mode, kcap, ta, Ni, nt, xoff, doff,
                     sfc_index, nbr, lperm, liperm, tlo, trb, gtiles);
}

}  // namespace sfcdd
