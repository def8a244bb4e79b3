// Coarse blocks of eq. restr: piece i (a contiguous curve range of
// floor(N/P) or floor(N/P) + 1 points, eq. sloc) is cut into q consecutive
// blocks, the first (size mod q) of them one point longer; block m of piece i
// is coarse unknown i q + m.
#pragma once
#include "common.h"
#include "kernels.h"

namespace sfcdd {

// Coarse unknown whose block contains curve position p (grid-local).
__device__ __forceinline__ int coarse_block(int64_t p, const GridDesc& g) {
  const int i = piece_of(p, g.base, g.rem);
  const int64_t o = p - piece_start(i, g.base, g.rem);
  const int64_t sz = g.base + (i < g.rem ? 1 : 0);
  const int64_t qb = sz / g.q, qr = sz % g.q;
  const int64_t big = qr * (qb + 1);
  const int m = o < big ? (int)(o / (qb + 1)) : (int)(qr + (o - big) / qb);
  return i * g.q + m;
}

// First curve position and size of the block of coarse unknown I.
__device__ __forceinline__ void block_range(int I, const GridDesc& g, int64_t* start, int64_t* size) {
  const int i = I / g.q, m = I % g.q;
  const int64_t sz = g.base + (i < g.rem ? 1 : 0);
  const int64_t qb = sz / g.q, qr = sz % g.q;
  *start = piece_start(i, g.base, g.rem) + (m < qr ? m * (qb + 1) : qr * (qb + 1) + (m - qr) * qb);
  *size = qb + (m < qr ? 1 : 0);
}

}  // namespace sfcdd
