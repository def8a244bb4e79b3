// Setup-phase kernels (Alg. 1): curve order, neighbour table, local and
// coarse assembly, for a batch of grids (one launch covers every grid).
#include "common.h"
#include "kernels.h"
#include "coarse_blocks.h"

namespace sfcdd {

// Number of k in [1, n] whose scaled coordinate k << s lies in [lo, hi].
__device__ __forceinline__ int64_t count_in(int64_t lo, int64_t hi, int n, int s) {
  int64_t a = (lo + ((int64_t)1 << s) - 1) >> s;  // ceil(lo / 2^s)
  int64_t b = hi >> s;                              // floor(hi / 2^s)
  if (a < 1) a = 1;
  if (b > n) b = n;
  return b >= a ? b - a + 1 : 0;
}

// Hilbert rank by Skilling's transform (transposed Hilbert index), one pass
// from the top bit level down.  At level lev the transform walks the axes: an
// axis i with a 1 at that level inverts the lower bits of axis 0, otherwise
// axes 0 and i exchange their lower bits.  Those operations reach only the
// levels below lev and depend only on bits at levels >= lev, so when level bi
// is reached the bits at bi already hold the transformed digit, and the same
// operations act on the bit-bi vector of every sibling cell (same bits above
// bi) as one affine map v[k] = c[perm[k]] ^ mask[k], built up level by level.
// The digit of a bit-bi vector: the axes Gray-coded in order (axis i XORed
// with the coded axis i - 1), inverted when the coded last axis has an odd
// number of ones above bi; axis 0 is its most significant bit.  At every
// level, the points of the sibling cells with a smaller digit come first;
// each cell is an axis-aligned box, so its interior points are counted as a
// product of interval counts.
__device__ int64_t hilbert_rank(const int64_t* C, const GridDesc& g) {
  const int d = g.d;
  uint64_t X[MAXD];
  int perm[MAXD], mask[MAXD];
  for (int j = 0; j < d; ++j) {
    X[j] = (uint64_t)C[j];
    perm[j] = j;
    mask[j] = 0;
  }
  int64_t rank = 0;
  for (int bi = g.nres - 1; bi >= 0; --bi) {
    uint64_t glast = 0;
    for (int i = 0; i < d; ++i) glast ^= X[i];
    const int flip = __popcll(glast >> (bi + 1)) & 1;
    int hp = 0, acc = 0;
    for (int i = 0; i < d; ++i) {
      acc ^= (int)((X[i] >> bi) & 1ull);
      hp = (hp << 1) | (acc ^ flip);
    }
    if (hp > 0) {
      for (int c = 0; c < (1 << d); ++c) {
        int dg = 0, ac = 0;
        for (int k = 0; k < d; ++k) {
          ac ^= ((c >> (d - 1 - perm[k])) & 1) ^ mask[k];
          dg = (dg << 1) | (ac ^ flip);
        }
        if (dg >= hp) continue;
        int64_t cnt = 1;
        for (int j = 0; j < d && cnt; ++j) {
          const int64_t lo = ((C[j] >> (bi + 1)) << (bi + 1)) | ((int64_t)((c >> (d - 1 - j)) & 1) << bi);
          cnt *= count_in(lo, lo + ((int64_t)1 << bi) - 1, g.n[j], g.shift[j]);
        }
        rank += cnt;
      }
    }
    if (bi > 0) {
      const uint64_t Q = 1ull << bi, low = Q - 1;
      for (int i = 0; i < d; ++i) {
        if (X[i] & Q) {
          X[0] ^= low;
          mask[0] ^= 1;
        } else {
          const uint64_t t = (X[0] ^ X[i]) & low;
          X[0] ^= t;
          X[i] ^= t;
          const int pt = perm[0], mt = mask[0];
          perm[0] = perm[i];
          mask[0] = mask[i];
          perm[i] = pt;
          mask[i] = mt;
        }
      }
    }
  }
  return rank;
}

// Curve rank of every point without sorting (Sec. 3.2/3.3, Alg. 1 sfc_index):
// the rank of key K is the number of grid points whose Morton key is smaller.
// Walking K's bits from the most significant one, each 1-bit contributes the
// points that share K's prefix above it and have a 0 there; on a tensor grid
// that count is a product over dimensions of interval counts, because a key
// prefix fixes the top bits of every scaled coordinate.
// Entry idx of grid g: natural index idx - goff; writes pos[idx] and
// sfc_index[goff + rank] as batch-global indices.
__global__ void k_sfc_rank(Batch B, int32_t* __restrict__ pos, int32_t* __restrict__ sfc_index) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B.Ntot) return;
  const GridDesc& g = B.grids[grid_of(B, B.gid, idx)];
  const int64_t nat = idx - g.goff;
  int64_t C[MAXD];
  for (int j = 0; j < g.d; ++j) {
    const int64_t k = (nat / g.stride[j]) % g.n[j] + 1;
    C[j] = k << g.shift[j];
  }
  int64_t rank = 0;
  if (g.curve == 1) {
    rank = hilbert_rank(C, g);
  } else {
  for (int t = g.nres - 1; t >= 0; --t) {
    for (int j = g.d - 1; j >= 0; --j) {
      if (!((C[j] >> t) & 1)) continue;
      int64_t cnt = 1;
      for (int jj = 0; jj < g.d && cnt; ++jj) {
        int64_t lo, hi;
        if (jj > j) {            // bit t already fixed at this level
          lo = (C[jj] >> t) << t;
          hi = lo + ((int64_t)1 << t) - 1;
        } else if (jj == j) {    // bits above t fixed, bit t = 0
          lo = (C[jj] >> (t + 1)) << (t + 1);
          hi = lo + ((int64_t)1 << t) - 1;
        } else {                 // bits above t fixed, bit t free
          lo = (C[jj] >> (t + 1)) << (t + 1);
          hi = lo + ((int64_t)1 << (t + 1)) - 1;
        }
        cnt *= count_in(lo, hi, g.n[jj], g.shift[jj]);
      }
      rank += cnt;
    }
  }
  }
  pos[idx] = (int32_t)(g.goff + rank);
  if (rank < g.N) sfc_index[g.goff + rank] = (int32_t)idx;
}

void launch_sfc_rank(const Batch& B, int32_t* pos, int32_t* sfc_index, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_sfc_rank, dim3((B.Ntot + th - 1) / th), dim3(th), 0, s, B, pos, sfc_index);
}

// Curve positions of the 2d stencil neighbours of every curve position
// (Alg. 1: map to neighbouring points), -1 on the Dirichlet boundary.
// Layout nbr[(2 j + side) * Ntot + p], side 0 = minus, 1 = plus; batch-global
// positions.
__global__ void k_build_nbr(Batch B, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ sfc_index, int32_t* __restrict__ nbr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.Ntot) return;
  const GridDesc& g = B.grids[grid_of(B, B.gid, p)];
  const int64_t nat = sfc_index[p];            // batch-global natural index
  const int64_t loc = nat - g.goff;
  for (int j = 0; j < B.dmax; ++j) {
    int32_t m = -1, q = -1;
    if (j < g.d) {
      const int64_t k = (loc / g.stride[j]) % g.n[j];
      if (k > 0) m = pos[nat - g.stride[j]];
      if (k < g.n[j] - 1) q = pos[nat + g.stride[j]];
    }
    nbr[(2 * j) * B.Ntot + p] = m;
    nbr[(2 * j + 1) * B.Ntot + p] = q;
  }
}

void launch_build_nbr(const Batch& B, const int32_t* pos, const int32_t* sfc_index, int32_t* nbr,
                      hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_build_nbr, dim3((B.Ntot + th - 1) / th), dim3(th), 0, s, B, pos, sfc_index,
                     nbr);
}

// Local matrices A_i = R_i A R_i^T (Sec. 3.1) in the local elimination
// order, written as the envelope tiles of the packed lower factor: local row
// t of subdomain b (grid g) is curve position (ta_b + lperm[t]) mod N of grid
// g, and tile (I, J), lo[I] <= J <= I, is tile off_b + rb[I] + J.  One
// workgroup per tile row: it clears the row's tiles (consecutive in memory)
// and then writes the diagonal and the stencil couplings left of it.  Rows
// past N_b are padding with a unit diagonal.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_local(Batch B, const int32_t* __restrict__ ta,
                                                        const int32_t* __restrict__ Ni,
                                                        const int32_t* __restrict__ nt,
                                                        const int64_t* __restrict__ fac_off,
                                                        const int64_t* __restrict__ xoff,
                                                        const int64_t* __restrict__ doff,
                                                        const int32_t* __restrict__ lperm,
                                                        const int32_t* __restrict__ liperm,
                                                        const int32_t* __restrict__ tlo,
                                                        const int32_t* __restrict__ trb,
                                                        const int32_t* __restrict__ nbr, T* __restrict__ fac) {
  const int b = blockIdx.y, I = blockIdx.x;
  const int ntb = nt[b];
  if (I >= ntb) return;
  const GridDesc& g = B.grids[grid_of(B, B.sgid, b)];
  const int64_t trow = xoff[b] / TS + I;
  const int lo = tlo[trow];
  const int64_t rb = trb[trow];
  T* F = fac + fac_off[b] * TS2;
  {
    typedef typename Vec16<T>::type V;
    constexpr int VEC = Vec16<T>::n;
    V* row = reinterpret_cast<V*>(F + (rb + lo) * TS2);
    const int64_t nv = (int64_t)(I - lo + 1) * TS2 / VEC;
    V z;
    if constexpr (VEC == 4) z = make_float4(0.f, 0.f, 0.f, 0.f);
    else z = make_double2(0.0, 0.0);
    for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) row[e] = z;
  }
  __syncthreads();
  const int r = threadIdx.x;
  if (r >= TS) return;
  const int t = I * TS + r;
  const int n = Ni[b];
  T* D = F + (rb + I) * TS2;
  if (t >= n) {
    D[r * TS + r] = T(1);
    return;
  }
  D[r * TS + r] = (T)g.diag;
  const int64_t t0 = ta[b];
  int64_t p = t0 + lperm[xoff[b] + t];
  if (p >= g.N) p -= g.N;
  p += g.goff;
  const int32_t* ip = liperm + doff[b];
  for (int j = 0; j < g.d; ++j) {
    for (int side = 0; side < 2; ++side) {
      const int64_t q = nbr[(2 * j + side) * B.Ntot + p];
      if (q < 0) continue;
      int64_t u = q - g.goff - t0;
      if (u < 0) u += g.N;
      if (u >= n) continue;
      const int tc = ip[u];
      if (tc < t) F[(rb + tc / TS) * TS2 + r * TS + tc % TS] = (T)(-g.c[j]);
    }
  }
}

template <typename T>
void launch_assemble_local(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                           const int64_t* fac_off, const int64_t* xoff, const int64_t* doff,
                           const int32_t* lperm, const int32_t* liperm, const int32_t* tlo, const int32_t* trb,
                           const int32_t* nbr, int max_nt, T* fac, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_local<T>, dim3(max_nt, B.Ptot), dim3(256), 0, s, B, ta, Ni, nt, fac_off, xoff,
                     doff, lperm, liperm, tlo, trb, nbr, fac);
}
#define INST(T)                                                                                         \
  template void launch_assemble_local<T>(const Batch&, const int32_t*, const int32_t*, const int32_t*, \
                                         const int64_t*, const int64_t*, const int64_t*, const int32_t*, \
                                         const int32_t*, const int32_t*, const int32_t*, const int32_t*, \
                                         int, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

// Position of a point's coarse block in its grid's dense coarse matrix: the
// permuted block (agg = 1), or its group of agg consecutive blocks (the
// Galerkin aggregation of A_0 that the iterative coarse solve uses as its
// second level, not permuted).
__device__ __forceinline__ int coarse_pos(const Batch& B, const GridDesc& g, int64_t q) {
  const int k = coarse_block(q - g.goff, g);
  return g.agg == 1 ? B.cperm[g.c0off + k] : k / g.agg;
}

// First nonzero column of every row of the dense coarse matrices: row I's
// cfnz[c0pad + I] is lowered to the smallest block coupled to it in any
// dimension (one atomic per point).
__global__ void k_coarse_fnz(Batch B, const int32_t* __restrict__ nbr, int32_t* __restrict__ cfnz) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.Ntot) return;
  const GridDesc& g = B.grids[grid_of(B, B.gid, p)];
  const int I = coarse_pos(B, g, p);
  int m = I;
  for (int j = 0; j < g.d; ++j)
    for (int side = 0; side < 2; ++side) {
      const int64_t q = nbr[(2 * j + side) * B.Ntot + p];
      if (q >= 0) m = min(m, coarse_pos(B, g, q));
    }
  if (m < I) atomicMin(&cfnz[g.c0pad + I], m);
}

void launch_coarse_fnz(const Batch& B, const int32_t* nbr, int32_t* cfnz, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_coarse_fnz, dim3((B.Ntot + th - 1) / th), dim3(th), 0, s, B, nbr, cfnz);
}

// Integer coupling counts of dimension j between coarse blocks (eq. csm with
// A = sum_j c_j L_j): cnt(I, J) = sum_{p in I, p' in J} (L_j)_{p p'} for
// J <= I, accumulated with integer atomics into the packed lower tiles of
// each grid's dense coarse matrix (first tile ctile_off[g]), in the permuted
// coarse numbering (block k at position cperm[k]).  Every count lies inside
// the envelope (k_coarse_fnz, k_coarse_env), whose tiles k_coarse_zero_env
// cleared.
__global__ void k_coarse_counts(Batch B, int j, const int32_t* __restrict__ nbr,
                                const int64_t* __restrict__ ctile_off, int32_t* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.Ntot) return;
  const int gi = grid_of(B, B.gid, p);
  const GridDesc& g = B.grids[gi];
  if (j >= g.d) return;
  int32_t* C = cnt + ctile_off[gi] * TS2;
  const int I = coarse_pos(B, g, p);
  atomicAdd(&C[tri_index(I / TS, I / TS) * TS2 + (I % TS) * TS + (I % TS)], 2);
  for (int side = 0; side < 2; ++side) {
    const int64_t q = nbr[(2 * j + side) * B.Ntot + p];
    if (q < 0) continue;
    const int J = coarse_pos(B, g, q);
    if (J > I) continue;
    atomicAdd(&C[tri_index(I / TS, J / TS) * TS2 + (I % TS) * TS + (J % TS)], -1);
  }
}

void launch_coarse_counts(const Batch& B, int j, const int32_t* nbr, const int64_t* ctile_off,
                          int32_t* cnt, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_coarse_counts, dim3((B.Ntot + th - 1) / th), dim3(th), 0, s, B, j, nbr,
                     ctile_off, cnt);
}

// Tile (I, J) = (blockIdx.x, blockIdx.y) of grid blockIdx.z when it lies inside
// the envelope of that grid's dense coarse matrix: its first element, else -1.
__device__ __forceinline__ int64_t env_tile(const Batch& B, const int64_t* __restrict__ off,
                                            const int32_t* __restrict__ clo, const GridDesc*& gp) {
  const GridDesc& g = B.grids[blockIdx.z];
  gp = &g;
  const int I = blockIdx.x, J = blockIdx.y;
  if (I >= g.nt0d || J > I || J < clo[g.c0pad / TS + I]) return -1;
  return (off[blockIdx.z] + tri_index(I, J)) * TS2;
}

// Zero the envelope tiles of the coarse matrices and of the count scratch.
__global__ __launch_bounds__(256) void k_coarse_zero_env(Batch B, const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ clo, double* __restrict__ A0,
                                                         int32_t* __restrict__ cnt) {
  const GridDesc* g;
  const int64_t t = env_tile(B, off, clo, g);
  if (t < 0) return;
  for (int e = 4 * threadIdx.x; e < TS2; e += 4 * 256) {
    *reinterpret_cast<double2*>(A0 + t + e) = make_double2(0.0, 0.0);
    *reinterpret_cast<double2*>(A0 + t + e + 2) = make_double2(0.0, 0.0);
    *reinterpret_cast<int4*>(cnt + t + e) = make_int4(0, 0, 0, 0);
  }
}

// A_0 += c_j E_j over the envelope tiles, clearing the counts for the next
// dimension (the sum over j runs in j order).
__global__ __launch_bounds__(256) void k_coarse_accumulate(Batch B, const int64_t* __restrict__ off,
                                                           const int32_t* __restrict__ clo, int j,
                                                           int32_t* __restrict__ cnt, double* __restrict__ A0) {
  const GridDesc* g;
  const int64_t t = env_tile(B, off, clo, g);
  if (t < 0 || j >= g->d) return;
  const double cj = g->c[j];
  for (int e = 4 * threadIdx.x; e < TS2; e += 4 * 256) {
    const int4 v = *reinterpret_cast<const int4*>(cnt + t + e);
    if (v.x | v.y | v.z | v.w) {
      double2 a = *reinterpret_cast<const double2*>(A0 + t + e);
      double2 b = *reinterpret_cast<const double2*>(A0 + t + e + 2);
      if (v.x) a.x += cj * (double)v.x;
      if (v.y) a.y += cj * (double)v.y;
      if (v.z) b.x += cj * (double)v.z;
      if (v.w) b.y += cj * (double)v.w;
      *reinterpret_cast<double2*>(A0 + t + e) = a;
      *reinterpret_cast<double2*>(A0 + t + e + 2) = b;
      *reinterpret_cast<int4*>(cnt + t + e) = make_int4(0, 0, 0, 0);
    }
  }
}

void launch_coarse_zero_env(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, double* A0,
                            int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_zero_env, dim3(max_nt0, max_nt0, B.G), dim3(256), 0, s, B, off, clo, A0, cnt);
}

void launch_coarse_accumulate(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, int j,
                              int32_t* cnt, double* A0, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_accumulate, dim3(max_nt0, max_nt0, B.G), dim3(256), 0, s, B, off, clo, j, cnt, A0);
}

// Rounds to FP32 the tiles inside the envelopes of the dense coarse matrices
// (packed triangles at off[g] tiles): the factorisation and the inversion
// read no other tile.  One workgroup per tile.
__global__ __launch_bounds__(256) void k_round_env(Batch B, const int64_t* __restrict__ off,
                                                   const int32_t* __restrict__ clo,
                                                   const double* __restrict__ src, float* __restrict__ dst) {
  const GridDesc* g;
  const int64_t t = env_tile(B, off, clo, g);
  if (t < 0) return;
  for (int e = 4 * threadIdx.x; e < TS2; e += 4 * 256) {
    const double2 a = *reinterpret_cast<const double2*>(src + t + e);
    const double2 b = *reinterpret_cast<const double2*>(src + t + e + 2);
    *reinterpret_cast<float4*>(dst + t + e) = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
  }
}

void launch_round_env(const Batch& B, int max_nt0, const int64_t* off, const int32_t* clo, const double* src,
                      float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_round_env, dim3(max_nt0, max_nt0, B.G), dim3(256), 0, s, B, off, clo, src, dst);
}

// Unit diagonal on the padding rows N0 .. nt0*TS-1 of each coarse matrix.
__global__ void k_coarse_pad(Batch B, const int64_t* __restrict__ ctile_off, double* __restrict__ A0) {
  const int gi = blockIdx.y;
  const GridDesc& g = B.grids[gi];
  const int r = g.N0d + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.nt0d * TS) return;
  const int I = r / TS;
  A0[(ctile_off[gi] + tri_index(I, I)) * TS2 + (r % TS) * TS + (r % TS)] = 1.0;
}

void launch_coarse_pad(const Batch& B, int max_nt0, const int64_t* ctile_off, double* A0,
                       hipStream_t s) {
  (void)max_nt0;
  hipLaunchKernelGGL(k_coarse_pad, dim3(1, B.G), dim3(64), 0, s, B, ctile_off, A0);
}

}  // namespace sfcdd
