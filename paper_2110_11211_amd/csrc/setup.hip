// Setup-phase kernels (Alg. 1): curve order, neighbour table, local and
// coarse assembly.
#include "common.h"
#include "kernels.h"

namespace sfcdd {

// Number of k in [1, n] whose scaled coordinate k << s lies in [lo, hi].
__device__ __forceinline__ int64_t count_in(int64_t lo, int64_t hi, int n, int s) {
  int64_t a = (lo + ((int64_t)1 << s) - 1) >> s;  // ceil(lo / 2^s)
  int64_t b = hi >> s;                              // floor(hi / 2^s)
  if (a < 1) a = 1;
  if (b > n) b = n;
  return b >= a ? b - a + 1 : 0;
}

// Curve rank of every point without sorting (Sec. 3.2/3.3, Alg. 1 sfc_index):
// the rank of key K is the number of grid points whose Morton key is smaller.
// Walking K's bits from the most significant one, each 1-bit contributes the
// points that share K's prefix above it and have a 0 there; on a tensor grid
// that count is a product over dimensions of interval counts, because a key
// prefix fixes the top bits of every scaled coordinate.
__global__ void k_sfc_rank(GridDesc g, int32_t* __restrict__ pos, int32_t* __restrict__ sfc_index) {
  const int64_t nat = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (nat >= g.N) return;
  int64_t C[MAXD];
  for (int j = 0; j < g.d; ++j) {
    const int64_t k = (nat / g.stride[j]) % g.n[j] + 1;
    C[j] = k << g.shift[j];
  }
  int64_t rank = 0;
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
  pos[nat] = (int32_t)rank;
  if (rank < g.N) sfc_index[rank] = (int32_t)nat;
}

void launch_sfc_rank(const GridDesc& g, int32_t* pos, int32_t* sfc_index, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_sfc_rank, dim3((g.N + th - 1) / th), dim3(th), 0, s, g, pos, sfc_index);
}

// Curve positions of the 2d stencil neighbours of every curve position
// (Alg. 1: map to neighbouring points), -1 on the Dirichlet boundary.
// Layout nbr[(2 j + side) * N + p], side 0 = minus, 1 = plus.
__global__ void k_build_nbr(GridDesc g, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ sfc_index, int32_t* __restrict__ nbr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.N) return;
  const int64_t nat = sfc_index[p];
  for (int j = 0; j < g.d; ++j) {
    const int64_t k = (nat / g.stride[j]) % g.n[j];
    nbr[(2 * j) * g.N + p] = k > 0 ? pos[nat - g.stride[j]] : -1;
    nbr[(2 * j + 1) * g.N + p] = k < g.n[j] - 1 ? pos[nat + g.stride[j]] : -1;
  }
}

void launch_build_nbr(const GridDesc& g, const int32_t* pos, const int32_t* sfc_index,
                      int32_t* nbr, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_build_nbr, dim3((g.N + th - 1) / th), dim3(th), 0, s, g, pos, sfc_index, nbr);
}

// Local matrices A_i = R_i A R_i^T (Sec. 3.1) written as packed lower tiles:
// row s of subdomain b is curve position (ta_b + s) mod N.  Rows past N_b are
// padding with a unit diagonal.  The tiles must be zeroed beforehand.
template <typename T>
__global__ void k_assemble_local(GridDesc g, const int32_t* __restrict__ ta,
                                 const int32_t* __restrict__ Ni, const int32_t* __restrict__ nt,
                                 const int64_t* __restrict__ fac_off,
                                 const int32_t* __restrict__ nbr, T* __restrict__ fac) {
  const int b = blockIdx.y;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int ntb = nt[b];
  if (s >= ntb * TS) return;
  T* F = fac + fac_off[b] * TS2;
  const int I = s / TS, r = s % TS;
  const int n = Ni[b];
  if (s >= n) {
    F[tri_index(I, I) * TS2 + r * TS + r] = T(1);
    return;
  }
  F[tri_index(I, I) * TS2 + r * TS + r] = (T)g.diag;
  const int64_t p = ((int64_t)ta[b] + s) % g.N;
  for (int j = 0; j < g.d; ++j) {
    for (int side = 0; side < 2; ++side) {
      const int64_t q = nbr[(2 * j + side) * g.N + p];
      if (q < 0) continue;
      const int64_t t = ((q - ta[b]) % g.N + g.N) % g.N;
      if (t < n && t < s) {
        const int J = (int)(t / TS), c = (int)(t % TS);
        F[tri_index(I, J) * TS2 + r * TS + c] = (T)(-g.c[j]);
      }
    }
  }
}

template <typename T>
void launch_assemble_local(const GridDesc& g, int P, const int32_t* ta, const int32_t* Ni,
                           const int32_t* nt, const int64_t* fac_off, const int32_t* nbr,
                           int max_nt, T* fac, hipStream_t s) {
  const int th = 256;
  dim3 grid((max_nt * TS + th - 1) / th, P);
  hipLaunchKernelGGL(k_assemble_local<T>, grid, dim3(th), 0, s, g, ta, Ni, nt, fac_off, nbr, fac);
}
template void launch_assemble_local<float>(const GridDesc&, int, const int32_t*, const int32_t*,
                                           const int32_t*, const int64_t*, const int32_t*, int,
                                           float*, hipStream_t);
template void launch_assemble_local<double>(const GridDesc&, int, const int32_t*, const int32_t*,
                                            const int32_t*, const int64_t*, const int32_t*, int,
                                            double*, hipStream_t);

// Coarse unknown (block) of curve position p: piece i and its m-th block of
// eq. (restr), index i q + m.
__device__ __forceinline__ int coarse_block(int64_t p, const PartDesc& pd) {
  const int i = piece_of(p, pd.base, pd.rem);
  const int64_t o = p - piece_start(i, pd.base, pd.rem);
  const int64_t sz = pd.base + (i < pd.rem ? 1 : 0);
  const int64_t qb = sz / pd.q, qr = sz % pd.q;
  const int64_t big = qr * (qb + 1);
  const int m = o < big ? (int)(o / (qb + 1)) : (int)(qr + (o - big) / qb);
  return i * pd.q + m;
}

// Integer coupling counts of dimension j between coarse blocks (eq. csm with
// A = sum_j c_j L_j): cnt(I, J) = sum_{p in I, p' in J} (L_j)_{p p'} for
// J <= I, accumulated with integer atomics into packed lower tiles.
__global__ void k_coarse_counts(GridDesc g, PartDesc pd, int j, const int32_t* __restrict__ nbr,
                                int32_t* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.N) return;
  const int I = coarse_block(p, pd);
  atomicAdd(&cnt[tri_index(I / TS, I / TS) * TS2 + (I % TS) * TS + (I % TS)], 2);
  for (int side = 0; side < 2; ++side) {
    const int64_t q = nbr[(2 * j + side) * g.N + p];
    if (q < 0) continue;
    const int J = coarse_block(q, pd);
    if (J > I) continue;
    atomicAdd(&cnt[tri_index(I / TS, J / TS) * TS2 + (I % TS) * TS + (J % TS)], -1);
  }
}

void launch_coarse_counts(const GridDesc& g, const PartDesc& pd, int j, const int32_t* nbr,
                          int32_t* cnt, hipStream_t s) {
  const int th = 256;
  hipLaunchKernelGGL(k_coarse_counts, dim3((g.N + th - 1) / th), dim3(th), 0, s, g, pd, j, nbr, cnt);
}

__global__ void k_coarse_accumulate(int64_t n, double cj, const int32_t* __restrict__ cnt,
                                    double* __restrict__ A0) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = cnt[e];
    if (v) A0[e] += cj * (double)v;
  }
}

void launch_coarse_accumulate(int64_t n, double cj, const int32_t* cnt, double* A0, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_accumulate, dim3(2048), dim3(256), 0, s, n, cj, cnt, A0);
}

// Unit diagonal on the padding rows N0 .. nt0*TS-1 of the coarse matrix.
__global__ void k_coarse_pad(int N0, int nt0, double* __restrict__ A0) {
  const int r = N0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nt0 * TS) return;
  const int I = r / TS;
  A0[tri_index(I, I) * TS2 + (r % TS) * TS + (r % TS)] = 1.0;
}

void launch_coarse_pad(int N0, int nt0, double* A0, hipStream_t s) {
  const int pad = nt0 * TS - N0;
  if (pad <= 0) return;
  hipLaunchKernelGGL(k_coarse_pad, dim3((pad + 63) / 64), dim3(64), 0, s, N0, nt0, A0);
}

}  // namespace sfcdd
