// Iterative solve of the coarse system A_0 d = c of one grid, for coarse
// spaces too large for a dense factor (the four-levels-coarser rule of
// Sec. 4.1 with many subdomains; the paper leaves the parallel coarse solve
// to future work).  A_0 = R_0 A R_0^T (eq. csm) is kept sparse, one row per
// coarse block, and solved by CG in FP64 preconditioned with a two-level
// additive operator of its own:
//  - exact solves with the 64 x 64 diagonal blocks of A_0 (64 consecutive
//    coarse unknowns along the curve, kept as their explicit FP32 inverses);
//  - a dense correction on the Galerkin aggregation of A_0 over the same
//    groups of 64 (a dense factor and inverse, as for a small coarse space).
// The CG scalars stay on the device: every workgroup that needs a step size
// sums the same partials in the same order, a flag stops the iteration once
// the residual is below tolerance, and later launches of the solve return at
// once.  No atomics on floating point values: results are reproducible.
#include "common.h"
#include "kernels.h"
#include "coarse_blocks.h"

namespace sfcdd {

constexpr int ELL_SLOTS = 512;  // LDS hash slots (distinct neighbour blocks) per coarse row

// Row I of A_0 in ELL form (entry k of row I at k * ld + I): the coarse blocks
// J that the points of block I couple to, and I itself, in increasing J, each
// with value sum_j c_j n_j(I, J) over j in order, where n_j are the integer
// coupling counts of the dense coarse matrix: n_j(I, I) = 2 |I| minus the
// ordered neighbour pairs in dimension j inside I, n_j(I, J) = minus the
// pairs (p, p') with p in I, p' in J, p' = p +- e_j.  Rows with more than kw
// entries, or more distinct neighbours than the table holds, set status.
// One workgroup per coarse block.
__global__ __launch_bounds__(256) void k_coarse_ell(Batch B, const int32_t* __restrict__ nbr, int kw,
                                                    int64_t ld, int32_t* __restrict__ deg,
                                                    int32_t* __restrict__ col, double* __restrict__ val,
                                                    int32_t* __restrict__ status) {
  __shared__ int32_t key[ELL_SLOTS];
  __shared__ int32_t cnt[MAXD * ELL_SLOTS];  // cnt[j * ELL_SLOTS + slot]
  __shared__ int32_t nused, lost;
  const GridDesc& g = B.grids[0];
  const int I = blockIdx.x;
  const int d = g.d;
  for (int e = threadIdx.x; e < ELL_SLOTS; e += blockDim.x) {
    key[e] = -1;
    for (int j = 0; j < d; ++j) cnt[j * ELL_SLOTS + e] = 0;
  }
  if (threadIdx.x == 0) {
    nused = 0;
    lost = 0;
  }
  __syncthreads();
  int64_t st, sz;
  block_range(I, g, &st, &sz);
  // open addressing with linear probing; at most ELL_SLOTS probes
  auto slot_of = [&](int J) -> int {
    unsigned h = ((unsigned)J * 2654435761u) & (ELL_SLOTS - 1);
    for (int t = 0; t < ELL_SLOTS; ++t) {
      const int prev = atomicCAS(&key[h], -1, J);
      if (prev == -1 || prev == J) return (int)h;
      h = (h + 1) & (ELL_SLOTS - 1);
    }
    return -1;
  };
  if (threadIdx.x == 0) {
    const int s = slot_of(I);  // the table is empty: always found
    for (int j = 0; j < d; ++j) cnt[j * ELL_SLOTS + s] = 2 * (int)sz;
  }
  __syncthreads();
  const int64_t nops = sz * 2 * d;
  for (int64_t e = threadIdx.x; e < nops; e += blockDim.x) {
    const int64_t p = st + e / (2 * d);
    const int k = (int)(e % (2 * d));  // neighbour plane 2 j + side
    const int32_t q = nbr[(int64_t)k * B.Ntot + g.goff + p];
    if (q < 0) continue;
    const int J = coarse_block(q - g.goff, g);
    const int s = slot_of(J);
    if (s < 0) {
      atomicOr(&lost, 1);
      continue;
    }
    atomicSub(&cnt[(k >> 1) * ELL_SLOTS + s], 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ELL_SLOTS; e += blockDim.x) {
    const int J = key[e];
    if (J < 0) continue;
    int r = 0;
    for (int f = 0; f < ELL_SLOTS; ++f) {
      const int K = key[f];
      r += (K >= 0 && K < J) ? 1 : 0;
    }
    atomicAdd(&nused, 1);
    if (r < kw) {
      double v = 0.0;
      for (int j = 0; j < d; ++j) {
        const int n = cnt[j * ELL_SLOTS + e];
        if (n) v += g.c[j] * (double)n;
      }
      col[(int64_t)r * ld + I] = J;
      val[(int64_t)r * ld + I] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    deg[I] = nused < kw ? nused : kw;
    if (nused > kw || lost) atomicOr(status, 1);
  }
}

void launch_coarse_ell(const Batch& B, int64_t n0, const int32_t* nbr, int kw, int64_t ld, int32_t* deg,
                       int32_t* col, double* val, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_ell, dim3((unsigned)n0), dim3(256), 0, s, B, nbr, kw, ld, deg, col, val, status);
}

// The diagonal 64 x 64 blocks of A_0 (coarse unknowns 64 t .. 64 t + 63) as
// dense row-major tiles (zeroed beforehand); rows past n0 get a unit diagonal.
__global__ void k_bj_extract(int64_t n0, int64_t ld, const int32_t* __restrict__ deg,
                             const int32_t* __restrict__ col, const double* __restrict__ val,
                             double* __restrict__ tiles) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= ld) return;
  const int64_t t = I / TS;
  double* row = tiles + t * TS2 + (I % TS) * TS;
  if (I >= n0) {
    row[I % TS] = 1.0;
    return;
  }
  const int n = deg[I];
  for (int k = 0; k < n; ++k) {
    const int J = col[(int64_t)k * ld + I];
    if (J / TS == t) row[J % TS] = val[(int64_t)k * ld + I];
  }
}

void launch_bj_extract(int64_t n0, int64_t ld, const int32_t* deg, const int32_t* col, const double* val,
                       double* tiles, hipStream_t s) {
  hipLaunchKernelGGL(k_bj_extract, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, s, n0, ld, deg, col, val,
                     tiles);
}

// M = X^T X for each tile X = L^{-1} (lower, row-major): the explicit inverse
// of the diagonal block, full and symmetric (M_ij and M_ji are the same sum
// in the same order), rounded to FP32.
__global__ __launch_bounds__(256) void k_bj_form(const double* __restrict__ X, float* __restrict__ M) {
  __shared__ double sx[TS * (TS + 1)];
  const double* Xt = X + (int64_t)blockIdx.x * TS2;
  for (int e = threadIdx.x; e < TS2; e += blockDim.x) sx[(e / TS) * (TS + 1) + e % TS] = Xt[e];
  __syncthreads();
  float* Mt = M + (int64_t)blockIdx.x * TS2;
  for (int e = threadIdx.x; e < TS2; e += blockDim.x) {
    const int i = e / TS, j = e % TS;
    double s = 0.0;
    for (int k = i > j ? i : j; k < TS; ++k) s += sx[k * (TS + 1) + i] * sx[k * (TS + 1) + j];
    Mt[e] = (float)s;
  }
}

void launch_bj_form(int ntiles, const double* X, float* M, hipStream_t s) {
  hipLaunchKernelGGL(k_bj_form, dim3(ntiles), dim3(256), 0, s, X, M);
}

// ---------------------------------------------------------------------------
// Inner CG.  Vectors have ld = nt0 * 64 entries (coarse unknowns padded to
// whole 64-blocks; the padding stays zero in r, p and z).  Scalars: sc[IC_*];
// flag: ACT_RUN while iterating, ACT_DONE once converged (or when the outer
// grid is not updating).

// Starts a solve: the flag from the outer grid's state, the iteration count.
__global__ void k_ic_begin(const int32_t* __restrict__ outer, int32_t* __restrict__ flag, double* __restrict__ sc) {
  if (threadIdx.x == 0) {
    *flag = (outer && !act_updating(outer[0])) ? ACT_DONE : ACT_RUN;
    sc[IC_ITS] = 0.0;
    sc[IC_CONV] = 0.0;
  }
}

// q = A_0 p (ELL), per-block partials of p . q.
__global__ __launch_bounds__(256) void k_ic_spmv(int64_t ld, const int32_t* __restrict__ deg,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ p, double* __restrict__ q,
                                                 double* __restrict__ part, const int32_t* __restrict__ flag) {
  if (*flag != ACT_RUN) return;
  __shared__ double sh[16];
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (I < ld) {
    const int n = deg[I];
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += val[(int64_t)k * ld + I] * p[col[(int64_t)k * ld + I]];
    q[I] = s;
    acc = p[I] * s;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Sum of n partials in a fixed order, returned to every thread of the block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* sh) {
  double a = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) a += part[e];
  a = block_sum(a, sh);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = a;
  __syncthreads();
  return bc;
}

// One workgroup per 64-block t.  first: x = 0, r = b.  Otherwise the CG step
// x += alpha p, r -= alpha q with alpha = rz / (p . q) (rz in sc[IC_RZ +
// (it - 1) % 2], p . q from the SpMV's nq partials).  Then the block solve
// z1 = M_t r_t, the aggregate c_t = sum of r over the block, and the
// partials rr_t = r_t . r_t, zr_t = z1_t . r_t.
__global__ __launch_bounds__(256) void k_ic_update(int first, int it, int64_t n0, int nq,
                                                   const double* __restrict__ qpart, const double* __restrict__ sc,
                                                   const double* __restrict__ b, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ p,
                                                   const double* __restrict__ q, const float* __restrict__ M,
                                                   double* __restrict__ z1, double* __restrict__ cagg,
                                                   double* __restrict__ part, const int32_t* __restrict__ flag) {
  if (*flag != ACT_RUN) return;
  __shared__ double sh[16];
  __shared__ double sr[TS];
  const int t = blockIdx.x;
  const int64_t I0 = (int64_t)t * TS;
  double alpha = 0.0;
  if (!first) alpha = sc[IC_RZ + ((it - 1) & 1)] / sum_partials(qpart, nq, sh);
  if (threadIdx.x < TS) {
    const int64_t I = I0 + threadIdx.x;
    double rv;
    if (first) {
      rv = I < n0 ? b[I] : 0.0;
      x[I] = 0.0;
    } else {
      x[I] += alpha * p[I];
      rv = r[I] - alpha * q[I];
    }
    r[I] = rv;
    sr[threadIdx.x] = rv;
  }
  __syncthreads();
  // z1 = M_t r_t: four lanes per row, 16 columns each
  const int row = threadIdx.x >> 2, qd = threadIdx.x & 3;
  const float* Mr = M + (int64_t)t * TS2 + row * TS + qd * 16;
  double zs = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) zs += (double)Mr[k] * sr[qd * 16 + k];
  zs += __shfl_xor(zs, 1, 64);
  zs += __shfl_xor(zs, 2, 64);
  if (qd == 0) z1[I0 + row] = zs;
  const double rv = qd == 0 ? sr[row] : 0.0;
  const double rr = block_sum(rv * rv, sh);
  const double zr = block_sum(qd == 0 ? zs * sr[row] : 0.0, sh);
  const double cs = block_sum(rv, sh);
  if (threadIdx.x == 0) {
    part[2 * t] = rr;
    part[2 * t + 1] = zr;
    cagg[t] = cs;
  }
}

// Direction update, one workgroup per `per` 64-blocks: rz = sum zr_t +
// d . c over the aggregates (d = A_agg^{-1} c, the second level),
// z = z1 + d[t], p = z (first) or z + (rz / rz_old) p.  Convergence:
// sum rr_t <= tol2 * (sum rr_t at the start); block 0 records the scalars and
// raises the flag.
__global__ __launch_bounds__(256) void k_ic_dir(int first, int it, int64_t n0, int nt, int per, double tol2,
                                                const double* __restrict__ part, const double* __restrict__ cagg,
                                                const double* __restrict__ dagg, double* __restrict__ sc,
                                                const double* __restrict__ z1, double* __restrict__ p,
                                                int32_t* __restrict__ flag) {
  if (*flag != ACT_RUN) return;
  __shared__ double sh[16];
  double a = 0.0, bz = 0.0, dc = 0.0;
  for (int e = threadIdx.x; e < nt; e += blockDim.x) {
    a += part[2 * e];
    bz += part[2 * e + 1];
    dc += dagg[e] * cagg[e];
  }
  a = block_sum(a, sh);
  bz = block_sum(bz, sh);
  dc = block_sum(dc, sh);
  __shared__ double bc[3];
  if (threadIdx.x == 0) {
    bc[0] = a;
    bc[1] = bz + dc;
  }
  __syncthreads();
  const double rr = bc[0], rz = bc[1];
  const double rr0 = first ? rr : sc[IC_RR0];
  const bool conv = rr <= tol2 * rr0;
  const double beta = first ? 0.0 : rz / sc[IC_RZ + ((it - 1) & 1)];
  const int t0 = blockIdx.x * per;
  for (int e = threadIdx.x; e < per * TS; e += blockDim.x) {
    const int t = t0 + e / TS;
    if (t >= nt) break;
    const int64_t I = (int64_t)t * TS + e % TS;
    const double z = I < n0 ? z1[I] + dagg[t] : 0.0;
    p[I] = first ? z : z + beta * p[I];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (first) sc[IC_RR0] = rr;
    sc[IC_RZ + (it & 1)] = rz;
    sc[IC_ITS] = (double)it;
    if (conv) {
      sc[IC_CONV] = 1.0;
      *flag = ACT_DONE;
    }
  }
}

// Right-hand side of the trial solve that sizes the inner step budget: a
// fixed pseudo-random vector (an integer hash of the index, values in
// [-1, 1)) on the coarse unknowns, zero on the padding.
__global__ void k_ic_trial(int64_t n0, int64_t ld, double* __restrict__ b) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= ld) return;
  if (I >= n0) {
    b[I] = 0.0;
    return;
  }
  uint64_t z = (uint64_t)I * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
  z = (z ^ (z >> 33)) * 0xFF51AFD7ED558CCDull;
  z = (z ^ (z >> 33)) * 0xC4CEB9FE1A85EC53ull;
  z ^= z >> 33;
  b[I] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

void launch_ic_trial(int64_t n0, int64_t ld, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_ic_trial, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, s, n0, ld, b);
}

void launch_ic_begin(const int32_t* outer, int32_t* flag, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_ic_begin, dim3(1), dim3(64), 0, s, outer, flag, sc);
}

void launch_ic_spmv(int64_t ld, const int32_t* deg, const int32_t* col, const double* val, const double* p,
                    double* q, double* part, const int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ic_spmv, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, s, ld, deg, col, val, p, q,
                     part, flag);
}

void launch_ic_update(int first, int it, int64_t n0, int nt, int nq, const double* qpart, const double* sc,
                      const double* b, double* x, double* r, const double* p, const double* q, const float* M,
                      double* z1, double* cagg, double* part, const int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ic_update, dim3(nt), dim3(256), 0, s, first, it, n0, nq, qpart, sc, b, x, r, p, q, M, z1,
                     cagg, part, flag);
}

void launch_ic_dir(int first, int it, int64_t n0, int nt, double tol2, const double* part, const double* cagg,
                   const double* dagg, double* sc, const double* z1, double* p, int32_t* flag, hipStream_t s) {
  constexpr int PER = 16;
  hipLaunchKernelGGL(k_ic_dir, dim3((nt + PER - 1) / PER), dim3(256), 0, s, first, it, n0, nt, PER, tol2, part,
                     cagg, dagg, sc, z1, p, flag);
}

}  // namespace sfcdd
