// Subdomain solves of the fine Schwarz level: forward and backward
// substitution with the tiled Cholesky factors (tile envelopes in the local
// elimination order), one workgroup per subdomain.
#include "common.h"
#include "kernels.h"

namespace sfcdd {

// ---------------------------------------------------------------------------
// Subdomain solves d_i = A_i^{-1} R_i w by forward and backward substitution
// with the packed tiled Cholesky factor (Sec. 3.1: factor once, then only
// forward/backward steps; Alg. 2 first two steps).  One workgroup per
// subdomain; R_i w (a cyclic contiguous curve range, permuted to the local
// order) is staged in LDS.
// Diagonal tiles hold L_II^{-1}, so every step is a tile matrix-vector product.
// Each wave streams whole 16-byte-per-lane row groups of the tiles.

template <typename T>
__device__ __forceinline__ T dotv(const typename Vec16<T>::type& a, const T* b);
template <>
__device__ __forceinline__ float dotv<float>(const float4& a, const float* b) {
  const float4 y = *reinterpret_cast<const float4*>(b);
  return a.x * y.x + a.y * y.y + a.z * y.z + a.w * y.w;
}
template <>
__device__ __forceinline__ double dotv<double>(const double2& a, const double* b) {
  const double2 y = *reinterpret_cast<const double2*>(b);
  return a.x * y.x + a.y * y.y;
}
template <typename T>
__device__ __forceinline__ void axpyv(T* acc, const typename Vec16<T>::type& a, T s);
template <>
__device__ __forceinline__ void axpyv<float>(float* acc, const float4& a, float s) {
  acc[0] += a.x * s; acc[1] += a.y * s; acc[2] += a.z * s; acc[3] += a.w * s;
}
template <>
__device__ __forceinline__ void axpyv<double>(double* acc, const double2& a, double s) {
  acc[0] += a.x * s; acc[1] += a.y * s;
}

// A 16-byte load of factor data with the non-temporal hint.  Factors that
// stream through once per sweep (about 2 GB at the (7,6,5) workload, far
// beyond the caches) are read faster with it: a plain streaming read goes
// from about 6.4 to 7.1 TB/s.  Factors small enough to stay in the
// last-level cache between iterations are read faster without it.
template <typename T>
__device__ __forceinline__ typename Vec16<T>::type load_stream(const T* p);
template <>
__device__ __forceinline__ float4 load_stream<float>(const float* p) {
  typedef float E __attribute__((ext_vector_type(4)));
  const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  return make_float4(e.x, e.y, e.z, e.w);
}
template <>
__device__ __forceinline__ double2 load_stream<double>(const double* p) {
  typedef double E __attribute__((ext_vector_type(2)));
  const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  return make_double2(e.x, e.y);
}

template <typename T, bool NT>
__device__ __forceinline__ typename Vec16<T>::type load_fac(const T* p) {
  if (NT) return load_stream<T>(p);
  return *reinterpret_cast<const typename Vec16<T>::type*>(p);
}

template <typename T>
__device__ __forceinline__ typename Vec16<T>::type vzero();
template <>
__device__ __forceinline__ float4 vzero<float>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ __forceinline__ double2 vzero<double>() { return make_double2(0.0, 0.0); }

// The factor of subdomain b is stored as its tile envelope in the local
// elimination order: local row t is subdomain offset lperm[t], tile row I
// holds the tiles J = lo[I] .. I at rb[I] + J (lo non-decreasing), and every
// tile outside is zero.  So the forward step of row I reads the tiles lo[I]
// .. I, and the backward step of column I the tiles (K, I), K = I + 1 ..
// hi[I], hi[I] the last row whose envelope reaches column I.
// Each wave owns G row groups of every tile; the first PF tiles of the next
// row (column) and its diagonal tile are loaded into registers before the
// current one is reduced, so their latency overlaps the reductions and the
// barriers of the step.
// NT: factor loads with the non-temporal hint (chosen by the caller when the
// factors being swept are larger than the last-level cache).
template <typename T, int W, bool NT>
__global__ __launch_bounds__(W * 64) void k_schwarz_trsv(
    Batch B, const int32_t* __restrict__ ta, const int32_t* __restrict__ Ni,
    const int32_t* __restrict__ nt, const int64_t* __restrict__ off,
    const int64_t* __restrict__ doff, const int64_t* __restrict__ xoff, const int32_t* __restrict__ lperm,
    const int32_t* __restrict__ tlo, const int32_t* __restrict__ trb, const T* __restrict__ fac,
    const double* __restrict__ w, double* __restrict__ dbuf, const int32_t* __restrict__ active) {
  typedef typename Vec16<T>::type V;
  constexpr int VEC = Vec16<T>::n;          // elements per lane per load
  constexpr int LPR = TS / VEC;             // lanes per tile row
  constexpr int RPI = 64 / LPR;             // rows per wave load
  constexpr int NGRP = TS / RPI;            // row groups per tile
  constexpr int G = NGRP / W;               // row groups per wave
  constexpr int PF = G >= 8 ? 1 : 8 / G;    // prefetched tiles per row group
  const int b = blockIdx.x;
  const int ntb = nt[b], n = Ni[b];
  const int64_t t0 = ta[b];
  const int gi = grid_of(B, B.sgid, b);
  if (active && !act_updating(active[gi])) return;
  const GridDesc& g = B.grids[gi];
  const int64_t N = g.N;
  const double* __restrict__ wg = w + g.goff;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* y = reinterpret_cast<T*>(smem_raw);    // ntb * TS
  T* sS = y + ntb * TS;                     // TS
  T* red = sS + TS;                         // W * TS
  int* slo = reinterpret_cast<int*>(red + W * TS);  // ntb
  int* shi = slo + ntb;                     // ntb
  int* srb = shi + ntb;                     // ntb
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lrow = lane / LPR, c0 = (lane % LPR) * VEC;
  const T* F = fac + off[b] * TS2;
  const int64_t xb = xoff[b];
  const int32_t* __restrict__ perm = lperm + xb;

  for (int I = tid; I < ntb; I += W * 64) {
    slo[I] = tlo[xb / TS + I];
    srb[I] = trb[xb / TS + I];
  }
  for (int s = tid; s < ntb * TS; s += W * 64) {
    T v = T(0);
    if (s < n) {
      int64_t p = t0 + perm[s];
      if (p >= N) p -= N;
      v = (T)wg[p];
    }
    y[s] = v;
  }
  __syncthreads();
  for (int J = tid; J < ntb; J += W * 64) {
    int h = J;
    while (h + 1 < ntb && slo[h + 1] <= J) ++h;
    shi[J] = h;
  }
  __syncthreads();

  // Rows at or past n are padding (unit diagonal, zero right-hand side, zero
  // solution): their tile rows are never read.  Chunks of the diagonal-tile
  // inverses right of the diagonal are zero and not read either.
  V cur[G][PF + 1], nxt[G][PF + 1];
  auto load_fwd = [&](int I, V (&buf)[G][PF + 1]) {
    const int lo = slo[I];
    const T* rowI = F + (int64_t)srb[I] * TS2;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
      const bool live = I * TS + r < n;
#pragma unroll
      for (int k = 0; k < PF; ++k)
        buf[gg][k] = (live && lo + k < I) ? load_fac<T, NT>(rowI + (int64_t)(lo + k) * TS2 + r * TS + c0)
                                          : vzero<T>();
      buf[gg][PF] = (live && c0 <= r) ? load_fac<T, NT>(rowI + (int64_t)I * TS2 + r * TS + c0) : vzero<T>();
    }
  };
  auto load_bwd = [&](int I, V (&buf)[G][PF + 1]) {
    const int hi = shi[I];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int K = I + 1 + k;
        buf[gg][k] = (K <= hi && K * TS + r < n)
                         ? load_fac<T, NT>(F + ((int64_t)srb[K] + I) * TS2 + r * TS + c0)
                         : vzero<T>();
      }
      buf[gg][PF] = (c0 <= r && I * TS + r < n)
                        ? load_fac<T, NT>(F + ((int64_t)srb[I] + I) * TS2 + r * TS + c0)
                        : vzero<T>();
    }
  };
  auto advance = [&]() {
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int k = 0; k <= PF; ++k) cur[gg][k] = nxt[gg][k];
  };

  // forward: y_I <- L_II^{-1} (g_I - sum_{lo_I <= J < I} L_IJ y_J)
  load_fwd(0, cur);
  for (int I = 0; I < ntb; ++I) {
    if (I + 1 < ntb) load_fwd(I + 1, nxt);
    else load_bwd(ntb - 1, nxt);
    const int lo = slo[I];
    const T* rowI = F + (int64_t)srb[I] * TS2;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
      T acc = T(0);
      if (I * TS + r < n) {
#pragma unroll
        for (int k = 0; k < PF; ++k)
          if (lo + k < I) acc += dotv<T>(cur[gg][k], y + (lo + k) * TS + c0);
        for (int J = lo + PF; J < I; ++J) {
          const V v = load_fac<T, NT>(rowI + (int64_t)J * TS2 + r * TS + c0);
          acc += dotv<T>(v, y + J * TS + c0);
        }
      }
      for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((lane % LPR) == 0) sS[r] = y[I * TS + r] - acc;
    }
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
      T acc = T(0);
      if (c0 <= r && I * TS + r < n) acc = dotv<T>(cur[gg][PF], sS + c0);
      for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((lane % LPR) == 0) y[I * TS + r] = acc;
    }
    __syncthreads();
    advance();
  }

  // backward: x_I <- L_II^{-T} (y_I - sum_{I < K <= hi_I} L_KI^T x_K), x overwrites y
  for (int I = ntb - 1; I >= 0; --I) {
    if (I > 0) load_bwd(I - 1, nxt);
    const int hi = shi[I];
    T accv[VEC];
    for (int e = 0; e < VEC; ++e) accv[e] = T(0);
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int K = I + 1 + k;
        if (K <= hi && K * TS + r < n) axpyv<T>(accv, cur[gg][k], y[K * TS + r]);
      }
      for (int K = I + 1 + PF; K <= hi; ++K) {
        if (K * TS + r < n) {
          const V v = load_fac<T, NT>(F + ((int64_t)srb[K] + I) * TS2 + r * TS + c0);
          axpyv<T>(accv, v, y[K * TS + r]);
        }
      }
    }
    for (int e = 0; e < VEC; ++e)
      for (int o = LPR; o < 64; o <<= 1) accv[e] += __shfl_xor(accv[e], o, 64);
    if (lane < LPR)
      for (int e = 0; e < VEC; ++e) red[wv * TS + c0 + e] = accv[e];
    __syncthreads();
    if (tid < TS) {
      T s = y[I * TS + tid];
      for (int q = 0; q < W; ++q) s -= red[q * TS + tid];
      sS[tid] = s;
    }
    __syncthreads();
    for (int e = 0; e < VEC; ++e) accv[e] = T(0);
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
      if (c0 <= r && I * TS + r < n) axpyv<T>(accv, cur[gg][PF], sS[r]);
    }
    for (int e = 0; e < VEC; ++e)
      for (int o = LPR; o < 64; o <<= 1) accv[e] += __shfl_xor(accv[e], o, 64);
    if (lane < LPR)
      for (int e = 0; e < VEC; ++e) red[wv * TS + c0 + e] = accv[e];
    __syncthreads();
    if (tid < TS) {
      T s = T(0);
      for (int q = 0; q < W; ++q) s += red[q * TS + tid];
      y[I * TS + tid] = s;
    }
    __syncthreads();
    advance();
  }

  double* out = dbuf + doff[b];
  for (int s = tid; s < n; s += W * 64) out[perm[s]] = (double)y[s];
}

static size_t trsv_lds(int max_nt, size_t es, int W) {
  return ((size_t)max_nt * TS + TS + (size_t)W * TS) * es + 3 * (size_t)max_nt * sizeof(int);
}
bool trsv_fits(int max_nt, int elem_bytes, int waves) {
  return trsv_lds(max_nt, (size_t)elem_bytes, waves) <= (size_t)160 * 1024;
}

// Waves per workgroup of the substitution kernel: 4, 8 or 16 (a tuning knob).
template <typename T, int W, bool NT>
static void trsv_w(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                   const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                   const int32_t* tlo, const int32_t* trb, int max_nt, const T* fac,
                   const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  const size_t sh = trsv_lds(max_nt, sizeof(T), W);
  if (sh > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_schwarz_trsv<T, W, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((k_schwarz_trsv<T, W, NT>), dim3(B.Ptot), dim3(W * 64), sh, s, B, ta, Ni, nt, off,
                     doff, xoff, lperm, tlo, trb, fac, w, dbuf, active);
}

template <typename T, bool NT>
static void trsv_nt(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                    const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                    const int32_t* tlo, const int32_t* trb, int max_nt, int waves, const T* fac,
                    const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  while (waves > 4 && !trsv_fits(max_nt, (int)sizeof(T), waves)) waves /= 2;
  if (waves <= 4)
    trsv_w<T, 4, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, w, dbuf, active, s);
  else if (waves <= 8)
    trsv_w<T, 8, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, w, dbuf, active, s);
  else
    trsv_w<T, 16, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, w, dbuf, active, s);
}

template <typename T>
void launch_schwarz_trsv(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                         const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                         const int32_t* tlo, const int32_t* trb, int max_nt, int waves, bool stream,
                         const T* fac, const double* w, double* dbuf, const int32_t* active,
                         hipStream_t s) {
  if (stream)
    trsv_nt<T, true>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, waves, fac, w, dbuf, active, s);
  else
    trsv_nt<T, false>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, waves, fac, w, dbuf, active, s);
}

#define INST(T)                                                                                    \
  template void launch_schwarz_trsv<T>(const Batch&, const int32_t*, const int32_t*,              \
                                       const int32_t*, const int64_t*, const int64_t*,             \
                                       const int64_t*, const int32_t*, const int32_t*,             \
                                       const int32_t*, int, int, bool, const T*, const double*,    \
                                       double*, const int32_t*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace sfcdd
