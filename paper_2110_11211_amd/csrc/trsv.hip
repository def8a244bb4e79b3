// Subdomain solves of the fine Schwarz level: forward and backward
// substitution with the packed tiled Cholesky factors, one workgroup per
// subdomain.
#include "common.h"
#include "kernels.h"

namespace sfcdd {

// ---------------------------------------------------------------------------
// Subdomain solves d_i = A_i^{-1} R_i w by forward and backward substitution
// with the packed tiled Cholesky factor (Sec. 3.1: factor once, then only
// forward/backward steps; Alg. 2 first two steps).  One workgroup per
// subdomain; R_i w (a cyclic contiguous curve range) is staged in LDS.
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

// NT: factor loads with the non-temporal hint (chosen by the caller when the
// factors being swept are larger than the last-level cache).
template <typename T, int W, bool NT>
__global__ __launch_bounds__(W * 64) void k_schwarz_trsv(
    Batch B, const int32_t* __restrict__ ta, const int32_t* __restrict__ Ni,
    const int32_t* __restrict__ nt, const int64_t* __restrict__ off,
    const int64_t* __restrict__ doff, const T* __restrict__ fac, const double* __restrict__ w,
    double* __restrict__ dbuf, const int32_t* __restrict__ active) {
  typedef typename Vec16<T>::type V;
  constexpr int VEC = Vec16<T>::n;          // elements per lane per load
  constexpr int LPR = TS / VEC;             // lanes per tile row
  constexpr int RPI = 64 / LPR;             // rows per wave load
  constexpr int NGRP = TS / RPI;            // row groups per tile
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
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lrow = lane / LPR, c0 = (lane % LPR) * VEC;
  const T* F = fac + off[b] * TS2;

  for (int s = tid; s < ntb * TS; s += W * 64) {
    T v = T(0);
    if (s < n) {
      int64_t p = t0 + s;
      if (p >= N) p -= N;
      v = (T)wg[p];
    }
    y[s] = v;
  }
  __syncthreads();

  // Rows at or past n are padding (unit diagonal, zero right-hand side, zero
  // solution): their tile rows and columns are never read.  Chunks of the
  // diagonal-tile inverses right of the diagonal are zero and not read either.
  // forward: y_I <- L_II^{-1} (g_I - sum_{J<I} L_IJ y_J)
  for (int I = 0; I < ntb; ++I) {
    const T* rowI = F + tri_index(I, 0) * TS2;
    for (int grp = wv; grp < NGRP; grp += W) {
      const int r = grp * RPI + lrow;
      T acc = T(0);
      if (I * TS + r < n) {
#pragma unroll 4
        for (int J = 0; J < I; ++J) {
          const V v = load_fac<T, NT>(rowI + (int64_t)J * TS2 + r * TS + c0);
          acc += dotv<T>(v, y + J * TS + c0);
        }
      }
      for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((lane % LPR) == 0) sS[r] = y[I * TS + r] - acc;
    }
    __syncthreads();
    const T* D = rowI + (int64_t)I * TS2;
    for (int grp = wv; grp < NGRP; grp += W) {
      const int r = grp * RPI + lrow;
      T acc = T(0);
      if (c0 <= r && I * TS + r < n) {
        const V v = load_fac<T, NT>(D + r * TS + c0);
        acc = dotv<T>(v, sS + c0);
      }
      for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((lane % LPR) == 0) y[I * TS + r] = acc;
    }
    __syncthreads();
  }

  // backward: x_I <- L_II^{-T} (y_I - sum_{K>I} L_KI^T x_K), x overwrites y
  for (int I = ntb - 1; I >= 0; --I) {
    T accv[VEC];
    for (int e = 0; e < VEC; ++e) accv[e] = T(0);
    for (int grp = wv; grp < NGRP; grp += W) {
      const int r = grp * RPI + lrow;
      const int Kend = ntb - 1;  // the last tile row may hold padding rows
#pragma unroll 4
      for (int K = I + 1; K < Kend; ++K) {
        const V v = load_fac<T, NT>(F + tri_index(K, I) * TS2 + r * TS + c0);
        axpyv<T>(accv, v, y[K * TS + r]);
      }
      if (I < Kend && Kend * TS + r < n) {
        const V v = load_fac<T, NT>(F + tri_index(Kend, I) * TS2 + r * TS + c0);
        axpyv<T>(accv, v, y[Kend * TS + r]);
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
    const T* D = F + tri_index(I, I) * TS2;
    for (int grp = wv; grp < NGRP; grp += W) {
      const int r = grp * RPI + lrow;
      if (c0 <= r && I * TS + r < n) {
        const V v = load_fac<T, NT>(D + r * TS + c0);
        axpyv<T>(accv, v, sS[r]);
      }
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
  }

  double* out = dbuf + doff[b];
  for (int s = tid; s < n; s += W * 64) out[s] = (double)y[s];
}

// Waves per workgroup of the substitution kernel: 4, 8 or 16 (a tuning knob).
template <typename T, int W, bool NT>
static void trsv_w(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                   const int64_t* off, const int64_t* doff, int max_nt, const T* fac,
                   const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  const size_t sh = ((size_t)max_nt * TS + TS + (size_t)W * TS) * sizeof(T);
  hipLaunchKernelGGL((k_schwarz_trsv<T, W, NT>), dim3(B.Ptot), dim3(W * 64), sh, s, B, ta, Ni, nt, off,
                     doff, fac, w, dbuf, active);
}

template <typename T, bool NT>
static void trsv_nt(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                    const int64_t* off, const int64_t* doff, int max_nt, int waves, const T* fac,
                    const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  if (waves <= 4) trsv_w<T, 4, NT>(B, ta, Ni, nt, off, doff, max_nt, fac, w, dbuf, active, s);
  else if (waves <= 8) trsv_w<T, 8, NT>(B, ta, Ni, nt, off, doff, max_nt, fac, w, dbuf, active, s);
  else trsv_w<T, 16, NT>(B, ta, Ni, nt, off, doff, max_nt, fac, w, dbuf, active, s);
}

template <typename T>
void launch_schwarz_trsv(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                         const int64_t* off, const int64_t* doff, int max_nt, int waves, bool stream,
                         const T* fac, const double* w, double* dbuf, const int32_t* active,
                         hipStream_t s) {
  if (stream) trsv_nt<T, true>(B, ta, Ni, nt, off, doff, max_nt, waves, fac, w, dbuf, active, s);
  else trsv_nt<T, false>(B, ta, Ni, nt, off, doff, max_nt, waves, fac, w, dbuf, active, s);
}

#define INST(T)                                                                                    \
  template void launch_schwarz_trsv<T>(const Batch&, const int32_t*, const int32_t*,              \
                                       const int32_t*, const int64_t*, const int64_t*, int, int,   \
                                       bool, const T*, const double*, double*, const int32_t*,     \
                                       hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace sfcdd
