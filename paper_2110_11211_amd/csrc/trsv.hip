// Subdomain solves of the fine Schwarz level: forward and backward
// substitution with the tiled Cholesky factors (tile envelopes in the local
// elimination order), one workgroup per subdomain.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sfcdd {

// ---------------------------------------------------------------------------
// Subdomain solves d_i = A_i^{-1} R_i w by forward and backward substitution
// with the tiled Cholesky factor (Sec. 3.1: factor once, then only
// forward/backward steps; Alg. 2 first two steps).  One workgroup per
// subdomain; R_i w (a cyclic contiguous curve range, permuted to the local
// order) is staged in LDS.  Every step is a tile matrix-vector product; each
// wave streams whole 16-byte-per-lane row groups of the tiles.

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

// Cross-lane sums without the LDS crossbar: DPP moves within rows of 16
// lanes, the gfx950 permlane swaps across rows.  Every lane receives the sum
// of its group, formed in a fixed order.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// v + the value of the lane in the paired row of 16 (rows 0 <-> 1, 2 <-> 3),
// or in the other half of the wave (lanes l <-> l ^ 32).
__device__ __forceinline__ float swap16_add(float v) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float swap32_add(float v) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ double swap16_add(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
         __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ double swap32_add(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
         __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
// Sum over each group of LPR consecutive lanes (LPR = 16 or 32).
template <int LPR, typename T>
__device__ __forceinline__ T sum_row_lanes(T v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  if constexpr (LPR == 32) v = swap16_add(v);
  return v;
}
// Sum over the lanes with the same lane % LPR.
template <int LPR, typename T>
__device__ __forceinline__ T sum_col_lanes(T v) {
  if constexpr (LPR == 16) v = swap16_add(v);
  return swap32_add(v);
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
// tile outside is zero.  The off-diagonal tiles hold the unit block-lower
// factor U_IJ = L_IJ L_JJ^{-1}, the diagonal tiles D_I = L_II^{-1}, so that
// A_i = U Delta Delta^T U^T (Delta the diagonal blocks of the Cholesky
// factor) and A_i^{-1} w takes three passes:
//   forward   w_I <- w_I - sum_{lo_I <= J < I} U_IJ w_J       (row I after row I - 1)
//   diagonal  v_I  = D_I^T (D_I w_I)                           (every row at once)
//   backward  x_I  = v_I - sum_{I < K <= hi_I} U_KI^T x_K      (column I after I + 1)
// with hi[I] the last row whose envelope reaches column I.  The dependent
// chains hold only the off-diagonal tiles: one barrier per forward step, two
// per backward step (the column sums of the waves are combined in LDS).
// Each wave owns G row groups of every tile.  The off-diagonal tiles of a
// chain step (at most PF per row group: 4, or 2 for the 4-wave shape meant
// for small subdomains) are loaded into one of NSET
// register sets NSET - 1 steps ahead, so that their latency overlaps the
// steps before.  When every row and column of the envelope holds at most PF
// off-diagonal tiles (the diagonal order keeps 2 to 4), a step issues
// exactly G PF unconditional loads (unused slots read a tile of zeros,
// ztile) and the chain loops hold no other loads, so every wait for a set is
// for that set alone; wider envelopes take
// the extra tiles with loads inside the step.  The barriers order the LDS
// only (lds_barrier).
// NT: factor loads with the non-temporal hint (chosen by the caller when the
// factors being swept are larger than the last-level cache).
constexpr int TRSV_PF = 4;
template <typename T, int W, bool NT>
__global__ __launch_bounds__(W * 64) void k_schwarz_trsv(
    Batch B, const int32_t* __restrict__ ta, const int32_t* __restrict__ Ni,
    const int32_t* __restrict__ nt, const int64_t* __restrict__ off,
    const int64_t* __restrict__ doff, const int64_t* __restrict__ xoff, const int32_t* __restrict__ lperm,
    const int32_t* __restrict__ tlo, const int32_t* __restrict__ trb, const T* __restrict__ fac,
    const T* __restrict__ ztile, const double* __restrict__ w, double* __restrict__ dbuf,
    const int32_t* __restrict__ active) {
  typedef typename Vec16<T>::type V;
  constexpr int VEC = Vec16<T>::n;          // elements per lane per load
  constexpr int LPR = TS / VEC;             // lanes per tile row
  constexpr int RPI = 64 / LPR;             // rows per wave load
  constexpr int NGRP = TS / RPI;            // row groups per tile
  constexpr int G = NGRP / W;               // row groups per wave
  constexpr int PF = G >= 4 ? TRSV_PF / 2 : TRSV_PF;  // prefetched tiles per row group
  constexpr int NSET = G * PF * 4 <= 16 ? 3 : 2;  // register sets in flight (16 bytes = 4 VGPRs a slot)
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
  T* red = y + ntb * TS;                    // W * TS
  int* slo = reinterpret_cast<int*>(red + W * TS);  // ntb
  int* shi = slo + ntb;                     // ntb
  int* srb = shi + ntb;                     // ntb
  __shared__ int s_wide;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lrow = lane / LPR, c0 = (lane % LPR) * VEC;
  const T* F = fac + off[b] * TS2;
  const int64_t xb = xoff[b];
  const int32_t* __restrict__ perm = lperm + xb;

  if (tid == 0) s_wide = 0;
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
  lds_barrier();
  for (int J = tid; J < ntb; J += W * 64) {
    int h = J;
    while (h + 1 < ntb && slo[h + 1] <= J) ++h;
    shi[J] = h;
    if (J - slo[J] > PF || h - J > PF) s_wide = 1;
  }
  lds_barrier();
  const bool wide = s_wide != 0;

  // Rows at or past n are padding: zero right-hand side, zero off-diagonal
  // tiles, zero solution.
  typedef V Set[G][PF];
  Set buf[NSET];
  // off-diagonal tiles of forward row I: (I, lo + k), k < PF
  auto load_fwd = [&](int I, Set& bf) {
    const int lo = slo[I];
    const T* rowI = F + (int64_t)srb[I] * TS2;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const T* p = lo + k < I ? rowI + (int64_t)(lo + k) * TS2 : ztile;
        bf[gg][k] = load_fac<T, NT>(p + r * TS + c0);
      }
    }
  };
  // tiles of backward column I: (I + 1 + k, I), k < PF
  auto load_bwd = [&](int I, Set& bf) {
    const int hi = shi[I];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int K = I + 1 + k;
        const T* p = K <= hi ? F + ((int64_t)srb[K] + I) * TS2 : ztile;
        bf[gg][k] = load_fac<T, NT>(p + r * TS + c0);
      }
    }
  };

  // forward: w_I <- w_I - sum_{lo_I <= J < I} U_IJ w_J
  auto forward = [&](auto wide_tag, int I, const Set& cur) {
    constexpr bool WIDE = decltype(wide_tag)::value;
    const int lo = slo[I];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < PF; ++k) acc += dotv<T>(cur[gg][k], y + min(lo + k, I) * TS + c0);
      if constexpr (WIDE) {
        const T* rowI = F + (int64_t)srb[I] * TS2;
        for (int J = lo + PF; J < I; ++J)
          acc += dotv<T>(load_fac<T, NT>(rowI + (int64_t)J * TS2 + r * TS + c0), y + J * TS + c0);
      }
      acc = sum_row_lanes<LPR>(acc);
      if ((lane % LPR) == 0) y[I * TS + r] -= acc;
    }
    lds_barrier();
  };

  // backward: x_I = v_I - sum_{I < K <= hi_I} U_KI^T x_K
  auto backward = [&](auto wide_tag, int I, const Set& cur) {
    constexpr bool WIDE = decltype(wide_tag)::value;
    T accv[VEC];
    for (int e = 0; e < VEC; ++e) accv[e] = T(0);
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      const int r = (wv + W * gg) * RPI + lrow;
#pragma unroll
      for (int k = 0; k < PF; ++k) axpyv<T>(accv, cur[gg][k], y[min(I + 1 + k, ntb - 1) * TS + r]);
      if constexpr (WIDE) {
        const int hi = shi[I];
        for (int K = I + 1 + PF; K <= hi; ++K)
          axpyv<T>(accv, load_fac<T, NT>(F + ((int64_t)srb[K] + I) * TS2 + r * TS + c0), y[K * TS + r]);
      }
    }
    for (int e = 0; e < VEC; ++e) accv[e] = sum_col_lanes<LPR>(accv[e]);
    if (lane < LPR)
      for (int e = 0; e < VEC; ++e) red[wv * TS + c0 + e] = accv[e];
    lds_barrier();
    if (tid < TS) {
      T s = y[I * TS + tid];
      for (int q = 0; q < W; ++q) s -= red[q * TS + tid];
      y[I * TS + tid] = s;
    }
    lds_barrier();
  };

  // forward chain: whole groups of NSET steps, then the rest
  auto forward_chain = [&](auto wide_tag) {
#pragma unroll
    for (int k = 0; k < NSET - 1; ++k) load_fwd(min(k, ntb - 1), buf[k]);
    int s0 = 0;
    for (; s0 + NSET <= ntb; s0 += NSET) {
#pragma unroll
      for (int u = 0; u < NSET; ++u) {
        load_fwd(min(s0 + u + NSET - 1, ntb - 1), buf[(u + NSET - 1) % NSET]);
        forward(wide_tag, s0 + u, buf[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < NSET - 1; ++u)
      if (s0 + u < ntb) forward(wide_tag, s0 + u, buf[u]);
  };
  if (wide) forward_chain(std::true_type{});
  else forward_chain(std::false_type{});

  // diagonal blocks, every tile row independently: wave wv takes the rows
  // I = wv, wv + W, ..; t = D_I w_I row by row, and v = D_I^T t accumulated
  // over the rows of the tile; the wave reads and then writes only y_I
  // All row groups' loads are issued before their products (chunks right of
  // the diagonal read the zero tile; padding rows carry zeros of y).
  // groups per batch of loads: 64 VGPRs of chunks where the prefetch sets are
  // small (one row group per wave), 16 beside larger sets
  constexpr int HB = (G == 1 ? 64 : 16) / 4 < NGRP ? (G == 1 ? 64 : 16) / 4 : NGRP;
  for (int I = wv; I < ntb; I += W) {
    const T* D = F + ((int64_t)srb[I] + I) * TS2;
    T accv[VEC];
    for (int e = 0; e < VEC; ++e) accv[e] = T(0);
    for (int h = 0; h < NGRP; h += HB) {
      V d[HB];
#pragma unroll
      for (int k = 0; k < HB; ++k) {
        const int r = (h + k) * RPI + lrow;
        d[k] = load_fac<T, NT>((c0 <= r ? D : ztile) + r * TS + c0);
      }
#pragma unroll
      for (int k = 0; k < HB; ++k) {
        T t = sum_row_lanes<LPR>(dotv<T>(d[k], y + I * TS + c0));
        axpyv<T>(accv, d[k], t);
      }
    }
    for (int e = 0; e < VEC; ++e) accv[e] = sum_col_lanes<LPR>(accv[e]);
    if (lane < LPR)
      for (int e = 0; e < VEC; ++e) y[I * TS + c0 + e] = I * TS + c0 + e < n ? accv[e] : T(0);
  }
  lds_barrier();

  // backward chain, columns ntb - 1 down to 0
  auto backward_chain = [&](auto wide_tag) {
#pragma unroll
    for (int k = 0; k < NSET - 1; ++k) load_bwd(max(ntb - 1 - k, 0), buf[k]);
    int s0 = 0;
    for (; s0 + NSET <= ntb; s0 += NSET) {
#pragma unroll
      for (int u = 0; u < NSET; ++u) {
        load_bwd(max(ntb - 1 - (s0 + u + NSET - 1), 0), buf[(u + NSET - 1) % NSET]);
        backward(wide_tag, ntb - 1 - (s0 + u), buf[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < NSET - 1; ++u)
      if (s0 + u < ntb) backward(wide_tag, ntb - 1 - (s0 + u), buf[u]);
  };
  if (wide) backward_chain(std::true_type{});
  else backward_chain(std::false_type{});

  double* out = dbuf + doff[b];
  for (int s = tid; s < n; s += W * 64) out[perm[s]] = (double)y[s];
}

static size_t trsv_lds(int max_nt, size_t es, int W) {
  return ((size_t)max_nt * TS + (size_t)W * TS) * es + 3 * (size_t)max_nt * sizeof(int) + 256;
}
bool trsv_fits(int max_nt, int elem_bytes, int waves) {
  return trsv_lds(max_nt, (size_t)elem_bytes, waves) <= (size_t)160 * 1024;
}

// Waves per workgroup of the substitution kernel: 4, 8 or 16 (a tuning knob).
template <typename T, int W, bool NT>
static void trsv_w(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                   const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                   const int32_t* tlo, const int32_t* trb, int max_nt, const T* fac, const T* ztile,
                   const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  const size_t sh = trsv_lds(max_nt, sizeof(T), W);
  if (sh > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_schwarz_trsv<T, W, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((k_schwarz_trsv<T, W, NT>), dim3(B.Ptot), dim3(W * 64), sh, s, B, ta, Ni, nt, off,
                     doff, xoff, lperm, tlo, trb, fac, ztile, w, dbuf, active);
}

template <typename T, bool NT>
static void trsv_nt(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                    const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                    const int32_t* tlo, const int32_t* trb, int max_nt, int waves, const T* fac,
                    const T* ztile, const double* w, double* dbuf, const int32_t* active, hipStream_t s) {
  while (waves > 4 && !trsv_fits(max_nt, (int)sizeof(T), waves)) waves /= 2;
  if (waves <= 4)
    trsv_w<T, 4, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, ztile, w, dbuf, active, s);
  else if (waves <= 8)
    trsv_w<T, 8, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, ztile, w, dbuf, active, s);
  else
    trsv_w<T, 16, NT>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, fac, ztile, w, dbuf, active, s);
}

template <typename T>
void launch_schwarz_trsv(const Batch& B, const int32_t* ta, const int32_t* Ni, const int32_t* nt,
                         const int64_t* off, const int64_t* doff, const int64_t* xoff, const int32_t* lperm,
                         const int32_t* tlo, const int32_t* trb, int max_nt, int waves, bool stream,
                         const T* fac, const T* ztile, const double* w, double* dbuf, const int32_t* active,
                         hipStream_t s) {
  if (stream)
    trsv_nt<T, true>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, waves, fac, ztile, w, dbuf, active,
                     s);
  else
    trsv_nt<T, false>(B, ta, Ni, nt, off, doff, xoff, lperm, tlo, trb, max_nt, waves, fac, ztile, w, dbuf, active,
                      s);
}

#define INST(T)                                                                                    \
  template void launch_schwarz_trsv<T>(const Batch&, const int32_t*, const int32_t*,              \
                                       const int32_t*, const int64_t*, const int64_t*,             \
                                       const int64_t*, const int32_t*, const int32_t*,             \
                                       const int32_t*, int, int, bool, const T*, const T*,         \
                                       const double*, double*, const int32_t*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace sfcdd
