// Device-side building blocks shared by the sfcdd kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfcdd {

// Edge of the square tiles of the packed lower-triangular factor layout.
constexpr int TS = 64;
constexpr int TS2 = TS * TS;
// Row stride (elements) of a tile staged in LDS; odd to spread LDS banks.
constexpr int LDS_S = TS + 1;
// Workgroup size of the tile kernels: 4 waves, each owning a 32x32 quadrant.
constexpr int TILE_THREADS = 256;
// K-chunk length of the split-K tile updates used for single matrices (16
// measured best at nt = 128: fewer partial tiles on the diagonal chain than
// 8, shorter partial workgroups than 24 or 32).
constexpr int SPLITK = 16;
// Blocks used by the first stage of the deterministic two-stage reductions.
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<float> {
  typedef f32x4 type;
  // row within a 16x16 block of register r of lane group g = lane / 16
  __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
};
template <> struct Acc<double> {
  typedef f64x4 type;
  __device__ __forceinline__ static int row(int g, int r) { return 4 * r + g; }
};

// One 16x16x4 MFMA step: c += a(16x4) * b(4x16).  Lane l supplies
// a[l%16][l/16] and b[l/16][l%16].  Lane l, register r of c holds
// C[4*(l/16) + r][l%16] for the f32 instruction and C[4*r + l/16][l%16] for
// the f64 one (both measured on gfx950).
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16-byte vector of T (one load per lane).
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };

// Index of lower tile (I, J), J <= I, in row-major packed tile order.
__device__ __host__ __forceinline__ int64_t tri_index(int I, int J) {
  return (int64_t)I * (I + 1) / 2 + J;
}

// Row stride (elements) of the tiles staged in LDS for the MFMA tile
// products: 16-byte aligned rows, consecutive rows 16 bytes apart in the bank
// space (68 floats, 66 doubles).
template <typename T> struct LdsV { static constexpr int v = TS + 16 / (int)sizeof(T); };

// Copies a row-major TS x TS tile from global memory into LDS (stride
// LdsV), as is or transposed.
template <typename T>
__device__ __forceinline__ void stage_tile(T* __restrict__ lds, const T* __restrict__ g) {
  constexpr int S = LdsV<T>::v;
  for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) lds[(e / TS) * S + (e % TS)] = g[e];
}
template <typename T>
__device__ __forceinline__ void stage_tile_t(T* __restrict__ lds, const T* __restrict__ g) {
  constexpr int S = LdsV<T>::v;
  for (int e = threadIdx.x; e < TS2; e += TILE_THREADS) lds[(e % TS) * S + (e / TS)] = g[e];
}

// One row-major TS x TS tile held in registers across the workgroup (16-byte
// vector loads, TS2 / TILE_THREADS elements per thread): the prefetch buffer
// that lets the next tiles load from memory while MFMA works on LDS.
template <typename T> struct TileRegs {
  static constexpr int VEC = 16 / sizeof(T);
  static constexpr int NV = TS2 / (TILE_THREADS * VEC);
  typedef T V __attribute__((ext_vector_type(VEC)));
  V v[NV];
  __device__ __forceinline__ void load(const T* __restrict__ g) {
    const V* gv = reinterpret_cast<const V*>(g);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = gv[threadIdx.x + q * TILE_THREADS];
  }
  // as is (16-byte stores)
  __device__ __forceinline__ void store_lds(T* __restrict__ lds) const {
    constexpr int S = LdsV<T>::v;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = (threadIdx.x + q * TILE_THREADS) * VEC;
      *reinterpret_cast<V*>(lds + (e / TS) * S + (e % TS)) = v[q];
    }
  }
  // transposed: LDS row c holds global column c
  __device__ __forceinline__ void store_lds_t(T* __restrict__ lds) const {
    constexpr int S = LdsV<T>::v;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = (threadIdx.x + q * TILE_THREADS) * VEC;
      const int r = e / TS, c0 = e % TS;
#pragma unroll
      for (int u = 0; u < VEC; ++u) lds[(c0 + u) * S + r] = v[q][u];
    }
  }
};

// Accumulator of one wave: 2x2 blocks of 16x16 covering a 32x32 quadrant of
// the 64x64 output tile.  Quadrant of wave w: rows 32*(w/2), cols 32*(w%2).
template <typename T> struct TileAcc {
  typename Acc<T>::type c[2][2];
  __device__ __forceinline__ void zero() {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) c[a][b][r] = T(0);
  }
  // Row / column of register r of block (a, b) for this lane.
  __device__ __forceinline__ static int row(int a, int r) {
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return 32 * (w >> 1) + 16 * a + Acc<T>::row(l >> 4, r);
  }
  __device__ __forceinline__ static int col(int b) {
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    return 32 * (w & 1) + 16 * b + (l & 15);
  }
  __device__ __forceinline__ void load(const T* __restrict__ g) {  // row-major global tile
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) c[a][b][r] = g[row(a, r) * TS + col(b)];
  }
  __device__ __forceinline__ void sub(const T* __restrict__ g) {  // acc -= row-major tile
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) c[a][b][r] -= g[row(a, r) * TS + col(b)];
  }
  __device__ __forceinline__ void store(T* __restrict__ g) const {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) g[row(a, r) * TS + col(b)] = c[a][b][r];
  }
  __device__ __forceinline__ void store_lds(T* __restrict__ s) const {  // row-major, stride LdsV
    constexpr int S = LdsV<T>::v;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) s[row(a, r) * S + col(b)] = c[a][b][r];
  }
  __device__ __forceinline__ void store_lds_t(T* __restrict__ s) const {  // transposed, stride LdsV
    constexpr int S = LdsV<T>::v;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int r = 0; r < 4; ++r) s[col(b) * S + row(a, r)] = c[a][b][r];
  }
};

// acc += sign * A Bt^T for LDS tiles sA[i][k] and sBt[j][k] (both
// k-contiguous, stride LdsV).  Lane (li, lk) reads four consecutive k of its
// rows with one vector load and feeds them to four MFMA steps: in group t,
// step u, lane group lk covers k = 16 t + 4 lk + u, the same k for A and B,
// so every k in 0..TS-1 is summed exactly once.
// Four consecutive elements from a 16-byte aligned LDS address (16-byte loads).
__device__ __forceinline__ void load4(float (&d)[4], const float* p) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
}
__device__ __forceinline__ void load4(double (&d)[4], const double* p) {
  const double2 v0 = *reinterpret_cast<const double2*>(p);
  const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
  d[0] = v0.x; d[1] = v0.y; d[2] = v1.x; d[3] = v1.y;
}

template <typename T>
__device__ __forceinline__ void tile_mma(TileAcc<T>& acc, const T* __restrict__ sA,
                                         const T* __restrict__ sBt, T sign) {
  constexpr int S = LdsV<T>::v;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = 32 * (w >> 1), j0 = 32 * (w & 1);
  const int li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < TS / 16; ++t) {
    const int kb = 16 * t + 4 * lk;
    T a[2][4], b[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      load4(a[m], sA + (i0 + 16 * m + li) * S + kb);
#pragma unroll
      for (int u = 0; u < 4; ++u) a[m][u] *= sign;
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) load4(b[n], sBt + (j0 + 16 * n + li) * S + kb);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc.c[m][n] = mfma16(a[m][u], b[n][u], acc.c[m][n]);
  }
}

// acc -= the n row-major tiles at base + c stride, c < n: the loads of four
// tiles are issued before their subtractions, so their latencies overlap.
template <typename T>
__device__ __forceinline__ void sub_tiles(TileAcc<T>& acc, const T* __restrict__ base, int64_t stride, int n) {
  int c = 0;
  for (; c + 4 <= n; c += 4) {
    T t[4][2][2][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            t[q][a][b][r] = base[(c + q) * stride + TileAcc<T>::row(a, r) * TS + TileAcc<T>::col(b)];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc.c[a][b][r] -= t[q][a][b][r];
  }
  for (; c < n; ++c) acc.sub(base + c * stride);
}

// Workgroup barrier that orders the LDS accesses only.  A plain
// __syncthreads also waits for every outstanding global load (loads and
// stores share one counter on this architecture), which would drain register
// prefetches; this one is for barriers that guard LDS reuse alone, with no
// global store before it that another wave reads after it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave-level sum (all 64 lanes receive the result).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-level sum for blockDim.x <= 1024; result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh /* >= 16 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// Piece (disjoint subdomain) containing curve position p, for P pieces of
// sizes floor(N/P)+1 (first N mod P) and floor(N/P).
__device__ __host__ __forceinline__ int piece_of(int64_t p, int64_t base, int64_t rem) {
  const int64_t big = rem * (base + 1);
  return p < big ? (int)(p / (base + 1)) : (int)(rem + (p - big) / base);
}
__device__ __host__ __forceinline__ int64_t piece_start(int i, int64_t base, int64_t rem) {
  return (int64_t)i * base + (i < rem ? i : rem);
}

}  // namespace sfcdd
