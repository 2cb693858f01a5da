// Shared device-side definitions of the PISO library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "piso_topology.h"

namespace piso {

constexpr int kWG = 256;                 // work-group size: 4 wave64s
constexpr int kWaves = kWG / 64;
constexpr int kRedGrid = 2048;           // work-groups of the reduction kernels (upper bound)
// Device block table: kTabStride ints per block as built by build_topology
// (piso_topology.h: extents, side offsets, division magic, periodic-side bits, colour
// parity).
struct Grid {
  int dim;
  int nblocks;
  int N;
  int NB;
  const int* __restrict__ tab;   // [nblocks][kTabStride]
  const int* __restrict__ fmap;  // per side face: neighbour cell (>= 0) or -1 - boundary face
};

// Exact n / d for 0 <= n < 2^31 with m = ceil(2^(31+l) / d), l = ceil(log2 d).
__host__ __device__ inline uint32_t fast_div(uint32_t n, uint64_t m, int s) {
  return (uint32_t)(((uint64_t)n * m) >> s);
}

struct Cell {
  int b, i, j, k;
};

__device__ __forceinline__ int tab(const Grid& g, int b, int f) { return g.tab[b * kTabStride + f]; }

__device__ __forceinline__ Cell locate(const Grid& g, int P) {
  Cell c;
  int b = 0;
  for (int q = 1; q < g.nblocks; ++q) b += (P >= tab(g, q, 0)) ? 1 : 0;
  const int* t = g.tab + b * kTabStride;
  uint32_t L = (uint32_t)(P - t[0]);
  uint64_t mx = (uint64_t)(uint32_t)t[10] | ((uint64_t)(uint32_t)t[11] << 32);
  uint32_t jk = fast_div(L, mx, t[12]);
  c.b = b;
  c.i = (int)(L - jk * (uint32_t)t[1]);
  if (g.dim == 3) {
    uint64_t mxy = (uint64_t)(uint32_t)t[13] | ((uint64_t)(uint32_t)t[14] << 32);
    uint32_t k = fast_div(L, mxy, t[15]);
    c.k = (int)k;
    c.j = (int)(jk - k * (uint32_t)t[2]);
  } else {
    c.k = 0;
    c.j = (int)jk;
  }
  return c;
}

// Neighbour of cell P (at position c) across face (axis, side): a cell index >= 0, or
// -1 - f for Dirichlet face f.
__device__ __forceinline__ int neighbour(const Grid& g, const Cell& c, int P, int axis, int side) {
  const int* t = g.tab + c.b * kTabStride;
  int pos = axis == 0 ? c.i : (axis == 1 ? c.j : c.k);
  int n = t[1 + axis];
  const int stride = axis == 0 ? 1 : (axis == 1 ? t[1] : t[1] * t[2]);
  if (side) {
    if (pos < n - 1) return P + stride;
    if ((t[kTabWrap] >> (2 * axis + 1)) & 1) return P - (n - 1) * stride;
  } else {
    if (pos > 0) return P - stride;
    if ((t[kTabWrap] >> (2 * axis)) & 1) return P + (n - 1) * stride;
  }
  int tg;
  if (axis == 0) tg = c.j + t[2] * c.k;
  else if (axis == 1) tg = c.i + t[1] * c.k;
  else tg = c.i + t[1] * c.j;
  return g.fmap[t[4 + 2 * axis + side] + tg];
}

__device__ __forceinline__ int neighbour_of(const Grid& g, int Q, int axis, int side) {
  Cell c = locate(g, Q);
  return neighbour(g, c, Q, axis, side);
}

// ---------------------------------------------------------------- reductions (FP64)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Work-group sum of NV doubles; result valid in thread 0.  Fixed order: deterministic.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* lds /* [NV][kWaves] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[q * kWaves + wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < kWaves; ++w) s += lds[q * kWaves + w];
      v[q] = s;
    }
  }
}

// Work-group sum of NV doubles broadcast to every thread (fixed order: deterministic).
template <int NV>
__device__ __forceinline__ void wg_sum_all(double (&v)[NV]) {
  __shared__ double lds[NV * kWaves];
  __shared__ double res[NV];
  wg_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) res[q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = res[q];
  __syncthreads();
}

// Grid reductions avoid device-scope fences and atomics (each costs a write-back of
// the XCD's L2 on this chip): every work-group writes its NV partial sums to
// partials[q * G + blockIdx.x], and a later kernel (after the launch boundary has made
// them visible) re-reduces them in work-group order with reduce_partials.
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double* partials) {
  __shared__ double lds[NV * kWaves];
  wg_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[q * gridDim.x + blockIdx.x] = v[q];
  }
}

// Sum of the G partials of NV values, identical in every thread of every work-group.
// The loads are issued U trips of kWG at a time before their adds (a loop with the add
// in it waits for each load in turn, about a microsecond per trip when the partials come
// from another XCD); U shrinks with NV to bound the registers.  The per-thread order of
// the adds is w ascending.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int G, double (&out)[NV]) {
  constexpr int U = NV == 1 ? 8 : (NV == 2 ? 4 : 2);
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = 0.0;
  for (int w0 = 0; w0 < G; w0 += U * kWG) {
    double v[NV][U];
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int w = w0 + (int)threadIdx.x + c * kWG;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q][c] = w < G ? partials[q * G + w] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int c = 0; c < U; ++c) out[q] += v[q][c];
  }
  wg_sum_all<NV>(out);
}

// Contiguous cell range of work-group `wg` when `nwg` groups share N cells, with the
// group index remapped so that each of the 8 XCDs (which receive work-groups round
// robin) covers one contiguous eighth of the cells (keeps stencil neighbours in the
// XCD's own L2).
__device__ __forceinline__ int xcd_logical_group() {
  const int G = gridDim.x, b = blockIdx.x;
  if (G < 8) return b;
  const int x = b & 7, q = b >> 3, per = G >> 3, rem = G & 7;
  return x * per + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ void chunk_range(int N, int& begin, int& end) {
  const int G = gridDim.x;
  int per = (N + G - 1) / G;
  per = (per + 63) & ~63;
  const int lg = xcd_logical_group();
  begin = lg * per;
  end = begin + per;
  if (end > N) end = N;
}

// Cell index of this thread in a one-cell-per-thread launch (XCD-aware), or -1.
__device__ __forceinline__ int cell_of_thread(int N) {
  const int P = xcd_logical_group() * kWG + threadIdx.x;
  return P < N ? P : -1;
}

}  // namespace piso
