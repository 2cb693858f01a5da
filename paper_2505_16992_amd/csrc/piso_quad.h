// Vectorised ("quad") stencil helpers shared by the Krylov and multigrid kernels.
#pragma once

#include "piso_common.h"

namespace piso {

// ------------------------------------------------------------ quad fast path
// Four consecutive x-cells of one row per thread (every block has nx % 4 == 0): the
// operand, coefficient and output streams move as 16-byte (float) or 32-byte (double)
// vectors; neighbours across a block side come from the face map cell by cell.

template <typename R>
struct Q4 {
  R v[4];
};

template <typename R>
__device__ __forceinline__ Q4<R> ldq(const R* __restrict__ p, int P) {
  Q4<R> q;
  if constexpr (sizeof(R) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p + P);
    q.v[0] = t.x; q.v[1] = t.y; q.v[2] = t.z; q.v[3] = t.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p + P);
    const double2 b = *reinterpret_cast<const double2*>(p + P + 2);
    q.v[0] = a.x; q.v[1] = a.y; q.v[2] = b.x; q.v[3] = b.y;
  }
  return q;
}

template <typename R>
__device__ __forceinline__ void stq(R* __restrict__ p, int P, const Q4<R>& q) {
  if constexpr (sizeof(R) == 4) {
    *reinterpret_cast<float4*>(p + P) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
  } else {
    *reinterpret_cast<double2*>(p + P) = make_double2(q.v[0], q.v[1]);
    *reinterpret_cast<double2*>(p + P + 2) = make_double2(q.v[2], q.v[3]);
  }
}

// M d over the quad starting at P0 for an operand given by dq(P, j, k) (the 4 cells of
// the quad at P, which lies in row j, plane k of the same block) and d1(F, known, i, j, k)
// (one cell; its position in this block when known, else it lies across a block side);
// dP is the operand at the quad.  Pf face arrays as in the scalar kernels.  Sides that
// wrap onto the same block are indexed arithmetically, other block sides through the
// face map.
template <typename R, int D, typename FQ, typename F1>
__device__ __forceinline__ Q4<R> quad_stencil(const Grid& g, const Cell& c, int P0, const R* __restrict__ Pf,
                                              const Q4<R>& dP, FQ dq, F1 d1) {
  const int N = g.N;
  const int* t = g.tab + c.b * kTabStride;
  const int nx = t[1], ny = t[2], nz = t[3];
  const int wrap = t[kTabWrap];
  Q4<R> M;
  // x faces
  const Q4<R> px = ldq(Pf, P0);
  int Lx, Rx, Li = 0, Ri = 0;
  bool Lk = true, Rk = true;
  if (c.i > 0) {
    Lx = P0 - 1;
    Li = c.i - 1;
  } else if (wrap & 1) {
    Lx = P0 + nx - 1;
    Li = nx - 1;
  } else {
    Lx = g.fmap[t[4] + c.j + ny * c.k];
    Lk = false;
  }
  if (c.i + 4 < nx) {
    Rx = P0 + 4;
    Ri = c.i + 4;
  } else if (wrap & 2) {
    Rx = P0 + 4 - nx;
    Ri = 0;
  } else {
    Rx = g.fmap[t[5] + c.j + ny * c.k];
    Rk = false;
  }
  const R dl = Lx >= 0 ? d1(Lx, Lk, Li, c.j, c.k) : R(0);
  const R pl = Lx >= 0 ? Pf[Lx] : R(0);
  const R dr = Rx >= 0 ? d1(Rx, Rk, Ri, c.j, c.k) : R(0);
  M.v[0] = px.v[0] * (dP.v[0] - dP.v[1]) + pl * (dP.v[0] - dl);
  M.v[1] = px.v[1] * (dP.v[1] - dP.v[2]) + px.v[0] * (dP.v[1] - dP.v[0]);
  M.v[2] = px.v[2] * (dP.v[2] - dP.v[3]) + px.v[1] * (dP.v[2] - dP.v[1]);
  M.v[3] = (Rx >= 0 ? px.v[3] * (dP.v[3] - dr) : R(0)) + px.v[2] * (dP.v[3] - dP.v[2]);
  // y and z faces
#pragma unroll
  for (int a = 1; a < D; ++a) {
    const int pos = a == 1 ? c.j : c.k;
    const int n = a == 1 ? ny : nz;
    const int stride = a == 1 ? nx : nx * ny;
    const R* Pa = Pf + (size_t)a * N;
    // +a side: own face coefficients
    const Q4<R> pp = ldq(Pa, P0);
    if (pos < n - 1 || ((wrap >> (2 * a + 1)) & 1)) {
      const bool in = pos < n - 1;
      const int Pn = in ? P0 + stride : P0 - (n - 1) * stride;
      const int q = in ? pos + 1 : 0;
      const Q4<R> nb = dq(Pn, a == 1 ? q : c.j, a == 2 ? q : c.k);
#pragma unroll
      for (int e = 0; e < 4; ++e) M.v[e] += pp.v[e] * (dP.v[e] - nb.v[e]);
    } else {
      const int base = t[4 + 2 * a + 1] + (a == 1 ? c.i + nx * c.k : c.i + nx * c.j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int F = g.fmap[base + e];
        if (F >= 0) M.v[e] += pp.v[e] * (dP.v[e] - d1(F, false, 0, 0, 0));
      }
    }
    // -a side: coefficients stored at the neighbour
    if (pos > 0 || ((wrap >> (2 * a)) & 1)) {
      const bool in = pos > 0;
      const int Pn = in ? P0 - stride : P0 + (n - 1) * stride;
      const int q = in ? pos - 1 : n - 1;
      const Q4<R> nb = dq(Pn, a == 1 ? q : c.j, a == 2 ? q : c.k);
      const Q4<R> pm = ldq(Pa, Pn);
#pragma unroll
      for (int e = 0; e < 4; ++e) M.v[e] += pm.v[e] * (dP.v[e] - nb.v[e]);
    } else {
      const int base = t[4 + 2 * a] + (a == 1 ? c.i + nx * c.k : c.i + nx * c.j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int F = g.fmap[base + e];
        if (F >= 0) M.v[e] += Pa[F] * (dP.v[e] - d1(F, false, 0, 0, 0));
      }
    }
  }
  return M;
}

// Quads of this work-group in XCD bands: the work-groups one XCD receives (round robin
// over the 8 XCDs) share that XCD's contiguous eighth of the quads and sweep it
// together, one band of (groups on the XCD) x kWG quads per trip.  The rows and planes
// next to a band are touched in the same or the adjacent trip, while they are still in
// the XCD's L2 (a contiguous range per work-group spreads the XCD's concurrent work
// over its whole eighth).
__device__ __forceinline__ void quad_sweep(int NQ, int& first, int& end, int& stride) {
  const int G = gridDim.x, b = blockIdx.x;
  if (G < 8) {
    first = b * kWG + (int)threadIdx.x;
    end = NQ;
    stride = G * kWG;
    return;
  }
  const int x = b & 7, w = b >> 3;
  const int gx = (G >> 3) + (x < (G & 7) ? 1 : 0);
  const int per = (NQ + 7) >> 3;
  const int x0 = x * per < NQ ? x * per : NQ;
  end = x0 + per < NQ ? x0 + per : NQ;
  first = x0 + w * kWG + (int)threadIdx.x;
  stride = gx * kWG;
}

__device__ __forceinline__ void quad_range(int NQ, int& beg, int& end) {
  const int G = gridDim.x;
  int per = (NQ + G - 1) / G;
  per = (per + 63) & ~63;
  beg = xcd_logical_group() * per;
  end = beg + per;
  if (end > NQ) end = NQ;
}

}  // namespace piso
