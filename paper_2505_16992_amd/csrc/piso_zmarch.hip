// Plane-marching forms of the three fine-grid kernels of the multigrid PCG on 3D grids
// whose blocks have nx % 4 == 0 (point smoothing on the fine level).
//
// The operator is the same as everywhere else: (M x)_P = sum_f P_f (x_P - x_F)
// (eq. pMatDiscrete), the PCG of App. A.6 with the aggregation V-cycle of piso_mg.hip.
// What changes is the order in which a work-group visits the cells.  In the one-quad-per-
// thread kernels every cell's neighbours in y and z are loaded again by the thread that
// needs them; on a 256^3 grid the chip keeps so many work-groups in flight that those
// lines have usually left the XCD's L2 before the second load arrives (measured: 12.8
// streams read by the fused update and restriction against 7 needed).  Here a work-group
// owns a tile of rows (a run of x-quads by an even number of rows) and marches it through
// an even run of planes:
//  * neighbours along z come from the plane before (kept in registers) and the plane
//    after (the next step's own loads): the face between planes k-1 and k is evaluated
//    once, at step k, and the result for plane k-1 is completed then;
//  * neighbours in x and y inside the tile come from LDS (one barrier per plane, double
//    buffered by plane parity);
//  * only the rows next to the tile, the planes next to the run and neighbours across
//    block sides are read from memory.
// The next plane's loads are issued before the current plane's barrier, so that their
// latency overlaps the LDS exchange and the arithmetic.
//
// Grid order: work-groups of one block run the tiles in y fastest, then x, then the runs
// of planes, so that the work-groups one XCD holds at a time are neighbours in y at the
// same planes (the halo rows they share are then read close together).
#include <cstdio>
#include <cstdlib>

#include "piso_impl.h"
#include "piso_quad.h"

namespace piso {

namespace {

// Work-group sum of NV doubles, broadcast to every thread (fixed order: deterministic).
template <int NV, int WGS>
__device__ __forceinline__ void zm_sum_all(double (&v)[NV]) {
  constexpr int NW = WGS / 64;
  __shared__ double lds[NV][NW];
  __shared__ double res[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[q][threadIdx.x >> 6] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += lds[q][w];
      res[q] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = res[q];
  __syncthreads();
}

// Sum of the G partials of NV values written by the previous kernel (one per work-group),
// identical in every thread; all loads of a trip are issued before the adds.
template <int NV, int WGS>
__device__ __forceinline__ void zm_reduce_partials(const double* __restrict__ partials, int G, double (&out)[NV]) {
  constexpr int U = NV == 1 ? 4 : 2;
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = 0.0;
  for (int w0 = 0; w0 < G; w0 += U * WGS) {
    double v[NV][U];
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int w = w0 + (int)threadIdx.x + c * WGS;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q][c] = w < G ? partials[q * G + w] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
      for (int c = 0; c < U; ++c) out[q] += v[q][c];
  }
  zm_sum_all<NV, WGS>(out);
}

template <int NV, int WGS>
__device__ __forceinline__ void zm_write_partials(double (&v)[NV], double* __restrict__ partials) {
  zm_sum_all<NV, WGS>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[q * gridDim.x + blockIdx.x] = v[q];
  }
}

// This thread's place: block, tile, x-quad and row, the run of planes [k0, k1).
struct ZmPos {
  const int* tf;   // the block's row of the fine block table
  int b, nx, ny, nz, nxq, wrap;
  int XQ, RT;      // quads per tile row, rows per tile
  int xl, jr;      // quad and row inside the tile (unit threadIdx.x = jr * XQ + xl)
  int xq, j;       // quad and row in the block
  int k0, k1;
  int base;        // first cell of the quad in plane 0 (0 when not active)
  bool act;        // a cell quad of the block (threads past the tile's edge only join barriers)
};

__device__ __forceinline__ ZmPos zm_pos(const Grid& g, const ZmTiles& tl) {
  ZmPos p;
  const int grp = xcd_logical_group();
  int b = 0;
  for (int q = 1; q < tl.nb; ++q) b += grp >= tl.off[q] ? 1 : 0;
  int l = grp - tl.off[b];
  const int nty = tl.nty[b], ntx = tl.ntx[b];
  const int ty = l % nty;
  l /= nty;
  const int tx = l % ntx, tz = l / ntx;
  p.b = b;
  p.tf = g.tab + b * kTabStride;
  p.nx = p.tf[1];
  p.ny = p.tf[2];
  p.nz = p.tf[3];
  p.nxq = p.nx >> 2;
  p.wrap = p.tf[kTabWrap];
  p.XQ = tl.xq[b];
  p.RT = tl.rt[b];
  p.xl = (int)threadIdx.x % p.XQ;
  p.jr = (int)threadIdx.x / p.XQ;
  p.xq = tx * p.XQ + p.xl;
  p.j = ty * p.RT + p.jr;
  p.k0 = tz * tl.ks[b];
  p.k1 = min(p.k0 + tl.ks[b], p.nz);
  p.act = p.jr < p.RT && p.xq < p.nxq && p.j < p.ny;
  p.base = p.act ? p.tf[0] + 4 * p.xq + p.nx * p.j : 0;
  return p;
}

template <typename R>
__device__ __forceinline__ Q4<R> zq4() {
  Q4<R> z;
#pragma unroll
  for (int e = 0; e < 4; ++e) z.v[e] = R(0);
  return z;
}

}  // namespace

// ---------------------------------------------------------------------------------
// Loop structure shared by the three kernels.  Step k: (a) issue the loads of plane k's
// neighbours that come from memory (the rows beside the tile, the plane after the run),
// (b) issue the next plane's own loads, unconditionally (the last step reads its own
// plane again), (c) compute plane k, exchange through LDS, complete plane k - 1.  Every
// load plane k needs is issued before (b): the hardware counts outstanding loads in
// order, so a load issued after (b) and used in (c) would make (c) wait for the next
// plane too.  Rarer paths (sides connected to other blocks, rows split over several
// tiles in x) load in (c) and pay that wait.

// PCG update fused with the fine-level pre-smoothing and restriction (the marching form
// of k_mg_down0uq): alpha = rz / (d.q) from the stencil kernel's partials, x += alpha d,
// r' = r - alpha q, y = omega D^-1 r', and the level-1 residual of each 2x2x2 aggregate,
// the sum over its cells of r' - sum over the faces leaving the aggregate of
// P_f (y_P - y_F).  Aggregates are pairs of quad cells (0,1) and (2,3), rows (j, j+1) with
// j even (the two rows are two threads of the tile: the odd row hands its sums to the
// even one through LDS) and planes (k, k+1) with k even (summed in the thread).
template <typename R, int WGS, bool GEN>
__global__ void __launch_bounds__(WGS)
k_zm_down(Grid g, Grid g1, ZmTiles tl, const R* __restrict__ Pf, const R* __restrict__ Dinv, R* __restrict__ x,
          const R* __restrict__ rin, R* __restrict__ rout, const R* __restrict__ dnew, const R* __restrict__ q,
          R* __restrict__ y, R omega, R* __restrict__ rc, CgState* st, const double* __restrict__ partA, int Gp,
          int par) {
  constexpr int HW = WGS / 2;
  __shared__ Q4<R> ly[2][WGS];   // y of each unit's quad, by plane parity
  __shared__ R lpx[2][WGS];      // its x-face coefficient at cell 3 (the right neighbour's left face)
  __shared__ Q4<R> lpy[2][HW];   // P_y of the odd rows (the face the even row above crosses)
  __shared__ R lag[2][HW][2];    // the odd row's aggregate sums for its even partner
  const int done = st->done;
  const double rzp = st->rz[par];
  const ZmPos p = zm_pos(g, tl);
  const int N = g.N, S = p.nx * p.ny;
  const R* __restrict__ Py = Pf + (size_t)N;
  const R* __restrict__ Pz = Pf + 2 * (size_t)N;
  const int u = threadIdx.x;
  const bool odd = (p.j & 1) != 0;
  const bool in_tile = p.jr < p.RT;
  const int hu = (p.jr >> 1) * p.XQ + p.xl;   // slot of the row pair (p.jr < p.RT)
  const int* tc = g1.tab + p.b * kTabStride;
  const int tc0 = tc[0], cx = tc[1], cy = tc[2];
  const int i0 = 4 * p.xq;
  const bool wym = (p.wrap >> 2) & 1, wyp = (p.wrap >> 3) & 1, wzp = (p.wrap >> 5) & 1;
  // y faces crossed through memory: -y by the even row starting the tile (or row 0 of a
  // block wrapping in y), +y by the odd row ending it (or the last row of a wrapping block,
  // also when that row is even: a one-row aggregate)
  const bool ym = p.act && !odd && (p.j > 0 ? p.jr == 0 : wym);
  const bool yp = p.act && (odd ? (p.j + 1 < p.ny ? p.jr + 1 == p.RT : wyp) : (p.j + 1 == p.ny && wyp));
  const int oym = p.j > 0 ? -p.nx : (p.ny - 1) * p.nx;
  const int oyp = p.j + 1 < p.ny ? p.nx : -(p.ny - 1) * p.nx;
  // P_y is needed by odd rows (and a one-row aggregate), P_z by odd planes (and a one-plane
  // aggregate): the other rows and planes read P_x's line again instead, without a branch
  const size_t oy = (odd || p.j + 1 == p.ny) ? (size_t)N : 0;   // offsets (a select of values, not of lvalues)
  struct Ld {
    Q4<R> x, d, r, q, D, px, py, pz;
  };
  auto load = [=](int k) __attribute__((always_inline)) {
    Ld L;
    const int P = p.act ? p.base + S * k : 0;
    const size_t oz = ((k & 1) || k + 1 == p.nz) ? 2 * (size_t)N : 0;
    L.x = ldq(x, P);
    L.d = ldq(dnew, P);
    L.r = ldq(rin, P);
    L.q = ldq(q, P);
    L.D = ldq(Dinv, P);
    L.px = ldq(Pf, P);
    L.py = ldq(Pf + oy, P);
    L.pz = ldq(Pf + oz, P);
    return L;
  };
  Ld bufA = load(p.k0), bufB;
  // the plane before the run (its y and P_z cross into plane k0), when it lies in the block
  Q4<R> hr = zq4<R>(), hq = zq4<R>(), hD = zq4<R>(), hpz = zq4<R>();
  const bool hz_in = p.k0 > 0 || ((p.wrap >> 4) & 1);
  if (p.act && hz_in) {
    const int Pm = p.base + S * (p.k0 > 0 ? p.k0 - 1 : p.nz - 1);
    hr = ldq(rin, Pm);
    hq = ldq(q, Pm);
    hD = ldq(Dinv, Pm);
    hpz = ldq(Pz, Pm);
  }
  double t[1];
  zm_reduce_partials<1, WGS>(partA, Gp, t);
  if (done) return;
  const double dq = t[0];
  if (!(dq > 0.0) || !std::isfinite(dq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->iters = st->k;
      st->done = 1;
    }
    return;
  }
  const R alpha = (R)(rzp / dq);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k = st->k + 1;   // no other group reads it here
  auto yv = [&](const Q4<R>& a, const Q4<R>& b, const Q4<R>& c) __attribute__((always_inline)) {
    Q4<R> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o.v[e] = omega * c.v[e] * (a.v[e] - alpha * b.v[e]);
    return o;
  };
  const Q4<R> yh = yv(hr, hq, hD);   // y of the plane before the run
  auto y1 = [&](int F) __attribute__((always_inline)) { return omega * Dinv[F] * (rin[F] - alpha * q[F]); };
  // completed aggregate sums (cells 0,1 and 2,3 of the quad) of the plane pair ck
  auto emit = [&](R a, R bb, int ck, int buf) __attribute__((always_inline)) {
    if (p.j + 1 < p.ny) {
      a += lag[buf][hu][0];
      bb += lag[buf][hu][1];
    }
    const int I = tc0 + 2 * p.xq + cx * ((p.j >> 1) + cy * ck);
    rc[I] = a;
    rc[I + 1] = bb;
  };
  Q4<R> yprev = zq4<R>(), pzprev = zq4<R>();
  R agA = R(0), agB = R(0), pendA = R(0), pendB = R(0);
  int pend = -1;   // plane pair of a completed aggregate waiting for the odd row's sums
  // one plane: cur holds its loads, the next plane's go to nxt (two buffers used in
  // turn, so that no register copy waits for the loads in flight)
  auto step = [&](const int k, const Ld& cur, Ld& nxt) __attribute__((always_inline)) {
    const int bs = k & 1;
    const int Pk = p.act ? p.base + S * k : 0;
    // (a) neighbours in memory
    Q4<R> a0, a1, a2, a3, b0, b1, b2, c0, c1, c2;
    if (ym) {
      a0 = ldq(rin, Pk + oym);
      a1 = ldq(q, Pk + oym);
      a2 = ldq(Dinv, Pk + oym);
      a3 = ldq(Py, Pk + oym);
    }
    if (yp) {
      b0 = ldq(rin, Pk + oyp);
      b1 = ldq(q, Pk + oyp);
      b2 = ldq(Dinv, Pk + oyp);
    }
    const bool zp = p.act && (k & 1) && k + 1 == p.k1 && (k + 1 < p.nz || wzp);
    if (zp) {
      const int Pn = k + 1 < p.nz ? Pk + S : Pk - (p.nz - 1) * S;
      c0 = ldq(rin, Pn);
      c1 = ldq(q, Pn);
      c2 = ldq(Dinv, Pn);
    }
    // (b) the next plane
    nxt = load(k + 1 < p.k1 ? k + 1 : k);
    // (c) this plane
    Q4<R> yk, res, xv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xv.v[e] = cur.x.v[e] + alpha * cur.d.v[e];
      res.v[e] = cur.r.v[e] - alpha * cur.q.v[e];
      yk.v[e] = omega * cur.D.v[e] * res.v[e];
    }
    if (p.act) {
      stq(x, Pk, xv);
      stq(rout, Pk, res);
      stq(y, Pk, yk);
    }
    ly[bs][u] = yk;
    lpx[bs][u] = cur.px.v[3];
    if (odd && in_tile) lpy[bs][hu] = cur.py;
    __syncthreads();
    if (pend >= 0) {
      if (p.act && !odd) emit(pendA, pendB, pend, 0);
      pend = -1;
    }
    if (p.act) {
      // x faces: cell 0 to the left quad, 1 | 2 between the quad's aggregates, 3 to the right
      {
        bool have = true;
        R yl = R(0), pl = R(0);
        if (i0 > 0) {
          if (!GEN || p.xl > 0) {
            yl = ly[bs][u - 1].v[3];
            pl = lpx[bs][u - 1];
          } else {
            yl = y1(Pk - 1);
            pl = Pf[Pk - 1];
          }
        } else if (p.wrap & 1) {
          if (!GEN || p.XQ == p.nxq) {
            yl = ly[bs][u + p.nxq - 1].v[3];
            pl = lpx[bs][u + p.nxq - 1];
          } else {
            yl = y1(Pk + p.nx - 1);
            pl = Pf[Pk + p.nx - 1];
          }
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[4] + p.j + p.ny * k];
          have = F >= 0;
          if (have) {
            yl = y1(F);
            pl = Pf[F];
          }
        }
        if (have) res.v[0] -= pl * (yk.v[0] - yl);
      }
      res.v[1] -= cur.px.v[1] * (yk.v[1] - yk.v[2]);
      res.v[2] -= cur.px.v[1] * (yk.v[2] - yk.v[1]);
      {
        bool have = true;
        R yr = R(0);
        if (i0 + 4 < p.nx) {
          yr = (!GEN || p.xl + 1 < p.XQ) ? ly[bs][u + 1].v[0] : y1(Pk + 4);
        } else if (p.wrap & 2) {
          yr = (!GEN || p.XQ == p.nxq) ? ly[bs][u - (p.nxq - 1)].v[0] : y1(Pk + 4 - p.nx);
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[5] + p.j + p.ny * k];
          have = F >= 0;
          if (have) yr = y1(F);
        }
        if (have) res.v[3] -= cur.px.v[3] * (yk.v[3] - yr);
      }
      // y faces: the even row crosses to row j - 1 (coefficient stored there), the odd
      // row to row j + 1 (its own coefficient)
      if (!odd) {
        if (p.j > 0 || wym) {
          Q4<R> yn, wn;
          if (p.jr > 0) {
            yn = ly[bs][u - p.XQ];
            wn = lpy[bs][((p.jr - 1) >> 1) * p.XQ + p.xl];
          } else {
            yn = yv(a0, a1, a2);
            wn = a3;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) res.v[e] -= wn.v[e] * (yk.v[e] - yn.v[e]);
        } else if constexpr (GEN) {
          const int bse = p.tf[6] + i0 + p.nx * k;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F = g.fmap[bse + e];
            if (F >= 0) res.v[e] -= Py[F] * (yk.v[e] - y1(F));
          }
        }
        if (GEN && p.j + 1 == p.ny) {   // a one-row aggregate at the block's end: its +y face leaves too
          if (wyp) {
            const Q4<R> yn = yv(b0, b1, b2);
#pragma unroll
            for (int e = 0; e < 4; ++e) res.v[e] -= cur.py.v[e] * (yk.v[e] - yn.v[e]);
          } else if constexpr (GEN) {
            const int bse = p.tf[7] + i0 + p.nx * k;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int F = g.fmap[bse + e];
              if (F >= 0) res.v[e] -= cur.py.v[e] * (yk.v[e] - y1(F));
            }
          }
        }
      } else {
        if (p.j + 1 < p.ny || wyp) {
          const Q4<R> yn = (p.j + 1 < p.ny && p.jr + 1 < p.RT) ? ly[bs][u + p.XQ] : yv(b0, b1, b2);
#pragma unroll
          for (int e = 0; e < 4; ++e) res.v[e] -= cur.py.v[e] * (yk.v[e] - yn.v[e]);
        } else if constexpr (GEN) {
          const int bse = p.tf[7] + i0 + p.nx * k;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F = g.fmap[bse + e];
            if (F >= 0) res.v[e] -= cur.py.v[e] * (yk.v[e] - y1(F));
          }
        }
      }
    }
    // z faces
    if ((k & 1) == 0) {
      // face (k-1 | k) leaves both aggregates: f = P_z (y_{k-1} - y_k) per cell
      Q4<R> f = zq4<R>();
      if (k > p.k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) f.v[e] = pzprev.v[e] * (yprev.v[e] - yk.v[e]);
      } else if (p.act) {
        if (hz_in) {
#pragma unroll
          for (int e = 0; e < 4; ++e) f.v[e] = hpz.v[e] * (yh.v[e] - yk.v[e]);
        } else if constexpr (GEN) {
          const int bse = p.tf[8] + i0 + p.nx * p.j;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F = g.fmap[bse + e];
            if (F >= 0) f.v[e] = Pz[F] * (y1(F) - yk.v[e]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) res.v[e] += f.v[e];
      if (k > p.k0) {   // the previous plane pair is complete
        agA -= f.v[0] + f.v[1];
        agB -= f.v[2] + f.v[3];
        pendA = agA;
        pendB = agB;
        pend = (k >> 1) - 1;
        if (odd && p.act) {
          lag[0][hu][0] = agA;
          lag[0][hu][1] = agB;
        }
      }
      agA = res.v[0] + res.v[1];
      agB = res.v[2] + res.v[3];
      if (GEN && k + 1 == p.nz && p.act) {   // a one-plane aggregate at the block's end
        if (wzp) {
          const Q4<R> yn = yv(ldq(rin, Pk - (p.nz - 1) * S), ldq(q, Pk - (p.nz - 1) * S),
                              ldq(Dinv, Pk - (p.nz - 1) * S));
          agA -= cur.pz.v[0] * (yk.v[0] - yn.v[0]) + cur.pz.v[1] * (yk.v[1] - yn.v[1]);
          agB -= cur.pz.v[2] * (yk.v[2] - yn.v[2]) + cur.pz.v[3] * (yk.v[3] - yn.v[3]);
        } else if constexpr (GEN) {
          const int bse = p.tf[9] + i0 + p.nx * p.j;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F = g.fmap[bse + e];
            const R fe = F >= 0 ? cur.pz.v[e] * (yk.v[e] - y1(F)) : R(0);
            if (e < 2) agA -= fe;
            else agB -= fe;
          }
        }
      }
    } else {
      agA += res.v[0] + res.v[1];
      agB += res.v[2] + res.v[3];
      yprev = yk;
      pzprev = cur.pz;
      if (k + 1 == p.k1 && p.act) {   // the run ends: face (k | k+1) to the next run or across the side
        if (zp) {
          const Q4<R> yn = yv(c0, c1, c2);
          agA -= cur.pz.v[0] * (yk.v[0] - yn.v[0]) + cur.pz.v[1] * (yk.v[1] - yn.v[1]);
          agB -= cur.pz.v[2] * (yk.v[2] - yn.v[2]) + cur.pz.v[3] * (yk.v[3] - yn.v[3]);
        } else if constexpr (GEN) {
          const int bse = p.tf[9] + i0 + p.nx * p.j;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F = g.fmap[bse + e];
            const R fe = F >= 0 ? cur.pz.v[e] * (yk.v[e] - y1(F)) : R(0);
            if (e < 2) agA -= fe;
            else agB -= fe;
          }
        }
      }
    }
  };
  for (int k = p.k0;;) {
    step(k, bufA, bufB);
    if (++k >= p.k1) break;
    step(k, bufB, bufA);
    if (++k >= p.k1) break;
  }
  // the run's last plane pair (and a pair completed at the last step)
  __syncthreads();
  if (pend >= 0 && p.act && !odd) emit(pendA, pendB, pend, 0);
  if (odd && p.act) {
    lag[1][hu][0] = agA;
    lag[1][hu][1] = agB;
  }
  __syncthreads();
  if (p.act && !odd) emit(agA, agB, (p.k1 - 1) >> 1, 1);
}

// ---------------------------------------------------------------------------------
// Direction update and M d with the d.q partials (the marching form of
// k_cg_spmv_q<R, 3, true>): the PCG's convergence test on the r.z, r.r partials of the
// V-cycle, beta = rz / rz_old, d = z + beta d_old, q = M d.  q of plane k - 1 is completed
// at step k (its face to plane k) and stored then.
template <typename R, int WGS, bool GEN>
__global__ void __launch_bounds__(WGS)
k_zm_spmv(Grid g, ZmTiles tl, const R* __restrict__ Pf, const R* __restrict__ zin, const R* __restrict__ dold,
          R* __restrict__ dnew, R* __restrict__ q, CgState* st, const double* __restrict__ partB,
          double* __restrict__ partA, int Gp, int par) {
  __shared__ Q4<R> ld[2][WGS];   // d of each unit's quad, by plane parity
  __shared__ R lpx[2][WGS];      // x-face coefficient at cell 3
  __shared__ Q4<R> lpy[2][WGS];  // P_y of the row (the face the row above crosses)
  const int done = st->done, kd = st->k, max_k = st->max_k;
  const double tol2bb = st->tol2 * st->bb, rz_old = st->rz[par ^ 1];
  const ZmPos p = zm_pos(g, tl);
  const int N = g.N, S = p.nx * p.ny;
  const R* __restrict__ Py = Pf + (size_t)N;
  const R* __restrict__ Pz = Pf + 2 * (size_t)N;
  const int u = threadIdx.x;
  const int i0 = 4 * p.xq;
  const bool wym = (p.wrap >> 2) & 1, wyp = (p.wrap >> 3) & 1, wzp = (p.wrap >> 5) & 1;
  // y faces crossed through memory: -y by the tile's first row, +y by its last
  const bool ym = p.act && (p.j > 0 ? p.jr == 0 : wym);
  const bool yp = p.act && (p.j + 1 < p.ny ? p.jr + 1 == p.RT : wyp);
  const int oym = p.j > 0 ? -p.nx : (p.ny - 1) * p.nx;
  const int oyp = p.j + 1 < p.ny ? p.nx : -(p.ny - 1) * p.nx;
  struct Ld {
    Q4<R> z, o, px, py, pz;
  };
  auto load = [&](int k) __attribute__((always_inline)) {
    Ld L;
    const int P = p.act ? p.base + S * k : 0;
    L.z = ldq(zin, P);
    L.o = ldq(dold, P);
    L.px = ldq(Pf, P);
    L.py = ldq(Py, P);
    L.pz = ldq(Pz, P);
    return L;
  };
  Ld bufA = load(p.k0), bufB;
  Q4<R> hz = zq4<R>(), ho = zq4<R>(), hpz = zq4<R>();
  const bool hz_in = p.k0 > 0 || ((p.wrap >> 4) & 1);
  if (p.act && hz_in) {
    const int Pm = p.base + S * (p.k0 > 0 ? p.k0 - 1 : p.nz - 1);
    hz = ldq(zin, Pm);
    ho = ldq(dold, Pm);
    hpz = ldq(Pz, Pm);
  }
  double t[2];
  zm_reduce_partials<2, WGS>(partB, Gp, t);
  if (done) return;
  const double rz = t[0], rr = t[1];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!std::isfinite(rz) || !std::isfinite(rr) || rr <= tol2bb || kd >= max_k) {
    if (lead) {
      st->rr = rr;
      st->iters = kd;
      if (!std::isfinite(rz) || !std::isfinite(rr)) st->status = PISO_E_NAN;
      else if (!(rr <= tol2bb)) st->status = PISO_NOT_CONVERGED;
      st->done = 1;
    }
    return;
  }
  const R beta = kd == 0 ? R(0) : (R)(rz / rz_old);
  if (lead) {
    st->rz[par] = rz;
    st->rr = rr;
  }
  auto d1 = [&](int F) __attribute__((always_inline)) { return zin[F] + beta * dold[F]; };
  auto dv = [&](const Q4<R>& a, const Q4<R>& b) __attribute__((always_inline)) {
    Q4<R> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o.v[e] = a.v[e] + beta * b.v[e];
    return o;
  };
  Q4<R> dprev = zq4<R>(), pzprev = zq4<R>(), Mprev = zq4<R>(), dzl = zq4<R>();
  double acc[1] = {0.0};
  // one plane: cur holds its loads, the next plane's go to nxt (two buffers used in
  // turn, so that no register copy waits for the loads in flight)
  auto step = [&](const int k, const Ld& cur, Ld& nxt) __attribute__((always_inline)) {
    const int bs = k & 1;
    const int Pk = p.act ? p.base + S * k : 0;
    // (a) neighbours in memory
    Q4<R> a0, a1, a3, b0, b1;
    if (ym) {
      a0 = ldq(zin, Pk + oym);
      a1 = ldq(dold, Pk + oym);
      a3 = ldq(Py, Pk + oym);
    }
    if (yp) {
      b0 = ldq(zin, Pk + oyp);
      b1 = ldq(dold, Pk + oyp);
    }
    const bool zp = p.act && k + 1 == p.k1 && (k + 1 < p.nz || wzp);
    if (zp) {
      const int Pn = k + 1 < p.nz ? Pk + S : Pk - (p.nz - 1) * S;
      dzl = dv(ldq(zin, Pn), ldq(dold, Pn));
    }
    // (b) the next plane
    nxt = load(k + 1 < p.k1 ? k + 1 : k);
    // (c) this plane
    Q4<R> dk, M;
#pragma unroll
    for (int e = 0; e < 4; ++e) dk.v[e] = cur.z.v[e] + beta * cur.o.v[e];
    if (p.act) stq(dnew, Pk, dk);
    ld[bs][u] = dk;
    lpx[bs][u] = cur.px.v[3];
    lpy[bs][u] = cur.py;
    __syncthreads();
    M = zq4<R>();
    if (p.act) {
      // x faces
      const Q4<R>& px = cur.px;
      {
        bool have = true;
        R dl = R(0), pl = R(0);
        if (i0 > 0) {
          if (!GEN || p.xl > 0) {
            dl = ld[bs][u - 1].v[3];
            pl = lpx[bs][u - 1];
          } else {
            dl = d1(Pk - 1);
            pl = Pf[Pk - 1];
          }
        } else if (p.wrap & 1) {
          if (!GEN || p.XQ == p.nxq) {
            dl = ld[bs][u + p.nxq - 1].v[3];
            pl = lpx[bs][u + p.nxq - 1];
          } else {
            dl = d1(Pk + p.nx - 1);
            pl = Pf[Pk + p.nx - 1];
          }
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[4] + p.j + p.ny * k];
          have = F >= 0;
          if (have) {
            dl = d1(F);
            pl = Pf[F];
          }
        }
        M.v[0] = px.v[0] * (dk.v[0] - dk.v[1]) + (have ? pl * (dk.v[0] - dl) : R(0));
      }
      M.v[1] = px.v[1] * (dk.v[1] - dk.v[2]) + px.v[0] * (dk.v[1] - dk.v[0]);
      M.v[2] = px.v[2] * (dk.v[2] - dk.v[3]) + px.v[1] * (dk.v[2] - dk.v[1]);
      {
        bool have = true;
        R dr = R(0);
        if (i0 + 4 < p.nx) {
          dr = (!GEN || p.xl + 1 < p.XQ) ? ld[bs][u + 1].v[0] : d1(Pk + 4);
        } else if (p.wrap & 2) {
          dr = (!GEN || p.XQ == p.nxq) ? ld[bs][u - (p.nxq - 1)].v[0] : d1(Pk + 4 - p.nx);
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[5] + p.j + p.ny * k];
          have = F >= 0;
          if (have) dr = d1(F);
        }
        M.v[3] = (have ? px.v[3] * (dk.v[3] - dr) : R(0)) + px.v[2] * (dk.v[3] - dk.v[2]);
      }
      // +y face: own coefficient
      if (p.j + 1 < p.ny || wyp) {
        const Q4<R> dn = (p.j + 1 < p.ny && p.jr + 1 < p.RT) ? ld[bs][u + p.XQ] : dv(b0, b1);
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += cur.py.v[e] * (dk.v[e] - dn.v[e]);
      } else if constexpr (GEN) {
        const int bse = p.tf[7] + i0 + p.nx * k;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += cur.py.v[e] * (dk.v[e] - d1(F));
        }
      }
      // -y face: coefficient stored at row j - 1
      if (p.j > 0 || wym) {
        Q4<R> dn, wn;
        if (p.jr > 0) {
          dn = ld[bs][u - p.XQ];
          wn = lpy[bs][u - p.XQ];
        } else {
          dn = dv(a0, a1);
          wn = a3;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += wn.v[e] * (dk.v[e] - dn.v[e]);
      } else if constexpr (GEN) {
        const int bse = p.tf[6] + i0 + p.nx * k;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += Py[F] * (dk.v[e] - d1(F));
        }
      }
      // -z face: the plane before (this run's, or read at the run's start)
      if (k > p.k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const R f = pzprev.v[e] * (dk.v[e] - dprev.v[e]);
          M.v[e] += f;
          Mprev.v[e] -= f;
        }
      } else if (hz_in) {
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += hpz.v[e] * (dk.v[e] - (hz.v[e] + beta * ho.v[e]));
      } else if constexpr (GEN) {
        const int bse = p.tf[8] + i0 + p.nx * p.j;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += Pz[F] * (dk.v[e] - d1(F));
        }
      }
      // plane k - 1 is complete
      if (k > p.k0) {
        stq(q, Pk - S, Mprev);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[0] += (double)dprev.v[e] * (double)Mprev.v[e];
      }
    }
    dprev = dk;
    pzprev = cur.pz;
    Mprev = M;
  };
  for (int k = p.k0;;) {
    step(k, bufA, bufB);
    if (++k >= p.k1) break;
    step(k, bufB, bufA);
    if (++k >= p.k1) break;
  }
  // +z face of the run's last plane
  if (p.act) {
    const int kl = p.k1 - 1;
    const int Pk = p.base + S * kl;
    if (kl + 1 < p.nz || wzp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) Mprev.v[e] += pzprev.v[e] * (dprev.v[e] - dzl.v[e]);
    } else {
      const int bse = p.tf[9] + i0 + p.nx * p.j;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int F = g.fmap[bse + e];
        if (F >= 0) Mprev.v[e] += pzprev.v[e] * (dprev.v[e] - d1(F));
      }
    }
    stq(q, Pk, Mprev);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[0] += (double)dprev.v[e] * (double)Mprev.v[e];
  }
  zm_write_partials<1, WGS>(acc, partA);
}

// ---------------------------------------------------------------------------------
// Prolongation and fine-level post-smoothing with the r.z, r.r partials (the marching
// form of k_mg_up0_q<R, 3>): with v = y + e_1[parent], z = v + omega D^-1 (r - M v).
template <typename R, int WGS, bool GEN>
__global__ void __launch_bounds__(WGS)
k_zm_up(Grid g, Grid g1, ZmTiles tl, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
        const R* __restrict__ y, const int* __restrict__ parent, const R* __restrict__ ec, R omega,
        R* __restrict__ z, double* __restrict__ partB, const CgState* st) {
  __shared__ Q4<R> lv[2][WGS];
  __shared__ R lpx[2][WGS];
  __shared__ Q4<R> lpy[2][WGS];
  if (st->done) return;
  const ZmPos p = zm_pos(g, tl);
  const int N = g.N, S = p.nx * p.ny;
  const R* __restrict__ Py = Pf + (size_t)N;
  const R* __restrict__ Pz = Pf + 2 * (size_t)N;
  const int u = threadIdx.x;
  const int i0 = 4 * p.xq;
  const int* tc = g1.tab + p.b * kTabStride;
  const int tc0 = tc[0], cx = tc[1], cy = tc[2];
  const bool wym = (p.wrap >> 2) & 1, wyp = (p.wrap >> 3) & 1, wzp = (p.wrap >> 5) & 1;
  const bool ym = p.act && (p.j > 0 ? p.jr == 0 : wym);
  const bool yp = p.act && (p.j + 1 < p.ny ? p.jr + 1 == p.RT : wyp);
  const int oym = p.j > 0 ? -p.nx : (p.ny - 1) * p.nx;
  const int oyp = p.j + 1 < p.ny ? p.nx : -(p.ny - 1) * p.nx;
  const int jm = p.j > 0 ? p.j - 1 : p.ny - 1, jp = p.j + 1 < p.ny ? p.j + 1 : 0;
  // coarse cell of aggregate row jj, plane kk (the quad's first aggregate; the second is +1)
  auto cbase = [&](int jj, int kk) __attribute__((always_inline)) { return tc0 + 2 * p.xq + cx * ((jj >> 1) + cy * (kk >> 1)); };
  // operand over a quad of this block from y and the two coarse values
  auto vq = [&](const Q4<R>& a, R e0, R e1) __attribute__((always_inline)) {
    Q4<R> o;
    o.v[0] = a.v[0] + e0;
    o.v[1] = a.v[1] + e0;
    o.v[2] = a.v[2] + e1;
    o.v[3] = a.v[3] + e1;
    return o;
  };
  // one cell of this block at (i, jj, kk), or (known = false) across a block side
  auto v1 = [&](int F, bool known, int i, int jj, int kk) __attribute__((always_inline)) {
    return y[F] + ec[known ? tc0 + (i >> 1) + cx * ((jj >> 1) + cy * (kk >> 1)) : parent[F]];
  };
  struct Ld {
    Q4<R> y, r, D, px, py, pz;
    R e0, e1;
  };
  auto load = [&](int k) __attribute__((always_inline)) {
    Ld L;
    const int P = p.act ? p.base + S * k : 0;
    const int cb = p.act ? cbase(p.j, k) : 0;
    L.y = ldq(y, P);
    L.r = ldq(r, P);
    L.D = ldq(Dinv, P);
    L.px = ldq(Pf, P);
    L.py = ldq(Py, P);
    L.pz = ldq(Pz, P);
    L.e0 = ec[cb];
    L.e1 = ec[cb + 1];
    return L;
  };
  Ld bufA = load(p.k0), bufB;
  const bool hz_in = p.k0 > 0 || ((p.wrap >> 4) & 1);
  const int km = p.k0 > 0 ? p.k0 - 1 : p.nz - 1;
  Q4<R> hy = zq4<R>(), hpz = zq4<R>();
  R he0 = R(0), he1 = R(0);
  if (p.act && hz_in) {
    const int Pm = p.base + S * km;
    const int cb = cbase(p.j, km);
    hy = ldq(y, Pm);
    hpz = ldq(Pz, Pm);
    he0 = ec[cb];
    he1 = ec[cb + 1];
  }
  Q4<R> vprev = zq4<R>(), pzprev = zq4<R>(), Mprev = zq4<R>(), rprev = zq4<R>(), Dprev = zq4<R>(),
        vzl = zq4<R>();
  double acc[2] = {0.0, 0.0};
  auto finish = [&](int P, const Q4<R>& v, const Q4<R>& M, const Q4<R>& rq, const Q4<R>& Dq) __attribute__((always_inline)) {
    Q4<R> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      o.v[e] = v.v[e] + omega * Dq.v[e] * (rq.v[e] - M.v[e]);
      acc[0] += (double)rq.v[e] * (double)o.v[e];
      acc[1] += (double)rq.v[e] * (double)rq.v[e];
    }
    stq(z, P, o);
  };
  // one plane: cur holds its loads, the next plane's go to nxt (two buffers used in
  // turn, so that no register copy waits for the loads in flight)
  auto step = [&](const int k, const Ld& cur, Ld& nxt) __attribute__((always_inline)) {
    const int bs = k & 1;
    const int Pk = p.act ? p.base + S * k : 0;
    // (a) neighbours in memory
    Q4<R> a0, a3, b0;
    R ae0, ae1, be0, be1;
    if (ym) {
      const int cb = cbase(jm, k);
      a0 = ldq(y, Pk + oym);
      a3 = ldq(Py, Pk + oym);
      ae0 = ec[cb];
      ae1 = ec[cb + 1];
    }
    if (yp) {
      const int cb = cbase(jp, k);
      b0 = ldq(y, Pk + oyp);
      be0 = ec[cb];
      be1 = ec[cb + 1];
    }
    const bool zp = p.act && k + 1 == p.k1 && (k + 1 < p.nz || wzp);
    if (zp) {
      const int kn = k + 1 < p.nz ? k + 1 : 0;
      const int cb = cbase(p.j, kn);
      vzl = vq(ldq(y, p.base + S * kn), ec[cb], ec[cb + 1]);
    }
    // (b) the next plane
    nxt = load(k + 1 < p.k1 ? k + 1 : k);
    // (c) this plane
    const Q4<R> vk = vq(cur.y, cur.e0, cur.e1);
    Q4<R> M;
    lv[bs][u] = vk;
    lpx[bs][u] = cur.px.v[3];
    lpy[bs][u] = cur.py;
    __syncthreads();
    M = zq4<R>();
    if (p.act) {
      const Q4<R>& px = cur.px;
      {
        bool have = true;
        R dl = R(0), pl = R(0);
        if (i0 > 0) {
          if (!GEN || p.xl > 0) {
            dl = lv[bs][u - 1].v[3];
            pl = lpx[bs][u - 1];
          } else {
            dl = v1(Pk - 1, true, i0 - 1, p.j, k);
            pl = Pf[Pk - 1];
          }
        } else if (p.wrap & 1) {
          if (!GEN || p.XQ == p.nxq) {
            dl = lv[bs][u + p.nxq - 1].v[3];
            pl = lpx[bs][u + p.nxq - 1];
          } else {
            dl = v1(Pk + p.nx - 1, true, p.nx - 1, p.j, k);
            pl = Pf[Pk + p.nx - 1];
          }
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[4] + p.j + p.ny * k];
          have = F >= 0;
          if (have) {
            dl = v1(F, false, 0, 0, 0);
            pl = Pf[F];
          }
        }
        M.v[0] = px.v[0] * (vk.v[0] - vk.v[1]) + (have ? pl * (vk.v[0] - dl) : R(0));
      }
      M.v[1] = px.v[1] * (vk.v[1] - vk.v[2]) + px.v[0] * (vk.v[1] - vk.v[0]);
      M.v[2] = px.v[2] * (vk.v[2] - vk.v[3]) + px.v[1] * (vk.v[2] - vk.v[1]);
      {
        bool have = true;
        R dr = R(0);
        if (i0 + 4 < p.nx) {
          dr = (!GEN || p.xl + 1 < p.XQ) ? lv[bs][u + 1].v[0] : v1(Pk + 4, true, i0 + 4, p.j, k);
        } else if (p.wrap & 2) {
          dr = (!GEN || p.XQ == p.nxq) ? lv[bs][u - (p.nxq - 1)].v[0] : v1(Pk + 4 - p.nx, true, 0, p.j, k);
        } else if constexpr (!GEN) {
          have = false;
        } else {
          const int F = g.fmap[p.tf[5] + p.j + p.ny * k];
          have = F >= 0;
          if (have) dr = v1(F, false, 0, 0, 0);
        }
        M.v[3] = (have ? px.v[3] * (vk.v[3] - dr) : R(0)) + px.v[2] * (vk.v[3] - vk.v[2]);
      }
      if (p.j + 1 < p.ny || wyp) {
        const Q4<R> vn = (p.j + 1 < p.ny && p.jr + 1 < p.RT) ? lv[bs][u + p.XQ] : vq(b0, be0, be1);
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += cur.py.v[e] * (vk.v[e] - vn.v[e]);
      } else if constexpr (GEN) {
        const int bse = p.tf[7] + i0 + p.nx * k;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += cur.py.v[e] * (vk.v[e] - v1(F, false, 0, 0, 0));
        }
      }
      if (p.j > 0 || wym) {
        Q4<R> vn, wn;
        if (p.jr > 0) {
          vn = lv[bs][u - p.XQ];
          wn = lpy[bs][u - p.XQ];
        } else {
          vn = vq(a0, ae0, ae1);
          wn = a3;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += wn.v[e] * (vk.v[e] - vn.v[e]);
      } else if constexpr (GEN) {
        const int bse = p.tf[6] + i0 + p.nx * k;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += Py[F] * (vk.v[e] - v1(F, false, 0, 0, 0));
        }
      }
      if (k > p.k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const R f = pzprev.v[e] * (vk.v[e] - vprev.v[e]);
          M.v[e] += f;
          Mprev.v[e] -= f;
        }
      } else if (hz_in) {
        const Q4<R> vn = vq(hy, he0, he1);
#pragma unroll
        for (int e = 0; e < 4; ++e) M.v[e] += hpz.v[e] * (vk.v[e] - vn.v[e]);
      } else if constexpr (GEN) {
        const int bse = p.tf[8] + i0 + p.nx * p.j;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int F = g.fmap[bse + e];
          if (F >= 0) M.v[e] += Pz[F] * (vk.v[e] - v1(F, false, 0, 0, 0));
        }
      }
      if (k > p.k0) finish(Pk - S, vprev, Mprev, rprev, Dprev);
    }
    vprev = vk;
    pzprev = cur.pz;
    Mprev = M;
    rprev = cur.r;
    Dprev = cur.D;
  };
  for (int k = p.k0;;) {
    step(k, bufA, bufB);
    if (++k >= p.k1) break;
    step(k, bufB, bufA);
    if (++k >= p.k1) break;
  }
  if (p.act) {
    const int kl = p.k1 - 1;
    const int Pk = p.base + S * kl;
    if (kl + 1 < p.nz || wzp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) Mprev.v[e] += pzprev.v[e] * (vprev.v[e] - vzl.v[e]);
    } else {
      const int bse = p.tf[9] + i0 + p.nx * p.j;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int F = g.fmap[bse + e];
        if (F >= 0) Mprev.v[e] += pzprev.v[e] * (vprev.v[e] - v1(F, false, 0, 0, 0));
      }
    }
    finish(Pk, vprev, Mprev, rprev, Dprev);
  }
  zm_write_partials<2, WGS>(acc, partB);
}

// ------------------------------------------------------------------ host

// Tiles of every block for work-groups of kZmWG threads: a tile is XQ x-quads (the whole
// row when it fits in half a work-group) by RT rows (even, RT * XQ <= kZmWG), run through
// KS planes (even); KS is chosen so that the grid holds about kZmTarget work-groups.
// PISO_ZM_TILE="xq,rt,ks" caps the three (tests use it to reach every halo path on small
// grids).
int zm_setup(piso_ctx* c) {
  c->zm_on = false;
  c->zm_force = false;
  if (c->dim != 3 || !c->quad || c->mg.empty()) return PISO_OK;
  if (const char* e = std::getenv("PISO_ZMARCH")) {
    if (e[0] == '0') return PISO_OK;
    c->zm_force = e[0] == '1';
  }
  int cap_xq = 1 << 30, cap_rt = 1 << 30, cap_ks = 1 << 30;
  if (const char* e = std::getenv("PISO_ZM_TILE")) {
    int a = 0, b = 0, k = 0;
    if (std::sscanf(e, "%d,%d,%d", &a, &b, &k) == 3 && a > 0 && b > 1 && k > 1) {
      cap_xq = a;
      cap_rt = b & ~1;
      cap_ks = k & ~1;
    }
  }
  ZmTiles& t = c->zm_tiles;
  t.nb = c->nblocks;
  t.off[0] = 0;
  for (int b = 0; b < c->nblocks; ++b) {
    const int* tb = &c->h_tab[(size_t)b * kTabStride];
    const int nxq = tb[1] / 4, ny = tb[2], nz = tb[3];
    int xq = std::min(std::min(nxq, kZmWG / 2), cap_xq);
    int rt = std::min(2 * (kZmWG / (2 * xq)), cap_rt);
    rt = std::min(rt, ny + (ny & 1));
    const int ntx = (nxq + xq - 1) / xq, nty = (ny + rt - 1) / rt;
    const double share = (double)tb[1] * ny * nz / c->N;
    const int want = std::max(1, (int)(kZmTarget * share) / (ntx * nty));
    int ks = (nz + want - 1) / want;
    ks = std::max(kZmMinPlanes, ks + (ks & 1));
    ks = std::min(ks, cap_ks);
    const int ntz = (nz + ks - 1) / ks;
    t.xq[b] = xq;
    t.rt[b] = rt;
    t.ks[b] = ks;
    t.ntx[b] = ntx;
    t.nty[b] = nty;
    t.off[b + 1] = t.off[b] + ntx * nty * ntz;
  }
  // the plain form (no code for sides connected to other blocks, rows split over tiles in
  // x, or one-row and one-plane aggregates): one block, every side a wall or wrapping onto
  // the block, whole rows per tile, even ny and nz
  t.plain = c->nblocks == 1 && t.xq[0] == c->h_tab[1] / 4 && c->h_tab[2] % 2 == 0 && c->h_tab[3] % 2 == 0;
  for (int side = 0; side < 6 && t.plain; ++side) {
    if ((c->h_tab[kTabWrap] >> side) & 1) continue;
    const int a = side / 2;
    const int faces = a == 0 ? c->h_tab[2] * c->h_tab[3] : (a == 1 ? c->h_tab[1] * c->h_tab[3] : c->h_tab[1] * c->h_tab[2]);
    for (int f = 0; f < faces; ++f)
      if (c->h_fmap[(size_t)c->h_tab[4 + side] + f] >= 0) {
        t.plain = false;
        break;
      }
  }
  // the groups' partial sums share the reduction buffers
  c->zm_on = t.off[c->nblocks] <= kRedGrid;
  return PISO_OK;
}

int zm_groups(const piso_ctx* c) { return c->zm_tiles.off[c->nblocks]; }

template <typename R>
int zm_launch_down(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout,
                   const R* dnew, const R* q, R* y, R* rc, CgState* st, const double* partA, int Gp, int par) {
  auto k = c->zm_tiles.plain ? k_zm_down<R, kZmWG, false> : k_zm_down<R, kZmWG, true>;
  launch_timed_wg(c, s, kTimeCgUpdateMg, k, zm_groups(c), kZmWG, c->grid, c->mg_g1, c->zm_tiles, Pf, Dinv, x, rin,
                  rout, dnew, q, y, (R)kMgOmega, rc, st, partA, Gp, par);
  return PISO_OK;
}

template <typename R>
int zm_launch_spmv(piso_ctx* c, hipStream_t s, const R* Pf, const R* z, const R* dold, R* dnew, R* q, CgState* st,
                   const double* partB, double* partA, int Gp, int par) {
  auto k = c->zm_tiles.plain ? k_zm_spmv<R, kZmWG, false> : k_zm_spmv<R, kZmWG, true>;
  launch_timed_wg(c, s, kTimeCgStencil, k, zm_groups(c), kZmWG, c->grid, c->zm_tiles, Pf, z, dold, dnew, q, st,
                  partB, partA, Gp, par);
  return PISO_OK;
}

template <typename R>
int zm_launch_up(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, const int* parent,
                 const R* e1, R* z, double* partB, const CgState* st) {
  auto k = c->zm_tiles.plain ? k_zm_up<R, kZmWG, false> : k_zm_up<R, kZmWG, true>;
  launch_timed_wg(c, s, kTimeMgUp0, k, zm_groups(c), kZmWG, c->grid, c->mg_g1, c->zm_tiles, Pf, Dinv, r, y, parent,
                  e1, (R)kMgOmega, z, partB, st);
  return PISO_OK;
}

#define PISO_ZM_INST(R)                                                                                          \
  template int zm_launch_down<R>(piso_ctx*, hipStream_t, const R*, const R*, R*, const R*, R*, const R*, const R*, \
                                 R*, R*, CgState*, const double*, int, int);                                     \
  template int zm_launch_spmv<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, R*, R*, CgState*,         \
                                 const double*, double*, int, int);                                              \
  template int zm_launch_up<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, const R*, const int*,        \
                               const R*, R*, double*, const CgState*);
PISO_ZM_INST(float)
PISO_ZM_INST(double)
#undef PISO_ZM_INST

}  // namespace piso
