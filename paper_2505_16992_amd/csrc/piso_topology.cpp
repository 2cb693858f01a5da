// Host-side topology of a block layout: see piso_topology.h.
#include "piso_topology.h"

#include <array>
#include <climits>
#include <string>
#include <vector>

namespace piso {

namespace {

int topo_fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

void tangential_extent(const int n[3], int side, int dim, int& t0n, int& t1n) {
  const int axis = side / 2;
  int e[2] = {1, 1}, q = 0;
  for (int a = 0; a < dim; ++a)
    if (a != axis) e[q++] = n[a];
  t0n = e[0];
  t1n = e[1];
}

}  // namespace

int validate_desc(const piso_domain_desc* desc, int precision, std::string* err) {
  if (!desc || !desc->block_cells || !desc->sides || !desc->T || !desc->J)
    return topo_fail(err, PISO_E_ARG, "null descriptor field");
  if (desc->dim != 2 && desc->dim != 3) return topo_fail(err, PISO_E_ARG, "dim must be 2 or 3");
  if (desc->n_blocks < 1 || desc->n_blocks > kMaxBlocks) return topo_fail(err, PISO_E_ARG, "n_blocks must be 1..16");
  if (desc->n_sides < 0) return topo_fail(err, PISO_E_ARG, "n_sides must be >= 0");
  if (precision < PISO_F64 || precision > PISO_MIXED) return topo_fail(err, PISO_E_ARG, "bad precision");
  if ((desc->Tb == nullptr) != (desc->Jb == nullptr))
    return topo_fail(err, PISO_E_ARG, "face metrics: Tb and Jb are given together or not at all");
  return PISO_OK;
}

// Build the block table and the per-side face map; validates coverage, ranges,
// conformity and reciprocity.
int build_topology(const piso_domain_desc* d, Topology* c, std::string* err) {
  const int D = d->dim, B = d->n_blocks;
  std::vector<int> off(B + 1, 0);
  std::vector<std::array<int, 3>> n(B);
  for (int b = 0; b < B; ++b) {
    for (int a = 0; a < 3; ++a) n[b][a] = d->block_cells[3 * b + a];
    if (n[b][0] < 1 || n[b][1] < 1 || n[b][2] < 1 || (D == 2 && n[b][2] != 1))
      return topo_fail(err, PISO_E_TOPOLOGY, "block " + std::to_string(b) + ": bad cell counts");
    const long long cells = (long long)n[b][0] * n[b][1] * n[b][2];
    if ((long long)off[b] + cells >= INT_MAX / 2) return topo_fail(err, PISO_E_ARG, "too many cells");
    off[b + 1] = off[b] + (int)cells;
  }
  c->N = off[B];
  c->tab.assign((size_t)B * kTabStride, 0);
  int fm = 0;
  for (int b = 0; b < B; ++b) {
    int* t = &c->tab[(size_t)b * kTabStride];
    t[0] = off[b];
    t[1] = n[b][0];
    t[2] = n[b][1];
    t[3] = n[b][2];
    for (int s = 0; s < 2 * D; ++s) {
      int t0n, t1n;
      tangential_extent(n[b].data(), s, D, t0n, t1n);
      t[4 + s] = fm;
      fm += t0n * t1n;
    }
    uint32_t lo, hi;
    int sh;
    div_magic((uint32_t)n[b][0], lo, hi, sh);
    t[10] = (int)lo; t[11] = (int)hi; t[12] = sh;
    div_magic((uint32_t)(n[b][0] * n[b][1]), lo, hi, sh);
    t[13] = (int)lo; t[14] = (int)hi; t[15] = sh;
  }
  c->fmap.assign((size_t)fm, INT_MIN);
  auto cell = [&](int b, int i, int j, int k) { return off[b] + i + n[b][0] * (j + n[b][1] * k); };
  auto from_t = [&](int axis, int along, int t0, int t1, int& i, int& j, int& k) {
    if (axis == 0) { i = along; j = t0; k = t1; }
    else if (axis == 1) { i = t0; j = along; k = t1; }
    else { i = t0; j = t1; k = along; }
  };
  int nbf = 0;
  for (int si = 0; si < d->n_sides; ++si) {
    const piso_side_desc& sd = d->sides[si];
    if (sd.block < 0 || sd.block >= B || sd.side < 0 || sd.side >= 2 * D)
      return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": bad block or side");
    const int b = sd.block, a = sd.side / 2, s = sd.side % 2;
    int t0n, t1n;
    tangential_extent(n[b].data(), sd.side, D, t0n, t1n);
    if (!(0 <= sd.begin[0] && sd.begin[0] < sd.end[0] && sd.end[0] <= t0n && 0 <= sd.begin[1] &&
          sd.begin[1] < sd.end[1] && sd.end[1] <= t1n))
      return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": range outside the side");
    const int along = s == 0 ? 0 : n[b][a] - 1;
    for (int t1 = sd.begin[1]; t1 < sd.end[1]; ++t1) {
      for (int t0 = sd.begin[0]; t0 < sd.end[0]; ++t0) {
        int i, j, k;
        from_t(a, along, t0, t1, i, j, k);
        const int slot = c->tab[(size_t)b * kTabStride + 4 + sd.side] + t0 + t0n * t1;
        if (c->fmap[slot] != INT_MIN)
          return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": face covered twice");
        if (sd.kind == PISO_SIDE_DIRICHLET) {
          c->fmap[slot] = -1 - nbf++;
        } else if (sd.kind == PISO_SIDE_CONNECT) {
          const int ob = sd.other_block;
          if (ob < 0 || ob >= B) return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": bad other block");
          int ot0n, ot1n;
          tangential_extent(n[ob].data(), 2 * a + (1 - s), D, ot0n, ot1n);
          const int o0 = t0 - sd.begin[0] + sd.other_begin[0], o1 = t1 - sd.begin[1] + sd.other_begin[1];
          if (o0 < 0 || o0 >= ot0n || o1 < 0 || o1 >= ot1n)
            return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": connection leaves the other block");
          const int oalong = s == 1 ? 0 : n[ob][a] - 1;
          int oi, oj, ok;
          from_t(a, oalong, o0, o1, oi, oj, ok);
          c->fmap[slot] = cell(ob, oi, oj, ok);
        } else {
          return topo_fail(err, PISO_E_TOPOLOGY, "segment " + std::to_string(si) + ": unknown kind");
        }
      }
    }
  }
  c->NB = nbf;
  // coverage and reciprocity
  for (int b = 0; b < B; ++b) {
    for (int side = 0; side < 2 * D; ++side) {
      const int a = side / 2, s = side % 2;
      int t0n, t1n;
      tangential_extent(n[b].data(), side, D, t0n, t1n);
      const int along = s == 0 ? 0 : n[b][a] - 1;
      for (int t1 = 0; t1 < t1n; ++t1)
        for (int t0 = 0; t0 < t0n; ++t0) {
          const int slot = c->tab[(size_t)b * kTabStride + 4 + side] + t0 + t0n * t1;
          const int v = c->fmap[slot];
          if (v == INT_MIN)
            return topo_fail(err, PISO_E_TOPOLOGY, "block " + std::to_string(b) + " side " + std::to_string(side) +
                                                ": face not covered");
          if (v >= 0) {
            // the other cell's opposite face must lead back here
            int ob = 0;
            while (ob + 1 < B && v >= off[ob + 1]) ++ob;
            const int L = v - off[ob];
            const int oi = L % n[ob][0], oj = (L / n[ob][0]) % n[ob][1], ok = L / (n[ob][0] * n[ob][1]);
            const int opos[3] = {oi, oj, ok};
            const int oside = 2 * a + (1 - s);
            const int oalong = (1 - s) == 0 ? 0 : n[ob][a] - 1;
            if (opos[a] != oalong) return topo_fail(err, PISO_E_TOPOLOGY, "connection does not land on a side");
            int ot0n, ot1n;
            tangential_extent(n[ob].data(), oside, D, ot0n, ot1n);
            int ot0 = 0, ot1 = 0, q = 0;
            for (int aa = 0; aa < 3; ++aa)
              if (aa != a) (q++ == 0 ? ot0 : ot1) = opos[aa];
            const int oslot = c->tab[(size_t)ob * kTabStride + 4 + oside] + ot0 + ot0n * ot1;
            int i, j, k;
            from_t(a, along, t0, t1, i, j, k);
            if (c->fmap[oslot] != cell(b, i, j, k))
              return topo_fail(err, PISO_E_TOPOLOGY, "non-reciprocal (non-conformal) connection at block " +
                                                  std::to_string(b) + " side " + std::to_string(side));
          }
        }
    }
  }
  // sides that wrap onto the opposite side of the same block cell for cell (periodicity):
  // the kernels then index them arithmetically instead of through the face map
  for (int b = 0; b < B; ++b) {
    int bits = 0;
    for (int side = 0; side < 2 * D; ++side) {
      const int a = side / 2, s = side % 2;
      int t0n, t1n;
      tangential_extent(n[b].data(), side, D, t0n, t1n);
      bool wraps = true;
      for (int t1 = 0; t1 < t1n && wraps; ++t1)
        for (int t0 = 0; t0 < t0n && wraps; ++t0) {
          const int slot = c->tab[(size_t)b * kTabStride + 4 + side] + t0 + t0n * t1;
          int i, j, k;
          from_t(a, s ? 0 : n[b][a] - 1, t0, t1, i, j, k);
          wraps = c->fmap[slot] == cell(b, i, j, k);
        }
      if (wraps) bits |= 1 << side;
    }
    c->tab[(size_t)b * kTabStride + kTabWrap] = bits;
  }
  // red-black colouring for the ILU(0) preconditioner of the velocity solve: colour
  // (i + j + k + parity_b) & 1 with one parity per block, propagated across the block
  // connections so that every face joins two colours; where no choice does (an odd
  // periodic extent, an odd cycle of blocks) ILU(0) is unavailable
  {
    std::vector<int> par(B, -1);
    bool ok = true;
    for (int b0 = 0; b0 < B && ok; ++b0) {
      if (par[b0] >= 0) continue;
      par[b0] = 0;
      std::vector<int> todo{b0};
      while (!todo.empty() && ok) {
        const int b = todo.back();
        todo.pop_back();
        for (int side = 0; side < 2 * D && ok; ++side) {
          const int a = side / 2, s = side % 2;
          int t0n, t1n;
          tangential_extent(n[b].data(), side, D, t0n, t1n);
          for (int t1 = 0; t1 < t1n && ok; ++t1)
            for (int t0 = 0; t0 < t0n && ok; ++t0) {
              const int v = c->fmap[c->tab[(size_t)b * kTabStride + 4 + side] + t0 + t0n * t1];
              if (v < 0) continue;
              int i, j, k;
              from_t(a, s ? n[b][a] - 1 : 0, t0, t1, i, j, k);
              int ob = 0;
              while (ob + 1 < B && v >= off[ob + 1]) ++ob;
              const int L = v - off[ob];
              const int osum = L % n[ob][0] + (L / n[ob][0]) % n[ob][1] + L / (n[ob][0] * n[ob][1]);
              const int need = (i + j + k + par[b] + 1 + osum) & 1;   // the other cell's colour differs
              if (par[ob] < 0) {
                par[ob] = need;
                todo.push_back(ob);
              } else if (par[ob] != need) {
                ok = false;
              }
            }
        }
      }
    }
    c->ilu_ok = ok;
    for (int b = 0; b < B; ++b) c->tab[(size_t)b * kTabStride + kTabColour] = par[b] > 0 ? 1 : 0;
  }
  return PISO_OK;
}


}  // namespace piso
