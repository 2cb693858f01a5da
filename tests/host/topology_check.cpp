// Host check of the topology and argument validation of piso_create (block layouts of
// Sec. 2.2 / App. A.4), built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py: hand-written valid and invalid layouts with their
// expected codes, then seeded random descriptors that must each end in PISO_OK,
// PISO_E_ARG or PISO_E_TOPOLOGY with a consistent table and face map.
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2505_16992_amd/csrc/piso_topology.h"

using namespace piso;

namespace {

int failures = 0;
const double kDummy[1] = {1.0};   // T and J are not read by the topology

struct Layout {
  int dim = 3;
  std::vector<int> cells;   // [n_blocks][3]
  std::vector<piso_side_desc> sides;
};

piso_side_desc side(int b, int s, int kind, int other = 0, int t0n = 0, int t1n = 0) {
  piso_side_desc d{};
  d.block = b;
  d.side = s;
  d.kind = kind;
  d.begin[0] = d.begin[1] = 0;
  d.end[0] = t0n;
  d.end[1] = t1n;
  d.other_block = other;
  return d;
}

void extents(const Layout& L, int b, int s, int& t0n, int& t1n) {
  const int a = s / 2;
  int e[2] = {1, 1}, q = 0;
  for (int x = 0; x < L.dim; ++x)
    if (x != a) e[q++] = L.cells[3 * b + x];
  t0n = e[0];
  t1n = e[1];
}

// whole-side segment
void add(Layout& L, int b, int s, int kind, int other = 0) {
  int t0n, t1n;
  extents(L, b, s, t0n, t1n);
  L.sides.push_back(side(b, s, kind, other, t0n, t1n));
}

int run(const Layout& L, Topology* t, std::string* err, int precision = PISO_F64, const double* Tb = nullptr,
        const double* Jb = nullptr) {
  piso_domain_desc d{};
  d.dim = L.dim;
  d.n_blocks = (int)L.cells.size() / 3;
  d.n_sides = (int)L.sides.size();
  d.block_cells = L.cells.data();
  d.sides = L.sides.data();
  d.T = kDummy;
  d.J = kDummy;
  d.Tb = Tb;
  d.Jb = Jb;
  if (int rc = validate_desc(&d, precision, err)) return rc;
  return build_topology(&d, t, err);
}

void expect(const char* name, int got, int want) {
  if (got != want) {
    std::printf("FAIL %s: code %d, expected %d\n", name, got, want);
    ++failures;
  }
}

// every face-map entry set, connections in range, boundary faces numbered 0..NB-1
void check_tables(const char* name, const Topology& t) {
  std::vector<int> seen(t.NB, 0);
  for (int v : t.fmap) {
    if (v >= t.N || v < -t.NB) {
      std::printf("FAIL %s: face map entry %d out of range (N %d, NB %d)\n", name, v, t.N, t.NB);
      ++failures;
      return;
    }
    if (v < 0) seen[-1 - v]++;
  }
  for (int q = 0; q < t.NB; ++q)
    if (seen[q] != 1) {
      std::printf("FAIL %s: boundary face %d used %d times\n", name, q, seen[q]);
      ++failures;
      return;
    }
}

Layout box(int nx, int ny, int nz, bool px, bool py, bool pz, int dim = 3) {
  Layout L;
  L.dim = dim;
  L.cells = {nx, ny, dim == 3 ? nz : 1};
  const bool per[3] = {px, py, pz};
  for (int a = 0; a < dim; ++a)
    for (int s = 0; s < 2; ++s) add(L, 0, 2 * a + s, per[a] ? PISO_SIDE_CONNECT : PISO_SIDE_DIRICHLET, 0);
  return L;
}

void handwritten() {
  Topology t;
  std::string err;
  {
    // face metrics come as a pair
    Layout L = box(4, 4, 4, true, false, true);
    expect("face metrics: Tb without Jb", run(L, &t, &err, PISO_F64, kDummy, nullptr), PISO_E_ARG);
    expect("face metrics: Jb without Tb", run(L, &t, &err, PISO_F64, nullptr, kDummy), PISO_E_ARG);
    expect("face metrics: both", run(L, &t, &err, PISO_F64, kDummy, kDummy), PISO_OK);
  }
  {
    Layout L = box(6, 4, 4, true, true, true);
    expect("periodic box", run(L, &t, &err), PISO_OK);
    check_tables("periodic box", t);
    expect("periodic box N", t.N, 96);
    expect("periodic box colourable", t.ilu_ok, 1);
  }
  {
    Layout L = box(6, 5, 4, true, true, true);
    expect("odd periodic box", run(L, &t, &err), PISO_OK);
    expect("odd periodic box not colourable", t.ilu_ok, 0);
  }
  {
    Layout L = box(8, 6, 4, true, false, true);
    expect("channel", run(L, &t, &err), PISO_OK);
    check_tables("channel", t);
    expect("channel NB", t.NB, 2 * 8 * 4);
  }
  {
    Layout L = box(5, 7, 1, false, false, false, 2);
    expect("cavity", run(L, &t, &err), PISO_OK);
    check_tables("cavity", t);
    expect("cavity NB", t.NB, 2 * (5 + 7));
  }
  // two blocks joined along x, walls elsewhere
  auto two = [](int ny1) {
    Layout L;
    L.dim = 2;
    L.cells = {3, 4, 1, 5, ny1, 1};
    add(L, 0, 1, PISO_SIDE_CONNECT, 1);
    add(L, 1, 0, PISO_SIDE_CONNECT, 0);
    add(L, 0, 0, PISO_SIDE_DIRICHLET);
    add(L, 1, 1, PISO_SIDE_DIRICHLET);
    for (int b = 0; b < 2; ++b)
      for (int s = 2; s < 4; ++s) add(L, b, s, PISO_SIDE_DIRICHLET);
    return L;
  };
  {
    Layout L = two(4);
    expect("two blocks", run(L, &t, &err), PISO_OK);
    check_tables("two blocks", t);
    expect("two blocks N", t.N, 32);
  }
  {
    Layout L = two(5);
    expect("non-conformal", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, false, false, false, 2);
    L.sides.pop_back();
    expect("uncovered side", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, false, false, false, 2);
    L.sides.push_back(L.sides[0]);
    expect("face covered twice", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, false, false, false, 2);
    L.sides[1].end[0] = 9;
    expect("range outside the side", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, false, false, false, 2);
    L.sides[2].side = 7;
    expect("bad side", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, false, false, false, 2);
    L.sides[2].kind = 9;
    expect("bad kind", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 1, true, false, false, 2);
    L.sides[0].other_begin[0] = 2;   // the connection leaves the other side
    expect("connection leaves block", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = two(4);
    L.sides[1].other_block = 1;   // block 1's -x side leads to itself: not reciprocal
    expect("non-reciprocal", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
  {
    Layout L = box(4, 4, 4, false, false, false);
    expect("bad precision", run(L, &t, &err, 7), PISO_E_ARG);
    L.dim = 4;
    expect("bad dim", run(L, &t, &err), PISO_E_ARG);
    Layout E;
    E.dim = 3;
    expect("no blocks", run(E, &t, &err), PISO_E_ARG);
    expect("null descriptor", validate_desc(nullptr, PISO_F64, &err), PISO_E_ARG);
    Layout M;
    M.dim = 2;
    for (int b = 0; b < 17; ++b) M.cells.insert(M.cells.end(), {2, 2, 1});
    M.sides.push_back(side(0, 0, PISO_SIDE_DIRICHLET, 0, 2, 1));
    expect("too many blocks", run(M, &t, &err), PISO_E_ARG);
  }
  {
    Layout L = box(0, 4, 1, false, false, false, 2);
    expect("empty block", run(L, &t, &err), PISO_E_TOPOLOGY);
  }
}

void fuzz(int n) {
  std::mt19937 rng(12345);
  auto R = [&](int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); };
  int ok = 0, bad = 0;
  for (int it = 0; it < n; ++it) {
    Layout L;
    L.dim = R(2, 3);
    const int B = R(1, 3);
    for (int b = 0; b < B; ++b) L.cells.insert(L.cells.end(), {R(0, 5), R(0, 5), L.dim == 3 ? R(0, 4) : R(0, 2)});
    const int ns = R(0, 14);
    for (int q = 0; q < ns; ++q) {
      piso_side_desc d{};
      d.block = R(-1, B);
      d.side = R(-1, 2 * L.dim);
      d.kind = R(-1, 2);
      d.begin[0] = R(-1, 3);
      d.begin[1] = R(-1, 3);
      d.end[0] = R(-1, 6);
      d.end[1] = R(-1, 6);
      d.other_block = R(-1, B);
      d.other_begin[0] = R(-2, 4);
      d.other_begin[1] = R(-2, 4);
      L.sides.push_back(d);
    }
    // half the time, whole-side segments that mostly form a valid layout
    if (it & 1) {
      L.sides.clear();
      for (int b = 0; b < B; ++b) {
        if (L.cells[3 * b] < 1) L.cells[3 * b] = 1;
        if (L.cells[3 * b + 1] < 1) L.cells[3 * b + 1] = 1;
        if (L.cells[3 * b + 2] < 1 || L.dim == 2) L.cells[3 * b + 2] = 1;
        for (int s = 0; s < 2 * L.dim; ++s) add(L, b, s, R(0, 1), R(0, B - 1));
      }
    }
    Topology t;
    std::string err;
    const int rc = run(L, &t, &err, R(-1, 3));
    if (rc == PISO_OK) {
      ++ok;
      check_tables("fuzz", t);
    } else if (rc == PISO_E_ARG || rc == PISO_E_TOPOLOGY) {
      ++bad;
      if (err.empty()) {
        std::printf("FAIL fuzz: code %d without a message\n", rc);
        ++failures;
      }
    } else {
      std::printf("FAIL fuzz: unexpected code %d\n", rc);
      ++failures;
    }
  }
  std::printf("fuzz: %d valid, %d rejected\n", ok, bad);
  if (ok == 0) {
    std::printf("FAIL fuzz: no valid layout generated\n");
    ++failures;
  }
}

}  // namespace

int main() {
  handwritten();
  fuzz(20000);
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "passed", failures);
  return failures ? 1 : 0;
}
