// Host-side topology of a block layout (Sec. 2.2, App. A.4 of arXiv 2505.16992): the
// block table and per-side face map the kernels index, built from a domain descriptor
// and validated (coverage, ranges, conformity, reciprocity), plus the red-black colouring
// of the ILU(0) preconditioner.  Plain C++ without HIP, so that it also builds on its
// own for the host sanitizer check (tests/host/).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/piso.h"

namespace piso {

constexpr int kMaxBlocks = 16;
constexpr int kTabStride = 20;           // ints per block in the device block table
constexpr int kTabWrap = 16;             // entry: bit (2 * axis + side) set when that side of the
                                         // block joins the opposite side of the same block
                                         // cell for cell (periodicity)
constexpr int kTabColour = 17;           // entry: parity of the block in the red-black colouring
                                         // (cell colour = (i + j + k + parity) & 1)

// Block table, kTabStride ints per block:
//   [0] offset  [1] nx  [2] ny  [3] nz  [4..9] offset of each side in the face map
//   [10,11] magic for /nx (lo, hi)  [12] shift  [13,14] magic for /(nx*ny)  [15] shift
//   [16] periodic-side bits (kTabWrap)  [17] colour parity (kTabColour)  [18, 19] unused
// Face map: per side face, the neighbour cell (>= 0) or -1 - (Dirichlet face index).
struct Topology {
  int N = 0, NB = 0;
  std::vector<int> tab, fmap;
  bool ilu_ok = false;   // two colours tile the grid with every face between colours
};

// Multiplier and shift for the exact division n / d of the kernels' cell indexing
// (fast_div): m = ceil(2^(31+l) / d), l = ceil(log2 d).
inline void div_magic(uint32_t d, uint32_t& lo, uint32_t& hi, int& shift) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t num = 1ull << (31 + l);
  const uint64_t m = (num + d - 1) / d;
  lo = (uint32_t)(m & 0xffffffffu);
  hi = (uint32_t)(m >> 32);
  shift = 31 + l;
}

// Argument checks of piso_create before the topology: descriptor pointers, dim,
// block count, precision.  PISO_OK or PISO_E_ARG with the message in *err.
int validate_desc(const piso_domain_desc* d, int precision, std::string* err);

// PISO_OK, or PISO_E_TOPOLOGY / PISO_E_ARG with the message in *err.
int build_topology(const piso_domain_desc* d, Topology* out, std::string* err);

}  // namespace piso
