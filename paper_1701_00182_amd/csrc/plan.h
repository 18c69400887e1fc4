// Host-only structure of a factorisation: the planar bisection cluster tree of
// a plane, the red/black level schedule over the planes and the validation of
// the options.  Plain C++ (no device code), so that it also builds and runs
// under the host sanitizers.
#pragma once
#include <vector>

#include "acr.h"

namespace acr {

// Planar bisection cluster tree of an nx x ny plane (Sections 2.1.1, 3.1).
// Split across the longer side (x on ties), first half ceil(side/2); the tree is
// complete (every box of a depth is split while any box of that depth holds
// more than `leaf` points); points are numbered leaf by leaf, row-major inside.
struct Tree {
  int nx = 0, ny = 0, M = 0, L = 0, leaf = 0, leaf_max = 0;
  std::vector<std::vector<int>> off, sz;  // [depth][segment]
  std::vector<int> perm;                   // cluster position -> j * nx + i
  // Returns false when the rule would have to split a single point.
  bool build(int nx_, int ny_, int leaf_);
  int nblk() const { return (1 << (L + 1)) - 2; }
  static int bid(int d, int s) { return (1 << (d + 1)) - 2 + s; }
};

// Red/black schedule (Section 2.2.2, Eq. permuted_system and Eq. next_step):
// the planes alive at each level, in order; positions 0, 2, 4, ... of a level
// are eliminated, the others are kept and renumbered for the next level, until
// one plane is left (returned in `last`).
std::vector<std::vector<int>> level_schedule(int nplanes, int* last);

// Option checks shared by every entry point that takes acr_options_t.
bool options_valid(const acr_options_t* o);

// Fills `info` and the non-null arrays of the structure queries (acr.h);
// elim[i][q] tells whether plane sched[i][q] was eliminated at level i;
// perm_src (may be null: the tree's own) supplies the permutation.
void fill_structure(const Tree& tr, const std::vector<std::vector<int>>& sched,
                    const std::vector<std::vector<char>>& elim, int last, const int32_t* perm_src,
                    acr_structure_t* info, int32_t* perm, int32_t* node_offset, int32_t* node_size,
                    int32_t* level_size, int32_t* sched_plane, int32_t* sched_elim);

}  // namespace acr
