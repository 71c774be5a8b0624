// Displacement-p distance-k probing colourings (paper Background, Probing).
#pragma once

#include <cstdint>
#include <vector>

namespace fs {

// Greedy colouring in site order (site = x + Lx (y + Ly (z + Lz t))): each site
// takes the smallest colour held by no earlier site within periodic taxicab
// distance k of its z-displaced neighbours x + p z^ or x - p z^.  Returns the
// colour per site; *n_colours the number used.
std::vector<int32_t> probing_colours(const int dims[4], int p, int k, int* n_colours);

}  // namespace fs
