// Host-side geometry preprocessing for the voxel Stokes solver.
#pragma once

#include <cstdint>
#include <vector>

namespace stokes {

struct Geometry {
    int N = 0;
    int64_t n3 = 0;
    int64_t nfluid_in = 0;       // fluid voxels of the mask as given
    int64_t nfluid = 0;          // fluid voxels that remain
    int64_t nsurf = 0;           // solid voxels with a fluid face neighbour
    int ncomp_all = 0;           // fluid components of the mask as given
    int ncomp_kept = 0;          // components that remain
    std::vector<uint8_t> fluid;        // remaining fluid, one byte per voxel
    std::vector<uint16_t> label;       // remaining component id per voxel, 0xFFFF in solid
    std::vector<int64_t> comp_size;    // voxels per remaining component
};

// Label the periodic 6-connected fluid components of `mask` and, unless
// keep_all is set, remove the components in which no closed path winds
// through the box with a non-zero component along `force` (their velocity is
// zero in the exact solution).  Labels are only filled when at most 65535
// components remain.  Also counts the surface voxels (eq. surface_area).
void preprocess(const uint8_t* mask, int N, const double force[3], bool keep_all, Geometry& g);

}  // namespace stokes
