// axgs.hpp -- the local operator fused with the direct-stiffness summation of
// the faces that one workgroup holds (launch wrappers of axgs_impl.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace sem {

// The structured element lattice as the fused kernel walks it.  Elements are
// numbered x fastest, so an x-line of nx elements is contiguous and the lines
// (ey, ez) follow each other in y, then z.  Each workgroup takes
// lines_per_wg consecutive lines and walks them tile by tile (epw elements of
// one line per tile).
struct AxgsLattice {
    int nx, ny;              // elements per x-line, x-lines per z-plane
    int64_t n_lines;         // ny * nz
    int lines_per_wg;        // consecutive lines per workgroup
    int tiles_per_line;      // ceil(nx / epw)
    int periodic_x, periodic_y;
    int64_t ext0, ext1;      // global lattice extents in x and y
    int mask_x_lo, mask_x_hi, mask_y_lo, mask_y_hi;  // Dirichlet lattice faces
    int mask_z_lo, mask_z_hi;
    int64_t ext2;
    int y_onchip;            // 1: faces between lines of one workgroup are summed on-chip
};

// Dynamic LDS of the fused kernel: the operator's tile slots, the x-face
// exchange of one tile, the x-face pending across tiles and the y-face line
// buffer (when y_onchip).
size_t axgs_lds_bytes(int N, int epw, int nx, bool y_onchip, size_t elem);

// Orders the fused kernel is built for (the others run the operator and the
// full gather-scatter as two launches).
constexpr int kAxgsMinOrder = 2, kAxgsMaxOrder = 12;
inline bool axgs_order_supported(int N) { return N >= kAxgsMinOrder && N <= kAxgsMaxOrder; }

// mode 0: w = A_L u with the on-chip sums; mode 2: the CG operator (prologue
// x, p updates and the p.Ap partial per workgroup, taken before any sum).
// grid receives the workgroups launched (= dot partials of mode 2).
template <typename T>
hipError_t launch_axgs(int N, int mode, const AxParams<T> &a, const AxgsLattice &L, hipStream_t s,
                       int64_t *grid = nullptr);
// resident workgroups of the fused kernel per compute unit (occupancy query)
template <typename T>
int axgs_blocks_per_cu(int N, int mode, bool helm, int epw, size_t lds);

}  // namespace sem
