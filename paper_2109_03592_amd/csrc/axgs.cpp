// axgs.cpp -- host side of the fused operator and gather-scatter: the launch
// shape (elements per tile, x-lines per workgroup) and the residual plan of
// the global ids the fused kernel leaves to a gather-scatter launch.
#include <algorithm>
#include <cstring>

#include "axgs_host.hpp"

namespace sem {

hipError_t upload_axgs64_dtables(const double *d64, const float *d32, hipStream_t s);
hipError_t upload_axgs32_dtables(const double *d64, const float *d32, hipStream_t s);

hipError_t upload_axgs_dtables(const double *d64, const float *d32, hipStream_t s)
{
    hipError_t e = upload_axgs64_dtables(d64, d32, s);
    if (e != hipSuccess) return e;
    return upload_axgs32_dtables(d64, d32, s);
}

// Does the fused kernel finish global node (a, b, c) itself?  Mirrors the
// kernel's per-column decision: the node must lie on an interior t-plane of
// its elements (c not a multiple of N); an x-face it lies on must join two
// elements of one x-line (not the periodic seam); a y-face must join two
// lines of the same workgroup (not the periodic seam).  Dirichlet nodes are
// set to 0 by the kernel and never reach a plan.
bool axgs_onchip(const HostMesh &h, int lines_per_wg, bool y_onchip, int64_t a, int64_t b, int64_t c)
{
    const int N = h.N;
    if (c % N == 0) return false;
    if (a % N == 0 && (a == 0 || a == (int64_t)h.nel[0] * N) && h.periodic[0]) return false;
    if (b % N == 0) {
        if (b == 0 || b == (int64_t)h.nel[1] * N) {
            if (h.periodic[1]) return false;
        } else {
            if (!y_onchip) return false;
            const int64_t ez = c / N, ey = b / N;
            const int64_t hi = ey + (int64_t)h.nel[1] * ez, lo = hi - 1;
            if (lo / lines_per_wg != hi / lines_per_wg) return false;
        }
    }
    return true;
}

void axgs_residual_plan(const HostMesh &h, int lines_per_wg, bool y_onchip, std::vector<int32_t> &off,
                        std::vector<int32_t> &idx)
{
    off.clear();
    idx.clear();
    const int64_t gx = h.ext[0], gy = h.ext[1];
    for (int64_t id = 0; id < h.gs_n_sum; ++id) {
        const int32_t q0 = h.gs_off[id], q1 = h.gs_off[id + 1];
        const int64_t g = h.gid[h.gs_idx[q0]];
        const int64_t a = g % gx, b = (g / gx) % gy, c = g / (gx * gy);
        if (axgs_onchip(h, lines_per_wg, y_onchip, a, b, c)) continue;
        off.push_back((int32_t)idx.size());
        for (int32_t q = q0; q < q1; ++q) idx.push_back(h.gs_idx[q]);
    }
    off.push_back((int32_t)idx.size());
}

AxgsLattice axgs_lattice(const HostMesh &h, int epw, int lines_per_wg, bool y_onchip)
{
    const sem_mesh_desc &d = h.desc;
    int faces = d.dirichlet_faces;
    if (faces < 0) {
        faces = 0;
        for (int ax = 0; ax < 3; ++ax)
            if (!h.periodic[ax]) faces |= 3 << (2 * ax);
    }
    auto bit = [&](int ax, int hi) { return (!h.periodic[ax] && ((faces >> (2 * ax + hi)) & 1)) ? 1 : 0; };
    AxgsLattice L{};
    L.nx = h.nel[0];
    L.ny = h.nel[1];
    L.n_lines = (int64_t)h.nel[1] * h.nel[2];
    L.lines_per_wg = lines_per_wg;
    L.tiles_per_line = (h.nel[0] + epw - 1) / epw;
    L.periodic_x = h.periodic[0];
    L.periodic_y = h.periodic[1];
    L.ext0 = h.ext[0];
    L.ext1 = h.ext[1];
    L.ext2 = h.ext[2];
    L.mask_x_lo = bit(0, 0);
    L.mask_x_hi = bit(0, 1);
    L.mask_y_lo = bit(1, 0);
    L.mask_y_hi = bit(1, 1);
    L.mask_z_lo = bit(2, 0);
    L.mask_z_hi = bit(2, 1);
    L.y_onchip = y_onchip ? 1 : 0;
    return L;
}

// Smallest line count per workgroup whose launch fits the resident
// workgroups in the fewest rounds: the makespan in lines is
// ceil(ceil(n_lines / L) / resident) * L.
int axgs_pick_lines(int64_t n_lines, int64_t resident, int64_t grid_cap)
{
    if (resident < 1) resident = 1;
    int64_t best = 0, best_cost = 0;
    for (int64_t Lw = 1; Lw <= n_lines; ++Lw) {
        const int64_t wgs = (n_lines + Lw - 1) / Lw;
        if (wgs > grid_cap) continue;
        const int64_t cost = (wgs + resident - 1) / resident * Lw;
        // equal cost: the larger count (more y-faces summed on chip)
        if (best == 0 || cost <= best_cost) {
            best = Lw;
            best_cost = cost;
        }
        if (wgs <= resident) break;  // larger counts only lengthen the one round
    }
    return (int)std::max<int64_t>(best, 1);
}

}  // namespace sem
