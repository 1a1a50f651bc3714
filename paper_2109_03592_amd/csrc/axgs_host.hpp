// axgs_host.hpp -- host state of the fused operator and gather-scatter.
#pragma once

#include <vector>

#include "axgs.hpp"
#include "sem_internal.hpp"

namespace sem {

// One precision's launch shape and its residual gather-scatter plan.
struct AxgsShape {
    int ready = 0;
    int epw = 0, lines_per_wg = 0, y_onchip = 0;
    int64_t grid = 0;
    AxgsLattice L{};
    // residual plan (device): CSR over the ids the kernel does not finish
    GsPlan res{};
    int64_t res_copies = 0;
    int32_t *res_off = nullptr, *res_idx = nullptr;
    bool owns_plan = false;  // false: shares the other precision's arrays
};

struct AxgsSpace {
    int enabled = 0;  // opt-in: measured slower than the two launches on the pipe
    int req_epw = 0, req_lines = 0;  // 0: automatic
    AxgsShape shape[2];              // FP64, FP32
};

hipError_t upload_axgs_dtables(const double *d64, const float *d32, hipStream_t s);
bool axgs_onchip(const HostMesh &h, int lines_per_wg, bool y_onchip, int64_t a, int64_t b, int64_t c);
void axgs_residual_plan(const HostMesh &h, int lines_per_wg, bool y_onchip, std::vector<int32_t> &off,
                        std::vector<int32_t> &idx);
AxgsLattice axgs_lattice(const HostMesh &h, int epw, int lines_per_wg, bool y_onchip);
int axgs_pick_lines(int64_t n_lines, int64_t resident, int64_t grid_cap);

}  // namespace sem
