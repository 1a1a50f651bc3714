// axgs32.hip -- FP32 instantiations of the fused operator and gather-scatter
// (axgs_impl.hpp).
#include "axgs_impl.hpp"

namespace sem {

template <>
hipError_t launch_axgs<float>(int N, int mode, const AxParams<float> &a, const AxgsLattice &L, hipStream_t s,
                              int64_t *grid)
{
    return launch_axgs_impl<float>(N, mode, a, L, s, grid);
}

template <>
int axgs_blocks_per_cu<float>(int N, int mode, bool helm, int epw, size_t lds)
{
    return axgs_blocks_per_cu_impl<float>(N, mode, helm, epw, lds);
}

// this code object's copy of the derivative tables
hipError_t upload_axgs32_dtables(const double *d64, const float *d32, hipStream_t s)
{
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D64), d64, sizeof(double) * kDTableSize, 0,
                                          hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D32), d32, sizeof(float) * kDTableSize, 0, hipMemcpyHostToDevice, s);
}

}  // namespace sem
