// axgs64.hip -- FP64 instantiations of the fused operator and gather-scatter
// (axgs_impl.hpp), with the launch helpers shared by both precisions.
#include "axgs_impl.hpp"

namespace sem {

size_t axgs_lds_bytes_impl(int N, int epw, int nx, bool y_onchip, size_t elem)
{
    const size_t P = (size_t)N + 1, P3 = P * P * P, K = N >= 1 ? (size_t)N - 1 : 0;
    size_t v = (size_t)epw * 3 * P3 + (size_t)epw * P * P * K + P * K;
    if (y_onchip) v += ((size_t)nx * N + 1) * K;
    return v * elem;
}

size_t axgs_lds_bytes(int N, int epw, int nx, bool y_onchip, size_t elem)
{
    return axgs_lds_bytes_impl(N, epw, nx, y_onchip, elem);
}

template <>
hipError_t launch_axgs<double>(int N, int mode, const AxParams<double> &a, const AxgsLattice &L, hipStream_t s,
                               int64_t *grid)
{
    return launch_axgs_impl<double>(N, mode, a, L, s, grid);
}

template <>
int axgs_blocks_per_cu<double>(int N, int mode, bool helm, int epw, size_t lds)
{
    return axgs_blocks_per_cu_impl<double>(N, mode, helm, epw, lds);
}

// this code object's copy of the derivative tables
hipError_t upload_axgs64_dtables(const double *d64, const float *d32, hipStream_t s)
{
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D64), d64, sizeof(double) * kDTableSize, 0,
                                          hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D32), d32, sizeof(float) * kDTableSize, 0, hipMemcpyHostToDevice, s);
}

}  // namespace sem
