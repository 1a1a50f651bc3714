// axgs_impl.hpp -- the local operator (Algorithm 1) fused with the
// direct-stiffness summation of every face that stays inside one workgroup
// (section 2: the global exchange of element face values after the local
// matrix-free work).  Included by axgs64.hip and axgs32.hip, one precision
// each.
//
// A workgroup owns whole x-lines of elements, lines_per_wg consecutive ones
// (y-neighbours within a z-plane), and walks them tile by tile in element
// order.  After the operator has produced a tile's columns of w in registers:
//
//  * a node on an x-face between two elements of one line, on a y-face
//    between two lines of the workgroup, or on the x-y edge between four of
//    its elements, and on an interior t-plane (0 < k < N), is summed here.
//    Its copies are met in ascending element order, which is ascending local
//    index, so the running sum starting from 0 adds them in exactly the order
//    of the full gather-scatter: the result is the same bits.  The partial
//    sum passes from one copy's lane to the next through LDS (within a tile),
//    through a pending x-face (to the next tile of the line) or through a
//    line buffer (to the next line); the lane of the last copy writes the sum
//    to every copy.
//  * a node on a Dirichlet face is written as 0 by each copy.
//  * every other node is written as computed; a residual plan of the
//    gather-scatter (the ids with copies in the t-planes k = 0, N, across
//    workgroups or across a periodic x- or y-boundary) completes them.
#pragma once

#include "axgs.hpp"
#include "operator.hpp"

namespace sem {

template <int N>
struct AxgsDims {
    static constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    static constexpr int K = N - 1;  // interior t-planes
};

size_t axgs_lds_bytes_impl(int N, int epw, int nx, bool y_onchip, size_t elem);

// status of one side of a column's face: no neighbour, neighbour met in this
// workgroup, neighbour elsewhere (or across a periodic boundary)
enum : int { kSideNone = 0, kSideOn = 1, kSideOff = 2 };

template <typename T, int N, int MODE, bool HELM>
__global__ __launch_bounds__(512) void axgs_kernel(AxParams<T> a, AxgsLattice L)
{
    using Dm = AxgsDims<N>;
    constexpr int P = Dm::P, P2 = Dm::P2, P3 = Dm::P3, K = Dm::K;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);

    if (MODE >= 2 && a.st->done) return;

    const int epw = a.epw;
    const int tid = threadIdx.x;
    const int el = tid / P2;
    const int ij = tid - el * P2;
    const int i = ij % P, j = ij / P;
    const bool inblk = el < epw;
    const int slot = inblk ? el : epw - 1;
    T *su = sm + (size_t)slot * 3 * P3;
    // behind the tile slots: the partial sums of the tile's shared columns,
    // the last element's i = N column (pending for the next tile of the
    // line) and the y = N faces of the previous line
    T *stage = sm + (size_t)epw * 3 * P3;       // [epw][P2][K]
    T *xpend = stage + (size_t)epw * P2 * K;    // [P][K]
    T *ybuf = xpend + (size_t)P * K;            // [nx N + 1][K]
    T *my_stage = stage + ((size_t)slot * P2 + ij) * K;
    const T *__restrict__ D = dtable<T>(N);
    __shared__ T sDt[lane_rows_lds<T, N>()];
    LaneRows<T, N> R;
    R.load(D, i, j, sDt);
    T beta = 0, alpha = 0;
    if (MODE >= 2) {
        beta = (T)a.st->beta;
        alpha = (T)a.st->alpha;
    }
    double dot = 0.0;

    // lattice position of this lane's column, fixed for the whole launch
    const int nx = L.nx, ny = L.ny;
    const bool mxl = i == 0 && !L.periodic_x && L.mask_x_lo, mxh = i == N && !L.periodic_x && L.mask_x_hi;
    const bool myl = j == 0 && !L.periodic_y && L.mask_y_lo, myh = j == N && !L.periodic_y && L.mask_y_hi;
    const int nz = (int)(L.n_lines / ny);
    const int l0 = (int)((int64_t)blockIdx.x * L.lines_per_wg);
    const int l1 = (int)min((int64_t)l0 + L.lines_per_wg, L.n_lines);
    // the walk: lines l0..l1-1, tiles 0..tiles_per_line-1 of each (counters
    // advanced in step, no divisions inside the loop)
    int line = l0, t = 0, ey = l0 % ny, ez = l0 / ny;
    const int nq = (l1 - l0) * L.tiles_per_line;
    for (int q = 0; q < nq; ++q) {
        const int ex = t * epw + el;
        const bool active = inblk && ex < nx;
        const int64_t e = (int64_t)line * nx + ex;
        // sides of this lane's column and its mask
        int xlo = kSideNone, xhi = kSideNone, ylo = kSideNone, yhi = kSideNone;
        if (i == 0) xlo = ex > 0 ? kSideOn : (L.periodic_x ? kSideOff : kSideNone);
        if (i == N) xhi = ex < nx - 1 ? kSideOn : (L.periodic_x ? kSideOff : kSideNone);
        if (j == 0)
            ylo = ey > 0 ? ((line == l0 || !L.y_onchip) ? kSideOff : kSideOn) : (L.periodic_y ? kSideOff : kSideNone);
        if (j == N)
            yhi = ey < ny - 1 ? ((line == l1 - 1 || !L.y_onchip) ? kSideOff : kSideOn)
                              : (L.periodic_y ? kSideOff : kSideNone);
        const bool masked = (mxl && ex == 0) || (mxh && ex == nx - 1) || (myl && ey == 0) || (myh && ey == ny - 1);
        const bool mz_lo = ez == 0 && L.mask_z_lo, mz_hi = ez == nz - 1 && L.mask_z_hi;
        const bool off = xlo == kSideOff || xhi == kSideOff || ylo == kSideOff || yhi == kSideOff;
        const bool shared = xlo == kSideOn || xhi == kSideOn || ylo == kSideOn || yhi == kSideOn;
        // chain: this column's interior nodes are summed here
        const bool chain = active && !masked && !off && shared;
        const int yslot = (ex * N + i) * K;
        T *__restrict__ col = a.out + (active ? e : 0) * P3 + ij;
        // each output as it is formed: written (0 on a Dirichlet face), or the
        // running sum of its node staged for the epilogue
        auto sink = [&](int k, T w) {
            if (!active) return;
            if (masked || (k == 0 && mz_lo) || (k == N && mz_hi)) {
                st_stream(T(0), col + k * P2);
                return;
            }
            if (!chain || k == 0 || k == N) {
                st_stream(w, col + k * P2);
                return;
            }
            const int kk = k - 1;
            T part = w;
            if (xlo == kSideOn) {
                if (el == 0) part = xpend[j * K + kk] + w;  // else the predecessor is in this tile
            } else if (ylo == kSideOn) {
                part = ybuf[yslot + kk] + w;
            } else {
                part = T(0) + w;  // first copy: the sum starts from 0
            }
            my_stage[kk] = part;
        };
        // the tile of the operator kernel, so that the results keep its bits
        if constexpr (plane_tile<T, N, MODE>())
            ax_tile_planes<T, N, MODE, HELM>(R, D, su, e, active, inblk, i, j, a.G, a.in, a.out, a.invdiag, a.p,
                                             beta, a.x, alpha, dot, a.h1, a.h2b, sink);
        else
            ax_tile<T, N, MODE, HELM>(R, D, su, e, active, inblk, i, j, a.G, a.in, a.out, a.invdiag, a.p, beta,
                                         a.x, alpha, dot, a.h1, a.h2b, nullptr, nullptr, sink);
        __syncthreads();
        if constexpr (K > 0) {
            if (chain) {
                const T *pred = (xlo == kSideOn && el > 0) ? stage + ((size_t)(el - 1) * P2 + N + P * j) * K : nullptr;
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int k = kk + 1;
                    T part = my_stage[kk];
                    if (pred) part = pred[kk] + part;
                    if (xhi == kSideOn) {
                        if (el == epw - 1) xpend[j * K + kk] = part;  // else the successor reads the stage
                    } else if (yhi == kSideOn) {
                        ybuf[yslot + kk] = part;
                    } else {
                        // last copy: the sum goes to every copy
                        st_stream(part, col + k * P2);
                        if (xlo == kSideOn) st_stream(part, col - P3 + N + k * P2);
                        if (ylo == kSideOn) {
                            T *cy = col - (int64_t)nx * P3 + P * N;
                            st_stream(part, cy + k * P2);
                            if (xlo == kSideOn) st_stream(part, cy - P3 + N + k * P2);
                        }
                    }
                }
            }
        }
        if (++t == L.tiles_per_line) {
            t = 0;
            ++line;
            if (++ey == ny) {
                ey = 0;
                ++ez;
            }
        }
    }
    if (MODE != 0) {
        double v[1] = {dot};
        block_reduce_store<1>(v, a.partial, 1);
    }
}

template <typename T, int MODE, bool HELM>
static const void *axgs_fn(int N)
{
    switch (N) {
#define SEM_AXGS_FN(n) \
    case n: return reinterpret_cast<const void *>(&axgs_kernel<T, n, MODE, HELM>);
        SEM_AXGS_FN(2) SEM_AXGS_FN(3) SEM_AXGS_FN(4) SEM_AXGS_FN(5) SEM_AXGS_FN(6) SEM_AXGS_FN(7)
        SEM_AXGS_FN(8) SEM_AXGS_FN(9) SEM_AXGS_FN(10) SEM_AXGS_FN(11) SEM_AXGS_FN(12)
#undef SEM_AXGS_FN
    default: return nullptr;
    }
}

template <typename T, int MODE, bool HELM>
static hipError_t launch_axgs_mode(int N, const AxParams<T> &a, const AxgsLattice &L, hipStream_t s, int64_t *grid)
{
    const int threads = ax_block_threads(N, a.epw);
    const size_t lds = axgs_lds_bytes_impl(N, a.epw, L.nx, L.y_onchip != 0, sizeof(T));
    if (threads > 512 || L.lines_per_wg < 1 || L.n_lines < 1 || L.nx < 1) return hipErrorInvalidConfiguration;
    const int64_t blocks = (L.n_lines + L.lines_per_wg - 1) / L.lines_per_wg;
    if (blocks > a.grid_cap) return hipErrorInvalidConfiguration;
    switch (N) {
#define SEM_AXGS_CASE(n)                                                                                     \
    case n:                                                                                                  \
        hipLaunchKernelGGL((axgs_kernel<T, n, MODE, HELM>), dim3((unsigned)blocks), dim3(threads), lds, s, a, \
                           L);                                                                               \
        break;
        SEM_AXGS_CASE(2) SEM_AXGS_CASE(3) SEM_AXGS_CASE(4) SEM_AXGS_CASE(5) SEM_AXGS_CASE(6) SEM_AXGS_CASE(7)
        SEM_AXGS_CASE(8) SEM_AXGS_CASE(9) SEM_AXGS_CASE(10) SEM_AXGS_CASE(11) SEM_AXGS_CASE(12)
#undef SEM_AXGS_CASE
    default: return hipErrorInvalidValue;
    }
    if (grid) *grid = blocks;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axgs_impl(int N, int mode, const AxParams<T> &a, const AxgsLattice &L, hipStream_t s,
                            int64_t *grid)
{
    if (!axgs_order_supported(N)) return hipErrorInvalidValue;
    if (mode == 0) return a.h1 ? launch_axgs_mode<T, 0, true>(N, a, L, s, grid)
                               : launch_axgs_mode<T, 0, false>(N, a, L, s, grid);
    if (mode == 2) return a.h1 ? launch_axgs_mode<T, 2, true>(N, a, L, s, grid)
                               : launch_axgs_mode<T, 2, false>(N, a, L, s, grid);
    return hipErrorInvalidValue;
}

template <typename T>
int axgs_blocks_per_cu_impl(int N, int mode, bool helm, int epw, size_t lds)
{
    const void *fn = nullptr;
    if (mode == 0) fn = helm ? axgs_fn<T, 0, true>(N) : axgs_fn<T, 0, false>(N);
    else if (mode == 2) fn = helm ? axgs_fn<T, 2, true>(N) : axgs_fn<T, 2, false>(N);
    if (!fn) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, ax_block_threads(N, epw), lds) != hipSuccess)
        return 0;
    return per_cu;
}

}  // namespace sem
