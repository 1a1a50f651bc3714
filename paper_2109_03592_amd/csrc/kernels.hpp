// kernels.hpp -- launch wrappers of the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sem_internal.hpp"

namespace sem {

// Derivative matrices of all orders 1..SEM_MAX_ORDER, concatenated.
constexpr int dtable_offset_host(int N)
{
    int o = 0;
    for (int n = 1; n < N; ++n) o += (n + 1) * (n + 1);
    return o;
}
__host__ __device__ constexpr int dtable_offset(int N)
{
    return N <= 1 ? 0 : dtable_offset(N - 1) + N * N;
}
constexpr int kDTableSize = dtable_offset_host(SEM_MAX_ORDER + 1);

template <typename T>
struct AxParams {
    int64_t E;             // elements
    int epw;               // elements per workgroup (element tile)
    int grid_cap;          // persistent grid: at most this many workgroups
    const T *G;            // [E][6][P^3]
    const T *in;           // u (modes 0/1) or r (mode 2)
    T *out;                // w
    double *partial;       // per-workgroup dot partials (modes 1/2)
    const T *invdiag;      // mode 2
    T *p;                  // mode 2: search direction, updated in place
    T *x;                  // mode 2: iterate, receives the previous step alpha*p
    const PcgState *st;    // mode 2: alpha, beta and the done flag
    const T *h1;           // Helmholtz: h1 per local point (nullptr: Poisson)
    const T *h2b;          // Helmholtz: h2*B per local point (with h1)
    // mode 3: mode 2 plus the coarse correction in the prologue (FP64 coarse data)
    const int32_t *evert;  // [E][8] vertex of each element corner
    const double *z0;      // coarse solution per vertex
    const double *cq;      // [2][N+1] 1-D hat weights at the GLL nodes
};

constexpr int kMaxPrecondOrder = 12;  // the coarse term, the Schwarz local solves and modes 3-5

int ax_block_threads(int N, int epw);
// dynamic LDS of an operator launch (mode: 0-5)
size_t ax_lds_bytes(int N, int epw, size_t elem, int mode);
hipError_t upload_dtables(const double *d64, const float *d32, hipStream_t s);
int vec_blocks(int64_t n);
int update_blocks(int64_t n);  // workgroups of the PCG update (one partial pair each)

// grid (may be null) receives the workgroups launched: the count of per-
// workgroup dot partials (modes 1-5)
template <typename T>
hipError_t launch_ax(int N, int mode, const AxParams<T> &a, hipStream_t s, int64_t *grid = nullptr);
// false when the mesh has a periodic axis of one element or the counts do not fit
template <typename T>
// force_stream: the row-streaming kernel at every order 2..7 (by default only
// at N = 7 with at least 2048 row walks, where it is the faster one)
hipError_t launch_gs_lattice(const GsLattice &L, T *v, const PcgState *st, hipStream_t s, bool force_stream = false);

template <typename T>
hipError_t launch_gs(const GsPlan &plan, const int32_t *off, const int32_t *idx, T *v, bool zero_only,
                     const PcgState *st, hipStream_t s);
hipError_t launch_scale(int64_t n, const double *a, const double *b, double *out, hipStream_t s);
hipError_t launch_scatter(int64_t n, const int32_t *gid, const double *vg, double *out, hipStream_t s);
hipError_t launch_residual(int64_t n, const double *b, const double *w, double *r, hipStream_t s);
hipError_t launch_to_fp32_scaled(int64_t n, const double *r, const double *scal, float *out, hipStream_t s);
hipError_t launch_axpy_fp32(int64_t n, const float *d, const double *scal, double *x, hipStream_t s);
hipError_t launch_fp64_to_fp32(int64_t n, const double *a, float *out, hipStream_t s);
template <typename T>
hipError_t launch_dot_unique(int64_t n, const T *a, const T *b, const uint8_t *mult, double *partial,
                             double *out, hipStream_t s);
template <typename T>
hipError_t launch_pcg_init(int64_t n, const T *r, const T *inv, const uint8_t *mult, double *partial,
                           PcgState *st, double stop2, int limit, hipStream_t s);
// the two halves of launch_pcg_init: vec_blocks(n) partial pairs, and the
// reduction of `pairs` pairs into the CG start state
template <typename T>
hipError_t launch_pcg_init_partials(int64_t n, const T *r, const T *inv, const uint8_t *mult, double *partial,
                                    hipStream_t s);
hipError_t launch_reduce_init(const double *partial, int64_t pairs, PcgState *st, double stop2, int limit,
                              hipStream_t s);
template <typename T>
hipError_t launch_pcg_update(int64_t n, const PcgState *st, T *r, const T *w, const T *inv, const uint8_t *mult,
                             double *partial, hipStream_t s);
// the update element by element (N >= 3: at least one full wavefront per
// element); update_elem_blocks(E) partial pairs
int update_elem_blocks(int64_t E);
template <typename T>
hipError_t launch_pcg_update_elem(int N, int64_t E, const PcgState *st, T *r, const T *w, const T *inv,
                                  const uint8_t *mult, double *partial, hipStream_t s);
// the element-wise update with the gather-scatter of w folded in (lattice
// meshes, Jacobi; FP64 and FP32); update_elem_blocks(E) partial pairs
template <typename T>
hipError_t launch_pcg_update_gs(const GsLattice &L, int N, int64_t E, const PcgState *st, T *r, const T *w,
                                const T *inv, const uint8_t *mult, double *partial, hipStream_t s);
template <typename T>
hipError_t launch_pcg_finish(int64_t n, const PcgState *st, T *x, const T *p, hipStream_t s);
hipError_t launch_reduce_sigma(const double *partial, int64_t n, PcgState *st, hipStream_t s);
hipError_t launch_reduce_rho(const double *partial, int64_t n, PcgState *st, hipStream_t s);
hipError_t launch_reduce_scalar(const double *partial, int64_t n, double *out, hipStream_t s);
// diagonal of the local Helmholtz operator (h1 == nullptr: 1, h2b == nullptr: 0)
hipError_t launch_helm_diag(int N, int64_t E, const double *G, const double *h1, const double *h2b, double *diag,
                            hipStream_t s);
// out = v > 0 ? 1/v : 0
hipError_t launch_invert_positive(int64_t n, const double *v, double *out, hipStream_t s);
hipError_t launch_fill(int64_t n, double value, double *out, hipStream_t s);

}  // namespace sem
