// coarse.hpp -- the coarse term of Eq. 6 (coarse.hip): vertex space, the
// assembled coarse operator and its Chebyshev solve, on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "sem_internal.hpp"

namespace sem {

constexpr int kMaxCoarseDotBlocks = 1024;  // partial pairs of the coarse dot, at most

struct CoarseSpace {
    int k = 0;               // Chebyshev steps
    double frac = 0.0;       // a = frac * b
    double a = 0.0, b = 0.0; // Chebyshev interval of D0^-1 A0
    double inv_theta = 0.0;
    std::vector<double> c1, c2;  // per-step Chebyshev coefficients
    int64_t nvert = 0;       // element vertices (periodic images merged)
    int64_t n_coarse = 0;    // vertices with a non-zero masked hat function
    int64_t nnz = 0;
    int dot_blocks = 0;      // workgroups of the coarse dot (partial pairs)
    // device
    int32_t *evert = nullptr;   // [E][8] vertex of each element corner
    int32_t *v_off = nullptr;   // [nvert+1] vertex -> element-corner entries
    int32_t *v_idx = nullptr;   //   e*8 + c, ascending
    double *qw = nullptr;       // [2][N+1] 1-D hat weights at the GLL nodes
    int32_t *a_off = nullptr, *a_col = nullptr;  // A0, CSR
    double *a_val = nullptr;
    double *d0inv = nullptr;    // [nvert] 1/diag(A0), 0 where the vertex is not a coarse unknown
    double *partial8 = nullptr; // [E][8] element restriction sums
    double *r0 = nullptr, *z0 = nullptr, *res = nullptr, *d = nullptr, *tmp = nullptr;
    std::vector<void *> allocations;
};

// Work vectors of one solve's coarse term: the mesh's own (coarse_work_own,
// for its single-mesh solves) or a batched slot's, carved from one buffer of
// coarse_work_doubles values in this order: element restriction sums [E][8],
// r0, z0, res, d, tmp [nvert each], the coarse dot's partial pairs and their
// sum rz (the last two only in carved sets).
struct CoarseWork {
    double *partial8, *r0, *z0, *res, *d, *tmp, *dot, *rz;
};
int64_t coarse_work_doubles(const CoarseSpace *C, int64_t E);
CoarseWork coarse_work_carve(const CoarseSpace *C, int64_t E, double *base);
CoarseWork coarse_work_own(const CoarseSpace *C);
template <typename T>
void coarse_restrict_w(sem_mesh *m, const CoarseWork &W, const T *r, const T *inv, hipStream_t s);
int coarse_solve_w(sem_mesh *m, const CoarseWork &W, double *dot_pairs, const PcgState *st, hipStream_t s);
// add: z += masked P z0; else z = masked P z0
void coarse_prolong_w(sem_mesh *m, const CoarseWork &W, double *z, bool add, hipStream_t s);
// z = masked P z0 rounded to FP32 (a mixed-precision batched slot's correction)
void coarse_prolong_w32(sem_mesh *m, const CoarseWork &W, float *z, hipStream_t s);

// Builds the coarse space of the mesh's current operator (synchronises s).
CoarseSpace *coarse_build(sem_mesh *m, int k, double frac, hipStream_t s);
void coarse_free(CoarseSpace *C);
// CG update (precision T) with the restriction fused in: r -= alpha w,
// partial pairs of <r,r>, <r, inv r> into `partial` (returns their count),
// element restriction sums of the new r.  Skips when st->done.
// with_rz = false: the second entry of each pair is 0 (another local
// preconditioner supplies <r, z>).
template <typename T>
int coarse_update(sem_mesh *m, T *r, const T *w, const T *inv, const PcgState *st, double *partial, bool with_rz,
                  hipStream_t s);
// element restriction sums of r (live nodes: inv > 0)
template <typename T>
void coarse_restrict(sem_mesh *m, const T *r, const T *inv, hipStream_t s);
// from the element sums: r0 = P^T r, z0 = C(A0) r0, and when dot_pairs is
// given the (0, r0.z0) pairs there (returns their count, C->dot_blocks);
// kernels skip when st->done.
int coarse_solve(sem_mesh *m, double *dot_pairs, const PcgState *st, hipStream_t s);
// z += masked P z0 (z0 from the last coarse_solve)
void coarse_prolong_add(sem_mesh *m, double *z, hipStream_t s);
// z = inv r
void launch_jacobi(int64_t n, const double *inv, const double *r, double *z, hipStream_t s);

}  // namespace sem
