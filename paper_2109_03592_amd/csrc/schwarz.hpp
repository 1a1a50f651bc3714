// schwarz.hpp -- overlapping Schwarz local solves of Eq. 6 (schwarz.hip):
// each element extended by one node layer, its separable local matrix
// inverted by fast diagonalisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "sem_internal.hpp"

namespace sem {

enum SideKind { kSideInterior = 0, kSideDirichlet = 1, kSideNeumann = 2 };

constexpr int kMaxSchwarzPairs = 8192;  // partial pairs of the local solves, at most

// 1-D factors of one direction of one extended element: the generalised
// eigenvectors S (S^T B S = I, S^T A S = diag(lam)) of the 1-D stiffness A and
// lumped mass B assembled on the element (length ell) and the neighbours
// that exist, restricted to the kept extended indices lo .. lo+count-1.
// S is count x count, row = kept position, column = mode.
void fdm_1d(int N, const std::vector<double> &xi, const std::vector<double> &w, const std::vector<double> &D,
            double ell, int left, int right, std::vector<double> &S, std::vector<double> &lam, int &lo, int &count);

struct SchwarzSpace {
    int n = 0;                 // N + 3: extended nodes per direction (padded)
    int64_t n_table = 0;       // distinct 1-D factors
    int dirichlet = 0;         // resolved Dirichlet face bits
    int32_t *tidx = nullptr;   // [E][3] table entry per direction
    double *table = nullptr;   // [n_table][n*n + n]: S padded (zero rows/columns), then lam (1 beyond count)
    int32_t *meta = nullptr;   // [n_table][2]: lo, count
    double *zext = nullptr;    // [E][n^3] local solutions on the extended elements
    double *zs = nullptr;      // [nL] assembled Schwarz output
    std::vector<void *> allocations;
};

SchwarzSpace *schwarz_build(sem_mesh *m, hipStream_t s);
void schwarz_free(SchwarzSpace *S);
// z = sum_k R_k^T A_k^-1 R_k r (masked, continuous); with `pairs`, the
// (0, <r, z>) partial pairs there (returns their count).  Kernels skip when
// st->done.
int schwarz_apply(sem_mesh *m, const double *r, double *z, double *pairs, const PcgState *st, hipStream_t s);

}  // namespace sem
