// batch.hpp -- device structures of batched (many-mesh) CG.
//
// A "slot" is one solve: a mesh's read-only data (geometric factors, Jacobi
// diagonal, multiplicities, gather-scatter plan) plus the solve's own vectors
// and CG state.  A "group" is a set of slots advanced together; its work
// tables list (slot, tile) items for the operator, (slot, id-chunk) items for
// the gather-scatter and (slot, point-chunk) items for vector kernels.  The
// persistent kernels walk those tables, so any mix of orders and sizes runs
// in one launch per CG phase, and every per-slot reduction sums that slot's
// item partials in a fixed order -- a slot's arithmetic does not depend on
// which other slots share the launch.
#pragma once

#include <cstdint>

#include "sem_internal.hpp"

namespace sem {

constexpr int kBatchBlock = 256;       // threads per workgroup of every batched kernel
constexpr int kGsChunk = 256;          // gather-scatter ids per item
constexpr int kVecChunk = 256 * 8;     // vector points per item

struct Item {
    int32_t slot;
    int32_t local;  // tile / chunk index inside the slot
};

struct SlotDesc {
    int N;
    int pad;
    int64_t E, nL;
    const void *G[2];   // [0] FP64, [1] FP32 geometric factors [E][6][P^3]
    const void *inv[2]; // inverse assembled diagonal
    const uint8_t *mult;
    const int32_t *gs_off, *gs_idx;
    int64_t gs_n_sum, gs_n_ids;
    GsLattice gsl;      // the lattice gather-scatter of the mesh, used when gs_lattice
    int gs_lattice;
    int pad2;
    const double *b;    // right-hand side (caller's)
    double *x64;        // solution (caller's)
    void *x[2];         // CG iterate per precision ([0] aliases x64, [1] the FP32 correction)
    void *r[2], *p[2], *w[2];
    PcgState *st;       // [0] FP64 CG, [1] FP32 inner CG
    double *scal;       // [0] <b,b>, [1] <r,r> of the last FP64 residual
    double stop2[2];    // stopping threshold on <r,r> per precision
    int limit[2];       // iteration limit per precision
    // coarse term of Eq. 6 (a mesh with a coarse space; else null): zc =
    // masked P z0 of the current r, in the precision zc_prec of the slot's CG
    // (0 FP64, 1 FP32 for a mixed slot's inner iterations), added in the
    // operator's p update; crz = r0.z0, added to <r, z> after the slot's partials
    const void *zc;
    const double *crz;
    int zc_prec;
    int pad3;
};

// counts[] of a group: [0] n_slots, [1] ax items, [2] gs items, [3] vec
// items, then per order N the operator items' [first, count] at
// kCountAxRange + 2N (operator items are sorted by order, then slot)
constexpr int kCountAxRange = 4;
constexpr int kCountSize = kCountAxRange + 2 * (SEM_MAX_ORDER + 1);

// Device view of one group (all arrays sized for the batch capacity).
struct GroupDev {
    const int32_t *slots;     // [n_slots] slot ids
    const int64_t *counts;    // kCountSize entries, see above
    const Item *ax_items, *gs_items, *vec_items;
    const int64_t *ax_first;  // per slot id: first ax item, count
    const int64_t *ax_count;
    const int64_t *vec_first;
    const int64_t *vec_count;
    double *ax_partial;       // per ax item
    double *vec_partial;      // 2 per vec item
};

struct BatchLaunch {
    int ax_grid;                     // persistent workgroups of each order's operator launch
    int vec_grid;                    // persistent workgroups of gs / vector kernels
    int max_slots;                   // grid of the per-slot reductions
    unsigned orders;                 // bit N set: launch the order-N operator
    int epw[SEM_MAX_ORDER + 1];      // elements per operator tile, per order
};

// phases of the batched kernels (the operator: one launch per order in L.orders)
hipError_t batch_ax(int prec, int mode, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L,
                    hipStream_t s);
hipError_t batch_gs(int prec, int check_done, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L,
                    hipStream_t s);
hipError_t batch_reduce_sigma(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// r -= alpha w after the gather-scatter, with the dot-product partials
hipError_t batch_update(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
hipError_t batch_reduce_rho(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// CG start: r[prec] holds the residual; p[prec] <- 0; rho, rr; limit/stop2 from the slot
hipError_t batch_cg_init(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// FP64: r = b - w (w holds A x), scal[1] = <r, r>; or (copy_b) r = b, x = 0
hipError_t batch_residual(int copy_b, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// mixed: r32 = r64 / sqrt(scal[1]), x32 = 0
hipError_t batch_to_fp32(const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// end of CG for the group's slots: the deferred last x step
hipError_t batch_finish(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// mixed: x64 += sqrt(scal[1]) x32
hipError_t batch_axpy(const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s);
// orders the batched operator is built for
bool batch_order_supported(int N);

}  // namespace sem
