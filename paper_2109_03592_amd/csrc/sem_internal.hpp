// sem_internal.hpp -- types shared by the host set-up, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "lattice.hpp"

namespace sem {

// ---------------------------------------------------------------------------
// error plumbing: every internal failure becomes a status + thread-local text
void set_error(const std::string &msg);
struct Failure {
    sem_status status;
};
[[noreturn]] void fail(sem_status st, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define SEM_HIP(call) ::sem::check_hip((call), #call)

// ---------------------------------------------------------------------------
// Host set-up products (section 2: GLL basis, element geometry, numbering).
struct HostMesh {
    int N = 0, P = 0;
    int nel[3] = {0, 0, 0};
    int periodic[3] = {0, 0, 0};
    int64_t E = 0, nL = 0, nG = 0;
    int64_t ext[3] = {0, 0, 0};          // global lattice extent per axis
    std::vector<double> xi, w, D;         // GLL nodes, weights, D[i*P+l]
    std::vector<double> xyz;              // [3][nL]
    std::vector<double> G;                // [E][6][P^3] element-blocked
    std::vector<double> B;                // [nL]
    std::vector<int32_t> gid;             // [nL]
    std::vector<uint8_t> gmask;           // [nG]
    std::vector<uint8_t> gmult;           // [nG]
    // gather-scatter plan: ids [0, n_sum) are summed, [n_sum, n_ids) zeroed
    int64_t gs_n_sum = 0, gs_n_ids = 0, gs_plan_len = 0;
    std::vector<int32_t> gs_off;          // [n_ids + 1]
    std::vector<int32_t> gs_idx;          // local ids, ascending within an id
    int64_t n_shared_local = 0, n_shared_global = 0, n_masked_global = 0;
    std::vector<double> invdiag;          // [nL]
    sem_mesh_desc desc{};                 // copy of the descriptor (vertices below)
    std::vector<double> vertices;
};

void gll_rule(int N, std::vector<double> &xi, std::vector<double> &w);
void lagrange_derivative(const std::vector<double> &xi, std::vector<double> &D);
void build_host_mesh(const sem_mesh_desc &d, HostMesh &h);
void build_host_coords(const sem_mesh_desc &d, HostMesh &h);
void build_jacobi(HostMesh &h);  // from h.G (element-blocked), h.gs plan, h.gid, h.gmask
void host_parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &body);

// ---------------------------------------------------------------------------
// Device-side PCG scalars (one block per solve, device memory).
struct PcgState {
    double rho;        // <r, z>
    double rho_new;
    double sigma;      // <p, A p>
    double alpha, beta;
    double rr;         // <r, r>
    double stop2;      // stop when rr <= stop2
    int iters;         // iterations performed
    int done;          // 1 = converged, 2 = breakdown
    int limit;         // iteration limit
    int pad;
};

// Device gather-scatter plan: CSR over global ids sorted in lattice order,
// summed ids [0, n_sum) first, then Dirichlet ids up to n_ids.
struct GsPlan {
    int64_t n_sum;
    int64_t n_ids;
};


// ---------------------------------------------------------------------------
struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct CoarseSpace;   // coarse.hpp
struct SchwarzSpace;  // schwarz.hpp
struct AxgsSpace;     // axgs_host.hpp

}  // namespace sem

struct sem_mesh {
    sem::HostMesh h;
    int device = 0;
    int with_fp32 = 0;
    // device arrays
    double *G64 = nullptr;     // [E][6][P^3]
    float *G32 = nullptr;
    double *B64 = nullptr;     // [nL]
    double *inv64 = nullptr;   // [nL]
    float *inv32 = nullptr;
    uint8_t *mult = nullptr;   // [nL] multiplicity per local node
    int32_t *gid = nullptr;    // [nL]
    int32_t *gs_off = nullptr;     // gather-scatter plan (CSR)
    int32_t *gs_idx = nullptr;
    sem::GsPlan gsplan{};
    // lattice gather-scatter (no plan read), used in place of the plan when
    // gs_lattice_ok and gs_kind != SEM_GS_PLAN
    sem::GsLattice gsl{};
    int gs_lattice_ok = 0;
    int gs_kind = 0;
    // Helmholtz coefficients (sem_set_helmholtz): h1 and h2*B per local node;
    // helm = 0 is the Poisson operator
    int helm = 0;
    int op_version = 0;  // bumped whenever the operator changes (projection bases follow it)
    double *h1_64 = nullptr, *h2b64 = nullptr;
    float *h1_32 = nullptr, *h2b32 = nullptr;
    // coarse term of the FP64 preconditioner (sem_set_coarse); nullptr: Jacobi
    sem::CoarseSpace *coarse = nullptr;
    // overlapping Schwarz local solves in place of Jacobi (sem_set_schwarz, FP64 solves)
    sem::SchwarzSpace *schwarz = nullptr;
    // fused operator and gather-scatter (sem_set_axgs_config); created at set-up
    sem::AxgsSpace *axgs = nullptr;
    // Krylov work space, allocated on the first solve
    double *x64 = nullptr, *r64 = nullptr, *p64 = nullptr, *w64 = nullptr;
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *w32 = nullptr;
    double *partials = nullptr;   // reduction partials
    int64_t n_partials = 0;
    sem::PcgState *state = nullptr;  // [2]: FP64 solve, FP32 inner solve
    double *scal = nullptr;          // small device scratch for norms
    int ax_epw = 1;                  // elements per workgroup of the FP64 operator
    int ax_epw32 = 1;                // ... of the FP32 operator
    int ax_epw_plain = 1;            // ... of the FP64 plain operator (modes 0, 1)
    int ax_grid_cap = 4096;          // persistent operator grid
    std::vector<hipEvent_t> events;  // profiling event pool
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // CG iteration blocks, FP64 / FP32
    int graph_k[2] = {0, 0};
    int graph_epw[2] = {0, 0};
    int graph_grid[2] = {0, 0};
    size_t device_bytes = 0;
    std::vector<void *> allocations;
};
