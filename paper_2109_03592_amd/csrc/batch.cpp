// batch.cpp -- host side of batched CG: slots, groups, phase transitions,
// the autotuner and the C ABI of sem_batch_*.
//
// Each slot walks a small state machine:
//   FP64 : START -> CG64 -> CHECK -> DONE   (CHECK restarts CG64 at most 3x)
//   mixed: RESID -> CG32 -> RESID -> ... -> DONE
// START/CHECK/RESID are served together by one batched FP64 residual
// (operator, gather-scatter, r = b - A x, <r,r>); CG64 and CG32 slots are
// advanced by replaying one hipGraph per precision whose kernels read the
// group's work tables from fixed device addresses, so membership changes only
// rewrite table contents.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "batch.hpp"
#include "coarse.hpp"
#include "kernels.hpp"

namespace sem {

hipError_t upload_batch_dtables(const double *d64, const float *d32, hipStream_t s);
void ensure_dtables_all(hipStream_t s);
int persistent_grid_cap_public();
double inner_tolerance(const sem_solve_opts &o, double rel);

enum Phase { PH_FREE = 0, PH_START, PH_CG64, PH_CHECK, PH_RESID, PH_CG32, PH_DONE };

struct HostSlot {
    int phase = PH_FREE;
    sem_mesh *mesh = nullptr;
    sem_solve_opts opts{};
    const double *b = nullptr;
    double *x = nullptr;
    int iters = 0, outer = 0, restarts = 0;
    double bb = -1.0, rel = 0.0;
    sem_status status = SEM_OK;
    void *buf = nullptr;     // slot-owned device vectors
    size_t buf_bytes = 0;
    // coarse term (slots of a mesh with a coarse space): zc = P z0 and
    // the coarse work vectors, in a second slot-owned buffer
    void *cbuf = nullptr;
    size_t cbuf_bytes = 0;
    CoarseWork cw{};
    uint64_t serial = 0;     // unique per admission (keys the graphs that bake this slot's launches)
    std::chrono::steady_clock::time_point t0;
    double seconds = 0.0;
};

struct Group {
    // device
    int32_t *slots = nullptr;
    int64_t *counts = nullptr;
    Item *ax_items = nullptr, *gs_items = nullptr, *vec_items = nullptr;
    int64_t *ax_first = nullptr, *ax_count = nullptr, *vec_first = nullptr, *vec_count = nullptr;
    double *ax_partial = nullptr, *vec_partial = nullptr;
    // capacities
    int64_t cap_ax = 0, cap_gs = 0, cap_vec = 0;
    // host mirror
    std::vector<int32_t> h_slots;
    std::vector<Item> h_ax, h_gs, h_vec;
    std::vector<int64_t> h_axf, h_axc, h_vf, h_vc;
    unsigned orders = 0;          // orders present in the tables
    int prec = 0;                 // precision of the operator launches (tile sizes follow it)
    hipGraphExec_t graph = nullptr;
    int graph_k = 0;
    unsigned graph_orders = 0;    // orders the cached graph launches
    // the coarse-term launches the cached graph holds: (slot, its admission serial)
    std::vector<std::pair<int, uint64_t>> graph_coarse;
    GroupDev dev() const
    {
        GroupDev g;
        g.slots = slots;
        g.counts = counts;
        g.ax_items = ax_items;
        g.gs_items = gs_items;
        g.vec_items = vec_items;
        g.ax_first = ax_first;
        g.ax_count = ax_count;
        g.vec_first = vec_first;
        g.vec_count = vec_count;
        g.ax_partial = ax_partial;
        g.vec_partial = vec_partial;
        return g;
    }
};

}  // namespace sem

struct sem_batch {
    int max_slots = 0;
    size_t budget = 0, used = 0;
    int device = 0;
    std::vector<sem::HostSlot> slots;
    std::vector<sem::SlotDesc> h_desc;
    sem::SlotDesc *d_desc = nullptr;
    sem::PcgState *d_state = nullptr;   // 2 per slot
    double *d_scal = nullptr;           // 2 per slot
    sem::Group g64, g32, gres;          // CG64, CG32, residual
    int epw[2][SEM_MAX_ORDER + 1] = {};  // elements per operator tile, per precision and order (0: default)
    sem::BatchLaunch L{};
    hipStream_t capture = nullptr;
    std::vector<void *> allocations;
    std::multimap<size_t, void *> free_bufs;
    uint64_t next_serial = 0;           // admissions so far (HostSlot::serial)
    std::vector<sem::PcgState> h_state;
};

namespace sem {

template <typename F>
static sem_status bguard(F &&f)
{
    try {
        return f();
    } catch (const Failure &x) {
        return x.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SEM_ENOMEM;
    } catch (const std::exception &x) {
        set_error(x.what());
        return SEM_EINVAL;
    }
}

static void *balloc(sem_batch *B, size_t bytes)
{
    void *p = nullptr;
    SEM_HIP(hipMalloc(&p, std::max<size_t>(bytes, 16)));
    B->allocations.push_back(p);
    return p;
}

// elements per operator tile: the single-mesh rule (fill whole waves)
int default_operator_epw(int N, bool fp32);

static int batch_epw(const sem_batch *B, int N, int prec)
{
    return B->epw[prec][N] > 0 ? B->epw[prec][N] : default_operator_epw(N, prec == 1);
}

static void group_alloc(sem_batch *B, Group &g, int prec)
{
    g.prec = prec;
    const int ms = B->max_slots;
    g.slots = (int32_t *)balloc(B, sizeof(int32_t) * ms);
    g.counts = (int64_t *)balloc(B, sizeof(int64_t) * kCountSize);
    g.ax_first = (int64_t *)balloc(B, sizeof(int64_t) * ms);
    g.ax_count = (int64_t *)balloc(B, sizeof(int64_t) * ms);
    g.vec_first = (int64_t *)balloc(B, sizeof(int64_t) * ms);
    g.vec_count = (int64_t *)balloc(B, sizeof(int64_t) * ms);
    g.cap_ax = g.cap_gs = g.cap_vec = 0;
    SEM_HIP(hipMemset(g.counts, 0, sizeof(int64_t) * kCountSize));
}

// grow item tables (device addresses change: cached graphs are dropped; the
// old buffers stay allocated until the batch is freed, since queued work may
// still read them)
static void group_reserve(sem_batch *B, Group &g, int64_t nax, int64_t ngs, int64_t nvec)
{
    bool grown = false;
    if (nax > g.cap_ax) {
        const int64_t c = std::max<int64_t>({nax, 2 * g.cap_ax, 1024});
        g.ax_items = (Item *)balloc(B, sizeof(Item) * c);
        g.ax_partial = (double *)balloc(B, sizeof(double) * c);
        g.cap_ax = c;
        grown = true;
    }
    if (ngs > g.cap_gs) {
        const int64_t c = std::max<int64_t>({ngs, 2 * g.cap_gs, 1024});
        g.gs_items = (Item *)balloc(B, sizeof(Item) * c);
        g.cap_gs = c;
        grown = true;
    }
    if (nvec > g.cap_vec) {
        const int64_t c = std::max<int64_t>({nvec, 2 * g.cap_vec, 1024});
        g.vec_items = (Item *)balloc(B, sizeof(Item) * c);
        g.vec_partial = (double *)balloc(B, sizeof(double) * 2 * c);
        g.cap_vec = c;
        grown = true;
    }
    if (grown && g.graph) {
        hipGraphExecDestroy(g.graph);
        g.graph = nullptr;
    }
}

// rebuild a group's tables for the given slots and upload them on stream s
static void group_build(sem_batch *B, Group &g, const std::vector<int> &ids, hipStream_t s)
{
    g.h_slots.assign(ids.begin(), ids.end());
    g.h_ax.clear();
    g.h_gs.clear();
    g.h_vec.clear();
    g.h_axf.assign(B->max_slots, 0);
    g.h_axc.assign(B->max_slots, 0);
    g.h_vf.assign(B->max_slots, 0);
    g.h_vc.assign(B->max_slots, 0);
    int64_t counts[kCountSize] = {0};
    g.orders = 0;
    // operator items by order (one launch per order), then by slot
    for (int N = 1; N <= SEM_MAX_ORDER; ++N) {
        const int64_t first = (int64_t)g.h_ax.size();
        for (int id : ids) {
            const SlotDesc &d = B->h_desc[id];
            if (d.N != N) continue;
            const int epw = batch_epw(B, N, g.prec);
            const int64_t nt = (d.E + epw - 1) / epw;
            g.h_axf[id] = (int64_t)g.h_ax.size();
            g.h_axc[id] = nt;
            for (int64_t t = 0; t < nt; ++t) g.h_ax.push_back(Item{id, (int32_t)t});
        }
        counts[kCountAxRange + 2 * N] = first;
        counts[kCountAxRange + 2 * N + 1] = (int64_t)g.h_ax.size() - first;
        if ((int64_t)g.h_ax.size() > first) g.orders |= 1u << N;
    }
    for (int id : ids) {
        const SlotDesc &d = B->h_desc[id];
        const int64_t ng = ((d.gs_lattice ? d.gsl.n_nodes : d.gs_n_ids) + kGsChunk - 1) / kGsChunk;
        for (int64_t t = 0; t < ng; ++t) g.h_gs.push_back(Item{id, (int32_t)t});
        const int64_t nv = (d.nL + kVecChunk - 1) / kVecChunk;
        g.h_vf[id] = (int64_t)g.h_vec.size();
        g.h_vc[id] = nv;
        for (int64_t t = 0; t < nv; ++t) g.h_vec.push_back(Item{id, (int32_t)t});
    }
    group_reserve(B, g, std::max<size_t>(g.h_ax.size(), 1), std::max<size_t>(g.h_gs.size(), 1),
                  std::max<size_t>(g.h_vec.size(), 1));
    counts[0] = (int64_t)ids.size();
    counts[1] = (int64_t)g.h_ax.size();
    counts[2] = (int64_t)g.h_gs.size();
    counts[3] = (int64_t)g.h_vec.size();
    SEM_HIP(hipMemcpyAsync(g.counts, counts, sizeof(counts), hipMemcpyHostToDevice, s));
    if (!ids.empty()) SEM_HIP(hipMemcpyAsync(g.slots, g.h_slots.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, s));
    if (!g.h_ax.empty()) SEM_HIP(hipMemcpyAsync(g.ax_items, g.h_ax.data(), sizeof(Item) * g.h_ax.size(), hipMemcpyHostToDevice, s));
    if (!g.h_gs.empty()) SEM_HIP(hipMemcpyAsync(g.gs_items, g.h_gs.data(), sizeof(Item) * g.h_gs.size(), hipMemcpyHostToDevice, s));
    if (!g.h_vec.empty()) SEM_HIP(hipMemcpyAsync(g.vec_items, g.h_vec.data(), sizeof(Item) * g.h_vec.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(g.ax_first, g.h_axf.data(), sizeof(int64_t) * B->max_slots, hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(g.ax_count, g.h_axc.data(), sizeof(int64_t) * B->max_slots, hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(g.vec_first, g.h_vf.data(), sizeof(int64_t) * B->max_slots, hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(g.vec_count, g.h_vc.data(), sizeof(int64_t) * B->max_slots, hipMemcpyHostToDevice, s));
    // host staging vectors must outlive the async copies
    SEM_HIP(hipStreamSynchronize(s));
}

static BatchLaunch launch_for(sem_batch *B, unsigned orders, int prec)
{
    BatchLaunch L = B->L;
    L.orders = orders;
    for (int N = 0; N <= SEM_MAX_ORDER; ++N) L.epw[N] = N >= 1 ? batch_epw(B, N, prec) : 1;
    return L;
}

static BatchLaunch launch_for(sem_batch *B, const Group &g) { return launch_for(B, g.orders, g.prec); }

static void upload_desc(sem_batch *B, int id, hipStream_t s)
{
    SEM_HIP(hipMemcpyAsync(B->d_desc + id, &B->h_desc[id], sizeof(SlotDesc), hipMemcpyHostToDevice, s));
}

// The coarse term of one FP64 slot from its current r: restriction, the
// Chebyshev coarse solve with r0.z0 reduced into crz, and zc = masked P z0.
// Launched per slot (the coarse vectors are small); the kernels of a
// converged slot skip or rewrite its own buffers only.
// at_start: the CG start -- the kernels run whatever the slot's state says
// (a mixed slot's FP32 state still holds the previous inner solve's flag).
static void slot_coarse(sem_batch *B, int id, hipStream_t s, bool at_start = false)
{
    HostSlot &h = B->slots[id];
    const SlotDesc &d = B->h_desc[id];
    sem_mesh *m = h.mesh;
    const int p = d.zc_prec;  // the precision of the slot's CG: FP64, or FP32 inner iterations
    if (p == 0) coarse_restrict_w<double>(m, h.cw, static_cast<const double *>(d.r[0]), m->inv64, s);
    else coarse_restrict_w<float>(m, h.cw, static_cast<const float *>(d.r[1]), m->inv32, s);
    const int pairs = coarse_solve_w(m, h.cw, h.cw.dot, at_start ? nullptr : d.st + p, s);
    SEM_HIP(launch_reduce_scalar(h.cw.dot, 2 * (int64_t)pairs, h.cw.rz, s));
    if (p == 0) coarse_prolong_w(m, h.cw, static_cast<double *>(const_cast<void *>(d.zc)), false, s);
    else coarse_prolong_w32(m, h.cw, static_cast<float *>(const_cast<void *>(d.zc)), s);
}

// the group's slots that take the coarse term in precision prec, with their
// admission serials: a graph that baked a slot's coarse launches (its mesh's
// coarse arrays, its work vectors) is replayed only for that same admission,
// never for a later one that reuses the slot and its cached buffers
static std::vector<std::pair<int, uint64_t>> coarse_slots(const sem_batch *B, const Group &g, int prec)
{
    std::vector<std::pair<int, uint64_t>> out;
    for (int32_t id : g.h_slots)
        if (B->h_desc[id].zc && B->h_desc[id].zc_prec == prec) out.emplace_back(id, B->slots[id].serial);
    return out;
}

// one CG iteration of every slot in g, precision prec
static void enqueue_batch_iters(sem_batch *B, Group &g, int prec, int k, unsigned orders, hipStream_t s)
{
    const GroupDev gd = g.dev();
    const BatchLaunch L = launch_for(B, orders, g.prec);
    const auto cs = coarse_slots(B, g, prec);
    for (int it = 0; it < k; ++it) {
        SEM_HIP(batch_ax(prec, 2, B->d_desc, gd, L, s));
        SEM_HIP(batch_gs(prec, 1, B->d_desc, gd, L, s));
        SEM_HIP(batch_reduce_sigma(prec, B->d_desc, gd, L, s));
        SEM_HIP(batch_update(prec, B->d_desc, gd, L, s));
        for (const auto &c : cs) slot_coarse(B, c.first, s);
        SEM_HIP(batch_reduce_rho(prec, B->d_desc, gd, L, s));
    }
}

static void run_batch_iters(sem_batch *B, Group &g, int prec, int k, bool use_graph, hipStream_t s)
{
    if (g.h_slots.empty()) return;
    if (!use_graph) {
        enqueue_batch_iters(B, g, prec, k, g.orders, s);
        return;
    }
    // a cached graph serves any membership whose orders it launches (an
    // order without items exits at once) and whose coarse-term slots it holds
    const auto cs = coarse_slots(B, g, prec);
    if (!g.graph || g.graph_k != k || (g.orders & ~g.graph_orders) != 0 || cs != g.graph_coarse) {
        const unsigned orders = g.orders | (g.graph ? g.graph_orders : 0u);
        if (g.graph) {
            SEM_HIP(hipGraphExecDestroy(g.graph));
            g.graph = nullptr;
        }
        if (!B->capture) SEM_HIP(hipStreamCreateWithFlags(&B->capture, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        SEM_HIP(hipStreamBeginCapture(B->capture, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_batch_iters(B, g, prec, k, orders, B->capture);
        } catch (...) {
            hipStreamEndCapture(B->capture, &gr);
            if (gr) hipGraphDestroy(gr);
            throw;
        }
        SEM_HIP(hipStreamEndCapture(B->capture, &gr));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        SEM_HIP(e);
        g.graph = ex;
        g.graph_k = k;
        g.graph_orders = orders;
        g.graph_coarse = cs;
    }
    SEM_HIP(hipGraphLaunch(g.graph, s));
}

static void read_states(sem_batch *B, hipStream_t s)
{
    B->h_state.resize(2 * B->max_slots);
    SEM_HIP(hipMemcpyAsync(B->h_state.data(), B->d_state, sizeof(PcgState) * 2 * B->max_slots,
                           hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
}

static void read_scal(sem_batch *B, std::vector<double> &sc, hipStream_t s)
{
    sc.resize(2 * B->max_slots);
    SEM_HIP(hipMemcpyAsync(sc.data(), B->d_scal, sizeof(double) * 2 * B->max_slots, hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
}

// initialise CG (precision prec) for the given slots from their current r
static void start_cg(sem_batch *B, const std::vector<int> &ids, int prec, hipStream_t s)
{
    if (ids.empty()) return;
    Group &g = B->gres;
    group_build(B, g, ids, s);
    // the coarse term of the start residual; its r0.z0 joins rho
    for (const auto &c : coarse_slots(B, g, prec)) slot_coarse(B, c.first, s, true);
    SEM_HIP(batch_cg_init(prec, B->d_desc, g.dev(), launch_for(B, g), s));
}

// FP64 residual of the given slots; copy_b ids start from x = 0
static void residuals(sem_batch *B, const std::vector<int> &ids, bool copy_b, hipStream_t s)
{
    if (ids.empty()) return;
    Group &g = B->gres;
    group_build(B, g, ids, s);
    const GroupDev gd = g.dev();
    const BatchLaunch L = launch_for(B, g);
    if (!copy_b) {
        SEM_HIP(batch_ax(0, 0, B->d_desc, gd, L, s));
        SEM_HIP(batch_gs(0, 0, B->d_desc, gd, L, s));
    }
    SEM_HIP(batch_residual(copy_b ? 1 : 0, B->d_desc, gd, L, s));
}

static void finish_slot(sem_batch *B, int id, sem_status st)
{
    HostSlot &h = B->slots[id];
    h.phase = PH_DONE;
    h.status = st;
    h.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - h.t0).count();
}

// Advance every active slot: serve pending residuals / transitions, then
// replay k CG iterations per precision, then read the states.
static void step_batch(sem_batch *B, int k, bool use_graph, hipStream_t s)
{
    const int ms = B->max_slots;
    // 1. residual-phase slots
    std::vector<int> fresh, resid;
    for (int id = 0; id < ms; ++id) {
        const HostSlot &h = B->slots[id];
        if (h.phase == PH_START && !h.opts.x0_given && h.opts.precision == SEM_PREC_FP64) fresh.push_back(id);
        else if (h.phase == PH_START || h.phase == PH_CHECK || h.phase == PH_RESID) resid.push_back(id);
    }
    std::vector<double> sc;
    std::vector<int> to64, to32;
    if (!fresh.empty()) {
        residuals(B, fresh, true, s);
        read_scal(B, sc, s);
        for (int id : fresh) {
            HostSlot &h = B->slots[id];
            h.bb = sc[2 * id];
            if (h.bb == 0.0) {
                h.rel = 0.0;
                finish_slot(B, id, SEM_OK);
                continue;
            }
            to64.push_back(id);
        }
    }
    if (!resid.empty()) {
        residuals(B, resid, false, s);
        read_scal(B, sc, s);
        for (int id : resid) {
            HostSlot &h = B->slots[id];
            if (h.bb < 0.0) h.bb = sc[2 * id];
            const double rr = sc[2 * id + 1];
            h.rel = h.bb > 0.0 ? std::sqrt(rr / h.bb) : 0.0;
            if (h.bb == 0.0 || h.rel <= h.opts.tol) {
                finish_slot(B, id, SEM_OK);
                continue;
            }
            if (h.opts.precision == SEM_PREC_FP64) {
                if (h.phase == PH_CHECK) {
                    if (h.iters >= h.opts.max_iter || h.restarts == 3) {
                        set_error("batched solve: no convergence within max_iter");
                        finish_slot(B, id, SEM_ENOCONV);
                        continue;
                    }
                    h.restarts++;
                }
                to64.push_back(id);
            } else {
                if (h.iters >= h.opts.max_iter || h.outer >= 100) {
                    set_error("batched mixed solve: no convergence within max_iter");
                    finish_slot(B, id, SEM_ENOCONV);
                    continue;
                }
                to32.push_back(id);
            }
        }
    }
    // 2. entering CG
    for (int id : to64) {
        HostSlot &h = B->slots[id];
        SlotDesc &d = B->h_desc[id];
        d.stop2[0] = h.opts.tol * h.opts.tol * h.bb;
        d.limit[0] = h.opts.max_iter - h.iters;
        upload_desc(B, id, s);
        h.phase = PH_CG64;
    }
    start_cg(B, to64, 0, s);
    if (!to32.empty()) {
        for (int id : to32) {
            HostSlot &h = B->slots[id];
            SlotDesc &d = B->h_desc[id];
            const double eta = inner_tolerance(h.opts, h.rel);
            d.stop2[1] = eta * eta;
            const int inner_max = h.opts.inner_max_iter > 0 ? h.opts.inner_max_iter : h.opts.max_iter;
            d.limit[1] = std::min(inner_max, h.opts.max_iter - h.iters);
            upload_desc(B, id, s);
            h.phase = PH_CG32;
        }
        Group &g = B->gres;
        group_build(B, g, to32, s);
        SEM_HIP(batch_to_fp32(B->d_desc, g.dev(), launch_for(B, g), s));
        // the coarse term of the FP32 start residual; its r0.z0 joins rho
        for (const auto &c : coarse_slots(B, g, 1)) slot_coarse(B, c.first, s, true);
        SEM_HIP(batch_cg_init(1, B->d_desc, g.dev(), launch_for(B, g), s));
    }
    // 3. CG iterations
    std::vector<int> cg64, cg32;
    for (int id = 0; id < ms; ++id) {
        if (B->slots[id].phase == PH_CG64) cg64.push_back(id);
        if (B->slots[id].phase == PH_CG32) cg32.push_back(id);
    }
    if (cg64 != B->g64.h_slots) group_build(B, B->g64, cg64, s);
    if (cg32 != B->g32.h_slots) group_build(B, B->g32, cg32, s);
    if (!cg64.empty()) run_batch_iters(B, B->g64, 0, k, use_graph, s);
    if (!cg32.empty()) run_batch_iters(B, B->g32, 1, k, use_graph, s);
    if (cg64.empty() && cg32.empty()) return;
    read_states(B, s);
    // 4. transitions out of CG (first the deferred last x step of every slot
    //    whose CG run ended)
    std::vector<int> fin64, fin32, axpy;
    for (int id : cg64)
        if (B->h_state[2 * id].done) fin64.push_back(id);
    for (int id : cg32)
        if (B->h_state[2 * id + 1].done) fin32.push_back(id);
    if (!fin64.empty()) {
        Group &g = B->gres;
        group_build(B, g, fin64, s);
        SEM_HIP(batch_finish(0, B->d_desc, g.dev(), launch_for(B, g), s));
    }
    if (!fin32.empty()) {
        Group &g = B->gres;
        group_build(B, g, fin32, s);
        SEM_HIP(batch_finish(1, B->d_desc, g.dev(), launch_for(B, g), s));
    }
    for (int id : fin64) {
        HostSlot &h = B->slots[id];
        const PcgState &st = B->h_state[2 * id];
        h.iters += st.iters;
        if (st.done == 2) {
            set_error("batched solve: CG breakdown");
            finish_slot(B, id, SEM_EBREAKDOWN);
            continue;
        }
        h.phase = PH_CHECK;
    }
    for (int id : fin32) {
        HostSlot &h = B->slots[id];
        const PcgState &st = B->h_state[2 * id + 1];
        h.iters += st.iters;
        h.outer++;
        if (st.done == 2 && st.iters == 0) {
            set_error("batched mixed solve: FP32 inner CG broke down at its first step");
            finish_slot(B, id, SEM_EBREAKDOWN);
            continue;
        }
        axpy.push_back(id);
        h.phase = PH_RESID;
    }
    if (!axpy.empty()) {
        Group &g = B->gres;
        group_build(B, g, axpy, s);
        SEM_HIP(batch_axpy(B->d_desc, g.dev(), launch_for(B, g), s));
    }
}

static int free_slot_index(sem_batch *B)
{
    for (int id = 0; id < B->max_slots; ++id)
        if (B->slots[id].phase == PH_FREE) return id;
    return -1;
}

// Layout of a slot's vector buffer: r, p, w in FP64, then (mixed) x, r, p, w
// in FP32, each starting on a 256-byte boundary.  off[0..6] receive the byte
// offsets (unused ones 0); returns the bytes the buffer must hold.  The one
// helper sizes the allocation and carves it, so the two cannot disagree.
size_t slot_layout(int64_t nL, int precision, size_t off[7])
{
    const size_t v64 = (size_t)nL * 8, v32 = (size_t)nL * 4;
    auto ru = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t o = 0;
    for (int q = 0; q < 7; ++q) off[q] = 0;
    for (int q = 0; q < 3; ++q) {
        off[q] = o;
        o += ru(v64);
    }
    if (precision == SEM_PREC_MIXED)
        for (int q = 3; q < 7; ++q) {
            off[q] = o;
            o += ru(v32);
        }
    return o;
}

static size_t slot_bytes(const sem_mesh *m, int precision)
{
    size_t off[7];
    return slot_layout(m->h.nL, precision, off);
}

static int admit_slot(sem_batch *B, sem_mesh *m, const double *b, double *x, const sem_solve_opts &o, hipStream_t s)
{
    if (!batch_order_supported(m->h.N)) fail(SEM_EUNSUPPORTED, "batched solves support orders 2..10");
    if (m->device != B->device) fail(SEM_EINVAL, "mesh is on another device");
    if (o.precision == SEM_PREC_MIXED && !m->with_fp32) fail(SEM_EINVAL, "mixed precision needs SEM_WITH_FP32");
    if (m->helm) fail(SEM_EUNSUPPORTED, "batched solves take the Poisson operator only (sem_set_helmholtz is set)");
    if (m->schwarz) fail(SEM_EUNSUPPORTED, "batched solves take Jacobi or Jacobi + coarse term (sem_set_schwarz is set)");
    const int id = free_slot_index(B);
    if (id < 0) fail(SEM_EBUDGET, "no free slot");
    // slots of a mesh with a coarse space take the coarse term in their CG
    // (FP64, or the FP32 inner iterations of a mixed slot)
    const bool coarse = m->coarse != nullptr;
    const int zc_prec = o.precision == SEM_PREC_MIXED ? 1 : 0;
    const size_t need = slot_bytes(m, o.precision);
    const size_t zc_bytes = ((size_t)m->h.nL * (zc_prec ? 4 : 8) + 255) / 256 * 256;
    const size_t cneed = coarse ? zc_bytes + (size_t)coarse_work_doubles(m->coarse, m->h.E) * 8 : 0;
    // a cached buffer of at least `bytes` (at most twice as large), else a new one
    auto acquire = [&](size_t bytes, size_t &have) -> void * {
        auto itb = B->free_bufs.lower_bound(bytes);
        if (itb != B->free_bufs.end() && itb->first <= 2 * bytes) {
            void *p = itb->second;
            have = itb->first;
            B->free_bufs.erase(itb);
            return p;
        }
        if (B->budget && B->used + bytes > B->budget) {
            // drop cached free buffers before refusing
            for (auto &fb : B->free_bufs) {
                hipFree(fb.second);
                B->allocations.erase(std::find(B->allocations.begin(), B->allocations.end(), fb.second));
                B->used -= fb.first;
            }
            B->free_bufs.clear();
            if (B->used + bytes > B->budget) fail(SEM_EBUDGET, "slot vectors exceed the batch budget");
        }
        void *p = balloc(B, bytes);
        B->used += bytes;
        have = bytes;
        return p;
    };
    size_t have = 0, chave = 0;
    void *buf = acquire(need, have);
    void *cbuf = nullptr;
    if (coarse) {
        try {
            cbuf = acquire(cneed, chave);
        } catch (...) {
            B->free_bufs.emplace(have, buf);
            throw;
        }
    }
    if (have < need || chave < cneed) fail(SEM_EINVAL, "slot buffer smaller than its layout");
    HostSlot &h = B->slots[id];
    h.buf_bytes = have;
    h.cbuf = cbuf;
    h.cbuf_bytes = chave;
    h.serial = ++B->next_serial;
    h.cw = coarse ? coarse_work_carve(m->coarse, m->h.E,
                                      reinterpret_cast<double *>(static_cast<char *>(cbuf) + zc_bytes))
                  : CoarseWork{};
    h.mesh = m;
    h.opts = o;
    h.b = b;
    h.x = x;
    h.iters = h.outer = h.restarts = 0;
    h.bb = -1.0;
    h.rel = 0.0;
    h.status = SEM_OK;
    h.buf = buf;
    h.t0 = std::chrono::steady_clock::now();
    h.phase = PH_START;
    if (o.precision == SEM_PREC_MIXED) h.phase = PH_RESID;
    SlotDesc &d = B->h_desc[id];
    std::memset(&d, 0, sizeof(d));
    const HostMesh &hm = m->h;
    d.N = hm.N;
    d.E = hm.E;
    d.nL = hm.nL;
    d.G[0] = m->G64;
    d.G[1] = m->G32;
    d.inv[0] = m->inv64;
    d.inv[1] = m->inv32;
    d.mult = m->mult;
    d.gs_off = m->gs_off;
    d.gs_idx = m->gs_idx;
    d.gs_n_sum = hm.gs_n_sum;
    d.gs_n_ids = hm.gs_n_ids;
    // the mesh's gather-scatter kind: the lattice kernel (same bits as the plan) where it runs
    d.gsl = m->gsl;
    d.gs_lattice = m->gs_lattice_ok && m->gs_kind != SEM_GS_PLAN ? 1 : 0;
    d.b = b;
    d.x64 = x;
    size_t off[7];
    slot_layout(hm.nL, o.precision, off);
    char *p = static_cast<char *>(buf);
    d.x[0] = x;
    d.r[0] = p + off[0];
    d.p[0] = p + off[1];
    d.w[0] = p + off[2];
    if (o.precision == SEM_PREC_MIXED) {
        d.x[1] = p + off[3];
        d.r[1] = p + off[4];
        d.p[1] = p + off[5];
        d.w[1] = p + off[6];
    }
    d.st = B->d_state + 2 * id;
    d.scal = B->d_scal + 2 * id;
    d.zc = coarse ? cbuf : nullptr;
    d.crz = coarse ? h.cw.rz : nullptr;
    d.zc_prec = zc_prec;
    SEM_HIP(hipMemsetAsync(d.st, 0, 2 * sizeof(PcgState), s));
    // mixed slots start with a residual of the caller's x: zero it unless it
    // is the initial guess (FP64 slots without a guess zero it themselves)
    if (o.precision == SEM_PREC_MIXED && !o.x0_given) SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * hm.nL, s));
    upload_desc(B, id, s);
    return id;
}

static void retire_slot(sem_batch *B, int id)
{
    HostSlot &h = B->slots[id];
    if (h.buf) B->free_bufs.emplace(h.buf_bytes, h.buf);
    if (h.cbuf) B->free_bufs.emplace(h.cbuf_bytes, h.cbuf);
    h = HostSlot();
}

}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_batch_slot_layout(int64_t n_local, int precision, size_t *offsets, size_t *bytes)
{
    return bguard([&]() -> sem_status {
        if (!offsets || !bytes || n_local < 1) fail(SEM_EINVAL, "sem_batch_slot_layout: bad arguments");
        if (precision != SEM_PREC_FP64 && precision != SEM_PREC_MIXED)
            fail(SEM_EINVAL, "sem_batch_slot_layout: unknown precision");
        *bytes = slot_layout(n_local, precision, offsets);
        return SEM_OK;
    });
}

sem_status sem_batch_create(int max_slots, size_t device_budget, void *stream, sem_batch **out)
{
    return bguard([&]() -> sem_status {
        if (!out || max_slots < 1 || max_slots > 65536) fail(SEM_EINVAL, "sem_batch_create: bad arguments");
        *out = nullptr;
        hipStream_t s = (hipStream_t)stream;
        ensure_dtables_all(s);
        sem_batch *B = new sem_batch();
        try {
            B->max_slots = max_slots;
            B->budget = device_budget;
            SEM_HIP(hipGetDevice(&B->device));
            B->slots.assign(max_slots, HostSlot());
            B->h_desc.assign(max_slots, SlotDesc());
            B->d_desc = (SlotDesc *)balloc(B, sizeof(SlotDesc) * max_slots);
            B->d_state = (PcgState *)balloc(B, sizeof(PcgState) * 2 * max_slots);
            B->d_scal = (double *)balloc(B, sizeof(double) * 2 * max_slots);
            SEM_HIP(hipMemsetAsync(B->d_state, 0, sizeof(PcgState) * 2 * max_slots, s));
            group_alloc(B, B->g64, 0);
            group_alloc(B, B->g32, 1);
            group_alloc(B, B->gres, 0);
            const int cap = persistent_grid_cap_public();
            B->L.ax_grid = cap;
            B->L.vec_grid = cap;
            B->L.max_slots = max_slots;
            SEM_HIP(hipStreamSynchronize(s));
        } catch (...) {
            sem_batch_free(B);
            throw;
        }
        *out = B;
        return SEM_OK;
    });
}

sem_status sem_batch_free(sem_batch *B)
{
    if (!B) return SEM_OK;
    for (Group *g : {&B->g64, &B->g32, &B->gres})
        if (g->graph) hipGraphExecDestroy(g->graph);
    if (B->capture) hipStreamDestroy(B->capture);
    for (void *p : B->allocations) hipFree(p);
    delete B;
    return SEM_OK;
}

sem_status sem_batch_admit(sem_batch *B, sem_mesh *mesh, const double *b, double *x, const sem_solve_opts *opts,
                           int *slot, void *stream)
{
    return bguard([&]() -> sem_status {
        if (!B || !mesh || !b || !x || !slot) fail(SEM_EINVAL, "sem_batch_admit: null argument");
        sem_solve_opts o;
        sem_solve_opts_default(&o);
        if (opts) o = *opts;
        if (!(o.tol > 0.0)) fail(SEM_EINVAL, "sem_batch_admit: tol must be positive");
        if (o.precision != SEM_PREC_FP64 && o.precision != SEM_PREC_MIXED) fail(SEM_EINVAL, "unknown precision");
        *slot = admit_slot(B, mesh, b, x, o, (hipStream_t)stream);
        return SEM_OK;
    });
}

sem_status sem_batch_step(sem_batch *B, int iterations, int use_graph, void *stream, int *n_active)
{
    return bguard([&]() -> sem_status {
        if (!B || iterations < 1) fail(SEM_EINVAL, "sem_batch_step: bad arguments");
        step_batch(B, iterations, use_graph != 0, (hipStream_t)stream);
        if (n_active) {
            int n = 0;
            for (const auto &h : B->slots)
                if (h.phase != PH_FREE && h.phase != PH_DONE) n++;
            *n_active = n;
        }
        return SEM_OK;
    });
}

sem_status sem_batch_finished(const sem_batch *B, int *slots, int capacity, int *n)
{
    return bguard([&]() -> sem_status {
        if (!B || !n) fail(SEM_EINVAL, "sem_batch_finished: null argument");
        int c = 0;
        for (int id = 0; id < B->max_slots; ++id)
            if (B->slots[id].phase == PH_DONE) {
                if (slots && c < capacity) slots[c] = id;
                c++;
            }
        *n = c;
        return SEM_OK;
    });
}

sem_status sem_batch_retire(sem_batch *B, int slot, sem_solve_stats *stats)
{
    return bguard([&]() -> sem_status {
        if (!B || slot < 0 || slot >= B->max_slots) fail(SEM_EINVAL, "sem_batch_retire: bad slot");
        HostSlot &h = B->slots[slot];
        if (h.phase == PH_FREE) fail(SEM_EINVAL, "sem_batch_retire: slot is free");
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->status = h.phase == PH_DONE ? h.status : SEM_ENOCONV;
            stats->iterations = h.iters;
            stats->outer_iterations = h.opts.precision == SEM_PREC_MIXED ? h.outer : h.restarts + 1;
            stats->rel_residual = h.rel;
            stats->bnorm = h.bb > 0 ? std::sqrt(h.bb) : 0.0;
            stats->seconds = h.seconds;
        }
        retire_slot(B, slot);
        return SEM_OK;
    });
}

sem_status sem_batch_solve(sem_batch *B, sem_mesh *const *meshes, int n, const double *const *b, double *const *x,
                           const sem_solve_opts *opts, sem_solve_stats *stats, void *stream)
{
    return bguard([&]() -> sem_status {
        if (!B || !meshes || !b || !x || n < 0) fail(SEM_EINVAL, "sem_batch_solve: null argument");
        if (n > B->max_slots) fail(SEM_EBUDGET, "sem_batch_solve: more systems than slots");
        hipStream_t s = (hipStream_t)stream;
        sem_solve_opts o;
        sem_solve_opts_default(&o);
        if (opts) o = *opts;
        std::vector<int> ids(n);
        for (int i = 0; i < n; ++i) {
            sem_status st = sem_batch_admit(B, meshes[i], b[i], x[i], &o, &ids[i], stream);
            if (st != SEM_OK) {
                for (int q = 0; q < i; ++q) retire_slot(B, ids[q]);
                return st;
            }
        }
        const int k = std::max(1, o.poll_every);
        for (;;) {
            step_batch(B, k, o.use_graph != 0, s);
            bool all = true;
            for (int id : ids)
                if (B->slots[id].phase != PH_DONE) all = false;
            if (all) break;
        }
        SEM_HIP(hipStreamSynchronize(s));
        sem_status worst = SEM_OK;
        for (int i = 0; i < n; ++i) {
            sem_solve_stats st{};
            sem_batch_retire(B, ids[i], &st);
            if (stats) stats[i] = st;
            if (st.status != SEM_OK && worst == SEM_OK) worst = st.status;
        }
        return worst;
    });
}

sem_status sem_batch_tune(sem_batch *B, sem_mesh *const *meshes, int n, void *stream)
{
    return bguard([&]() -> sem_status {
        if (!B || (!meshes && n > 0) || n < 0) fail(SEM_EINVAL, "sem_batch_tune: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        for (int id = 0; id < B->max_slots; ++id)
            if (B->slots[id].phase != PH_FREE) fail(SEM_EINVAL, "sem_batch_tune: the batch must be empty");
        if (n > B->max_slots) n = B->max_slots;
        // scratch right-hand sides and solutions (zeros) for the timing slots
        size_t maxnl = 0;
        for (int i = 0; i < n; ++i) maxnl = std::max<size_t>(maxnl, (size_t)meshes[i]->h.nL);
        double *zb = nullptr, *zx = nullptr;
        SEM_HIP(hipMalloc(&zb, std::max<size_t>(maxnl, 1) * 8));
        SEM_HIP(hipMalloc(&zx, std::max<size_t>(maxnl, 1) * 8));
        SEM_HIP(hipMemsetAsync(zb, 0, maxnl * 8, s));
        SEM_HIP(hipMemsetAsync(zx, 0, maxnl * 8, s));
        hipEvent_t e0, e1;
        SEM_HIP(hipEventCreate(&e0));
        SEM_HIP(hipEventCreate(&e1));
        sem_solve_opts o;
        sem_solve_opts_default(&o);
        std::vector<int> ids;
        auto cleanup = [&]() {
            for (int id : ids) retire_slot(B, id);
            ids.clear();
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            hipFree(zb);
            hipFree(zx);
        };
        try {
            // time the CG operator (MODE 2) of a set of slots in precision prec
            // (the slots' CG states are zero: beta = alpha = 0, not done)
            auto time_group = [&](const std::vector<int> &grp, int prec) {
                Group &g = B->gres;
                g.prec = prec;
                group_build(B, g, grp, s);
                const GroupDev gd = g.dev();
                const BatchLaunch Lc = launch_for(B, g);
                SEM_HIP(batch_ax(prec, 2, B->d_desc, gd, Lc, s));
                // best of three runs of five launches
                double best = 1e300;
                for (int run = 0; run < 3; ++run) {
                    SEM_HIP(hipEventRecord(e0, s));
                    for (int r = 0; r < 5; ++r) SEM_HIP(batch_ax(prec, 2, B->d_desc, gd, Lc, s));
                    SEM_HIP(hipEventRecord(e1, s));
                    SEM_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    SEM_HIP(hipEventElapsedTime(&ms, e0, e1));
                    best = std::min(best, (double)ms);
                }
                g.prec = 0;
                return best;
            };
            bool all32 = true;
            for (int i = 0; i < n; ++i) {
                sem_solve_opts oi = o;
                oi.precision = meshes[i]->with_fp32 ? SEM_PREC_MIXED : SEM_PREC_FP64;
                all32 = all32 && meshes[i]->with_fp32;
                ids.push_back(admit_slot(B, meshes[i], zb, zx, oi, s));
            }
            // elements per tile, one order and precision at a time
            for (int N = 1; N <= SEM_MAX_ORDER; ++N) {
                std::vector<int> grp;
                bool grp32 = true;
                for (int id : ids)
                    if (B->h_desc[id].N == N) {
                        grp.push_back(id);
                        grp32 = grp32 && B->slots[id].mesh->with_fp32;
                    }
                if (grp.empty()) continue;
                const int P2 = (N + 1) * (N + 1), P3 = P2 * (N + 1);
                for (int prec = 0; prec < (grp32 ? 2 : 1); ++prec) {
                    int emax = (N >= 10 ? 256 : 512) / P2;
                    while (emax > 1 && (size_t)3 * emax * P3 * sizeof(double) > 150 * 1024) --emax;
                    double best = 1e300;
                    int best_e = default_operator_epw(N, prec == 1);
                    for (int e = 1; e <= emax; ++e) {
                        if (emax > 8 && e != 1 && e != emax && (e & (e - 1)) != 0 && e != best_e) continue;
                        B->epw[prec][N] = e;
                        const double t = time_group(grp, prec);
                        if (t < best * 0.995) {
                            best = t;
                            best_e = e;
                        }
                    }
                    B->epw[prec][N] = best_e;
                }
            }
            // (the persistent grid stays at its default: a grid tuned on one
            // precision's launches underfills the GPU for the other's)
            for (Group *g : {&B->g64, &B->g32})
                if (g->graph) {
                    hipGraphExecDestroy(g->graph);
                    g->graph = nullptr;
                }
        } catch (...) {
            cleanup();
            throw;
        }
        cleanup();
        SEM_HIP(hipStreamSynchronize(s));
        return SEM_OK;
    });
}

sem_status sem_batch_set_epw(sem_batch *B, int N, int epw)
{
    return bguard([&]() -> sem_status {
        if (!B || N < 1 || N > SEM_MAX_ORDER) fail(SEM_EINVAL, "sem_batch_set_epw: bad order");
        const int P2 = (N + 1) * (N + 1);
        if (epw < 0 || epw * P2 > 512) fail(SEM_EINVAL, "sem_batch_set_epw: epw out of range");
        for (int id = 0; id < B->max_slots; ++id)
            if (B->slots[id].phase != PH_FREE) fail(SEM_EINVAL, "sem_batch_set_epw: the batch must be empty");
        B->epw[0][N] = epw;
        B->epw[1][N] = epw;
        for (Group *g : {&B->g64, &B->g32})
            if (g->graph) {
                hipGraphExecDestroy(g->graph);
                g->graph = nullptr;
            }
        return SEM_OK;
    });
}

sem_status sem_batch_set_grid(sem_batch *B, int ax_grid, int vec_grid)
{
    return bguard([&]() -> sem_status {
        if (!B || ax_grid < 0 || vec_grid < 0) fail(SEM_EINVAL, "sem_batch_set_grid: bad arguments");
        for (int id = 0; id < B->max_slots; ++id)
            if (B->slots[id].phase != PH_FREE) fail(SEM_EINVAL, "sem_batch_set_grid: the batch must be empty");
        const int cap = persistent_grid_cap_public();
        B->L.ax_grid = ax_grid > 0 ? ax_grid : cap;
        B->L.vec_grid = vec_grid > 0 ? vec_grid : cap;
        for (Group *g : {&B->g64, &B->g32, &B->gres})
            if (g->graph) {
                hipGraphExecDestroy(g->graph);
                g->graph = nullptr;
            }
        return SEM_OK;
    });
}

sem_status sem_batch_get_grid(const sem_batch *B, int *ax_grid, int *vec_grid)
{
    return bguard([&]() -> sem_status {
        if (!B || !ax_grid || !vec_grid) fail(SEM_EINVAL, "sem_batch_get_grid: bad arguments");
        *ax_grid = B->L.ax_grid;
        *vec_grid = B->L.vec_grid;
        return SEM_OK;
    });
}

sem_status sem_batch_get_epw(const sem_batch *B, int N, int precision, int *epw)
{
    return bguard([&]() -> sem_status {
        if (!B || !epw || N < 1 || N > SEM_MAX_ORDER || (precision != SEM_FP64 && precision != SEM_FP32))
            fail(SEM_EINVAL, "sem_batch_get_epw: bad arguments");
        *epw = batch_epw(B, N, precision == SEM_FP32 ? 1 : 0);
        return SEM_OK;
    });
}

}  // extern "C"
