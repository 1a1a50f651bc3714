// api.cpp -- the C ABI (include/sem.h): mesh set-up and upload, operators,
// and the Jacobi-PCG drivers (FP64, and FP32-inner / FP64-outer defect
// correction).  All arithmetic of the path runs in the kernels of
// kernels.hip; this file only allocates, uploads and sequences launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "axgs_host.hpp"
#include "coarse.hpp"
#include "kernels.hpp"
#include "schwarz.hpp"
#include "sem_internal.hpp"

namespace sem {

hipError_t upload_batch_dtables(const double *d64, const float *d32, hipStream_t s);

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

void fail(sem_status st, const std::string &msg)
{
    set_error(msg);
    throw Failure{st};
}

void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        const sem_status st = (e == hipErrorOutOfMemory) ? SEM_ENOMEM : SEM_EHIP;
        fail(st, std::string(what) + ": " + hipGetErrorString(e));
    }
}

template <typename F>
static sem_status guarded(F &&f)
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
    } catch (...) {
        set_error("unknown internal error");
        return SEM_EINVAL;
    }
}

template <typename T>
static T *dalloc(sem_mesh *m, size_t count)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    SEM_HIP(hipMalloc(&p, bytes));
    m->allocations.push_back(p);
    m->device_bytes += bytes;
    return static_cast<T *>(p);
}

static void upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    SEM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}

// Elements per workgroup of the operator: the count that fills the 64-wide
// waves best (ties: the smaller count), within 150 KB of LDS and a lane
// budget -- FP64: 512 (256 from N = 10 on, where the kernel runs one wave
// per SIMD); FP32 (lighter kernels, more waves per SIMD): 256.
int default_operator_epw(int N, bool fp32)
{
    const int P2 = (N + 1) * (N + 1), P3 = P2 * (N + 1);
    const int max_lanes = (fp32 || N >= 10) ? 256 : 512;
    int best = 1;
    double best_fill = 0.0;
    for (int epw = 1; epw * P2 <= max_lanes; ++epw) {
        if ((size_t)3 * epw * P3 * sizeof(double) > 150 * 1024) break;
        const int t = epw * P2, tr = (t + 63) / 64 * 64;
        const double fill = (double)t / tr;
        if (fill > best_fill + 0.005) {
            best_fill = fill;
            best = epw;
        }
    }
    return best;
}

// The single-mesh operator from order 8 on runs the plane tile, whose LDS no
// longer bounds the tile: elements per workgroup measured fastest on pipes of
// about 10^8 points (CG operator for FP64, plain operator for FP32); beyond
// order 12 the fullest 64-lane waves.
static int default_epw(int N, bool fp32 = false)
{
    // FP64 N=7: the plane-tile plain operator is fastest at 4 elements per
    // workgroup, and the CG operator (whole-element tile) runs as fast there
    if (N == 7 && !fp32) return 4;
    if (N < 8) return default_operator_epw(N, fp32);
    static const int f64[] = {3, 1, 2, 3, 3}, f32[] = {3, 5, 2, 3, 3};
    if (N <= 12) return fp32 ? f32[N - 8] : f64[N - 8];
    const int P2 = (N + 1) * (N + 1);
    int best = 1;
    double best_fill = 0.0;
    for (int epw = 1; epw * P2 <= 512; ++epw) {
        const int t = epw * P2, tr = (t + 63) / 64 * 64;
        if ((double)t / tr > best_fill + 0.005) {
            best_fill = (double)t / tr;
            best = epw;
        }
    }
    return best;
}

// FP64 plain operator (modes 0, 1): at N = 9 the plane tile runs 5% faster at
// five elements per workgroup, where the CG operator loses 2% (it stays at
// one); elsewhere the two share the setting.
static int default_plain_epw(int N) { return N == 9 ? 5 : default_epw(N); }

// Derivative matrices of every order in the kernels' constant table, once
// per device.
static void ensure_dtables(hipStream_t s)
{
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    SEM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)done.size() <= dev) done.resize(dev + 1, 0);
    if (done[dev]) return;
    std::vector<double> d64;
    for (int N = 1; N <= SEM_MAX_ORDER; ++N) {
        std::vector<double> xi, w, D;
        gll_rule(N, xi, w);
        lagrange_derivative(xi, D);
        if ((int)d64.size() != dtable_offset_host(N)) fail(SEM_EINVAL, "derivative table layout");
        d64.insert(d64.end(), D.begin(), D.end());
    }
    std::vector<float> d32(d64.begin(), d64.end());
    SEM_HIP(upload_dtables(d64.data(), d32.data(), s));
    SEM_HIP(upload_batch_dtables(d64.data(), d32.data(), s));
    SEM_HIP(upload_axgs_dtables(d64.data(), d32.data(), s));
    SEM_HIP(hipStreamSynchronize(s));
    done[dev] = 1;
}

void ensure_dtables_all(hipStream_t s) { ensure_dtables(s); }
int persistent_grid_cap_public();

// Persistent operator grid: a few resident workgroups per compute unit.
static int persistent_grid_cap()
{
    int dev = 0;
    SEM_HIP(hipGetDevice(&dev));
    int cus = 0;
    SEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(64, cus * 16);
}

int persistent_grid_cap_public() { return persistent_grid_cap(); }

static void require_device_gfx950()
{
    int dev = 0;
    SEM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SEM_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(SEM_EHIP, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
}

static void ensure_solve_space(sem_mesh *m, bool need32)
{
    const int64_t nL = m->h.nL;
    if (!m->r64) {
        m->r64 = dalloc<double>(m, nL);
        m->p64 = dalloc<double>(m, nL);
        m->w64 = dalloc<double>(m, nL);
        m->x64 = dalloc<double>(m, nL);
    }
    if (need32 && !m->r32) {
        m->x32 = dalloc<float>(m, nL);
        m->r32 = dalloc<float>(m, nL);
        m->p32 = dalloc<float>(m, nL);
        m->w32 = dalloc<float>(m, nL);
    }
}

static hipStream_t cap_stream(sem_mesh *m)
{
    if (!m->capture_stream) SEM_HIP(hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking));
    return m->capture_stream;
}

// --- building blocks --------------------------------------------------------
template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static const double *G(sem_mesh *m) { return m->G64; }
    static const double *inv(sem_mesh *m) { return m->inv64; }
    static double *x(sem_mesh *m) { return m->x64; }
    static double *r(sem_mesh *m) { return m->r64; }
    static double *p(sem_mesh *m) { return m->p64; }
    static double *w(sem_mesh *m) { return m->w64; }
    static PcgState *st(sem_mesh *m) { return m->state; }
    static const double *h1(sem_mesh *m) { return m->helm ? m->h1_64 : nullptr; }
    static const double *h2b(sem_mesh *m) { return m->helm ? m->h2b64 : nullptr; }
};
template <>
struct Prec<float> {
    static const float *G(sem_mesh *m) { return m->G32; }
    static const float *inv(sem_mesh *m) { return m->inv32; }
    static float *x(sem_mesh *m) { return m->x32; }
    static float *r(sem_mesh *m) { return m->r32; }
    static float *p(sem_mesh *m) { return m->p32; }
    static float *w(sem_mesh *m) { return m->w32; }
    static PcgState *st(sem_mesh *m) { return m->state + 1; }
    static const float *h1(sem_mesh *m) { return m->helm ? m->h1_32 : nullptr; }
    static const float *h2b(sem_mesh *m) { return m->helm ? m->h2b32 : nullptr; }
};

// elements per workgroup of the operator kernel in use for precision T
template <typename T>
static int op_epw(const sem_mesh *m)
{
    return sizeof(T) == 8 ? m->ax_epw : m->ax_epw32;
}
// ... of the plain operator (modes 0, 1)
template <typename T>
static int plain_epw(const sem_mesh *m)
{
    return sizeof(T) == 8 ? m->ax_epw_plain : m->ax_epw32;
}

// the CG iteration of precision T adds the coarse correction
template <typename T>
static bool coarse_cg(const sem_mesh *m) { return m->coarse != nullptr; }
// the CG iteration of precision T takes its local part from the Schwarz solves (FP64)
template <typename T>
static bool schwarz_cg(const sem_mesh *m) { return sizeof(T) == 8 && m->schwarz != nullptr; }

// operator mode of the CG iteration: 2 Jacobi, 3 Jacobi + coarse, 4 Schwarz,
// 5 Schwarz + coarse
template <typename T>
static int cg_mode(const sem_mesh *m) { return (schwarz_cg<T>(m) ? 4 : 2) + (coarse_cg<T>(m) ? 1 : 0); }

// elements per workgroup of the column kernel for precision T
template <typename T>
static int column_epw(const sem_mesh *m) { return sizeof(T) == 8 ? m->ax_epw : m->ax_epw32; }

// elements per workgroup of the CG operator launch (modes 3-5 run the column kernel)
template <typename T>
static int cg_epw(const sem_mesh *m) { return cg_mode<T>(m) > 2 ? column_epw<T>(m) : op_epw<T>(m); }

// launches the operator; returns its workgroup count (the number of dot
// partials of modes 1-5)
template <typename T>
static AxParams<T> ax_params(sem_mesh *m, int mode, const T *in, T *out)
{
    AxParams<T> a{};
    a.E = m->h.E;
    a.epw = mode >= 3 ? column_epw<T>(m) : (mode <= 1 ? plain_epw<T>(m) : op_epw<T>(m));
    a.grid_cap = m->ax_grid_cap;
    a.G = Prec<T>::G(m);
    a.in = in;
    a.out = out;
    a.partial = m->partials;
    a.h1 = Prec<T>::h1(m);
    a.h2b = Prec<T>::h2b(m);
    if (mode >= 2) {
        a.invdiag = Prec<T>::inv(m);
        a.p = Prec<T>::p(m);
        a.x = Prec<T>::x(m);
        a.st = Prec<T>::st(m);
    }
    if (mode == 3 || mode == 5) {
        a.evert = m->coarse->evert;
        a.z0 = m->coarse->z0;
        a.cq = m->coarse->qw;
    }
    return a;
}

template <typename T>
static int64_t enqueue_ax(sem_mesh *m, int mode, const T *in, T *out, hipStream_t s, double *partial = nullptr,
                          int64_t partial_cap = 0)
{
    AxParams<T> a = ax_params<T>(m, mode, in, out);
    if (partial) a.partial = partial;
    if (partial_cap > 0 && partial_cap < a.grid_cap) a.grid_cap = (int)partial_cap;  // never more partials
    int64_t grid = 0;
    SEM_HIP(launch_ax<T>(m->h.N, mode, a, s, &grid));
    return grid;
}

template <typename T>
static void enqueue_gs(sem_mesh *m, T *v, const PcgState *st, hipStream_t s)
{
    if (m->gs_lattice_ok && m->gs_kind != SEM_GS_PLAN)
        SEM_HIP(launch_gs_lattice<T>(m->gsl, v, st, s, m->gs_kind == SEM_GS_STREAM));
    else
        SEM_HIP(launch_gs<T>(m->gsplan, m->gs_off, m->gs_idx, v, false, st, s));
}

// --- fused operator and gather-scatter ---------------------------------------
static void axgs_drop(AxgsShape &sh)
{
    if (sh.owns_plan) {
        hipFree(sh.res_off);
        hipFree(sh.res_idx);
    }
    sh = AxgsShape();
}

static void axgs_reset(sem_mesh *m)
{
    if (!m->axgs) return;
    // a shape that shares the other's plan goes first
    for (int q = 0; q < 2; ++q)
        if (!m->axgs->shape[q].owns_plan) axgs_drop(m->axgs->shape[q]);
    for (int q = 0; q < 2; ++q) axgs_drop(m->axgs->shape[q]);
}

// The launch shape and residual plan of precision T (built by
// axgs_build at set-up and on a change of configuration, never inside a
// launch sequence, which may be under graph capture); nullptr when the fused
// kernel does not apply (disabled, order outside its range, no tile fits).
template <typename T>
static AxgsShape *axgs_shape(sem_mesh *m)
{
    AxgsSpace *A = m->axgs;
    if (!A || !A->enabled) return nullptr;
    AxgsShape &sh = A->shape[sizeof(T) == 8 ? 0 : 1];
    return sh.ready == 1 ? &sh : nullptr;
}

template <typename T>
static void axgs_build_shape(sem_mesh *m)
{
    AxgsSpace *A = m->axgs;
    const HostMesh &h = m->h;
    const int prec = sizeof(T) == 8 ? 0 : 1;
    AxgsShape &sh = A->shape[prec];
    if (sh.ready) return;
    sh.ready = -1;  // not usable unless completed below
    if (!A->enabled || !axgs_order_supported(h.N)) return;
    const int P2 = h.P * h.P;
    const size_t elem = sizeof(T);
    int dev = 0, cus = 0, lds_cap = 0;
    SEM_HIP(hipGetDevice(&dev));
    SEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SEM_HIP(hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lds_limit = (size_t)lds_cap - 4096;  // static LDS of the kernel
    // elements per tile, with or without the y line buffer, among the counts
    // that keep at least three quarters of the most resident waves any count
    // reaches: the largest of at most 256 lanes if its lanes fill at least
    // 90% of its waves, else the fullest waves (then the larger count).
    // Larger tiles carry fewer per-tile costs: on the pipe at N=7 four
    // elements per tile and nine lines per workgroup ran 1.92 ms, one
    // element 2.29 ms, eight 2.23 ms; at N=9 five (500 of 512 lanes) ran
    // 2.33 ms, two (200 of 256) 2.76 ms.
    auto pick = [&](bool yon, int &best_e, int &best_blocks) {
        best_e = 0;
        best_blocks = 0;
        int resident[513] = {0};
        int most = 0;
        for (int e = 1; e * P2 <= 512; ++e) {
            if (A->req_epw && e != A->req_epw) continue;
            const size_t lds = axgs_lds_bytes(h.N, e, h.nel[0], yon, elem);
            if (lds > lds_limit) continue;
            const int blocks = axgs_blocks_per_cu<T>(h.N, 2, m->helm != 0, e, lds);
            if (blocks < 1) continue;
            resident[e] = blocks * ((e * P2 + 63) / 64);
            most = std::max(most, resident[e]);
        }
        auto fill = [&](int e) { return (double)(e * P2) / (((e * P2 + 63) / 64) * 64); };
        for (int e = 1; e * P2 <= 256; ++e)
            if (resident[e] > 0 && 4 * resident[e] >= 3 * most && fill(e) >= 0.9) best_e = e;
        if (best_e == 0) {
            double best_fill = -1.0;
            for (int e = 1; e * P2 <= 512; ++e)
                if (resident[e] > 0 && 4 * resident[e] >= 3 * most && fill(e) >= best_fill - 1e-9) {
                    best_fill = fill(e);
                    best_e = e;
                }
        }
        if (best_e > 0) best_blocks = resident[best_e] / ((best_e * P2 + 63) / 64);
    };
    const int64_t n_lines = (int64_t)h.nel[1] * h.nel[2];
    const int64_t cap = m->n_partials - 64;
    // one line per workgroup leaves no y-face to sum on-chip: no line buffer
    bool best_y = A->req_lines != 1 && h.nel[1] > 1;
    int best_e = 0, best_blocks = 0;
    if (best_y) pick(true, best_e, best_blocks);
    if (best_e == 0) {
        best_y = false;
        pick(false, best_e, best_blocks);
    }
    if (best_e == 0) return;  // no tile shape fits the LDS
    int Lw = A->req_lines ? A->req_lines : axgs_pick_lines(n_lines, (int64_t)best_blocks * cus, cap);
    if (Lw == 1 && best_y) {
        best_y = false;
        pick(false, best_e, best_blocks);
        if (best_e == 0) return;
    }
    if ((n_lines + Lw - 1) / Lw > cap) fail(SEM_EINVAL, "fused operator: more workgroups than dot partials");
    sh.epw = best_e;
    sh.lines_per_wg = Lw;
    sh.y_onchip = best_y ? 1 : 0;
    sh.grid = (n_lines + Lw - 1) / Lw;
    sh.L = axgs_lattice(h, best_e, Lw, best_y);
    const AxgsShape &other = A->shape[1 - prec];
    if (other.ready == 1 && other.lines_per_wg == Lw && other.y_onchip == sh.y_onchip) {
        sh.res = other.res;
        sh.res_copies = other.res_copies;
        sh.res_off = other.res_off;
        sh.res_idx = other.res_idx;
        sh.owns_plan = false;
    } else {
        std::vector<int32_t> off, idx;
        axgs_residual_plan(h, Lw, best_y, off, idx);
        sh.res.n_sum = sh.res.n_ids = (int64_t)off.size() - 1;
        sh.res_copies = (int64_t)idx.size();
        SEM_HIP(hipMalloc((void **)&sh.res_off, sizeof(int32_t) * off.size()));
        sh.owns_plan = true;
        if (hipMalloc((void **)&sh.res_idx, sizeof(int32_t) * std::max<size_t>(idx.size(), 1)) != hipSuccess) {
            hipFree(sh.res_off);
            sh = AxgsShape();
            fail(SEM_ENOMEM, "fused operator: residual plan");
        }
        hipStream_t s = nullptr;
        SEM_HIP(hipMemcpyAsync(sh.res_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s));
        if (!idx.empty())
            SEM_HIP(hipMemcpyAsync(sh.res_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipStreamSynchronize(s));
    }
    sh.ready = 1;
}

// both precisions' shapes (FP32 with the FP32 copies)
static void axgs_build(sem_mesh *m)
{
    if (!m->axgs) return;
    axgs_build_shape<double>(m);
    if (m->with_fp32) axgs_build_shape<float>(m);
}

// The fused kernel (modes 0 and 2); returns its workgroup count (the dot
// partials of mode 2).  The residual gather-scatter follows with enqueue_axgs_rest.
template <typename T>
static int64_t enqueue_axgs_fused(sem_mesh *m, AxgsShape &sh, int mode, const T *in, T *out, hipStream_t s)
{
    AxParams<T> a = ax_params<T>(m, mode, in, out);
    a.epw = sh.epw;
    a.grid_cap = (int)std::min<int64_t>(m->n_partials - 64, INT32_MAX);
    int64_t grid = 0;
    SEM_HIP(launch_axgs<T>(m->h.N, mode, a, sh.L, s, &grid));
    return grid;
}

template <typename T>
static void enqueue_axgs_rest(AxgsShape &sh, T *out, const PcgState *st, hipStream_t s)
{
    SEM_HIP(launch_gs<T>(sh.res, sh.res_off, sh.res_idx, out, false, st, s));
}

// w = mask(Q Q^T A_L u): the fused kernel and its residual plan where it
// applies, else the operator and the full gather-scatter
template <typename T>
static void enqueue_ax_gs(sem_mesh *m, const T *in, T *out, hipStream_t s)
{
    if (AxgsShape *sh = axgs_shape<T>(m)) {
        enqueue_axgs_fused<T>(m, *sh, 0, in, out, s);
        enqueue_axgs_rest<T>(*sh, out, nullptr, s);
        return;
    }
    enqueue_ax<T>(m, 0, in, out, s);
    enqueue_gs<T>(m, out, nullptr, s);
}

// Per-kernel-class timing with HIP events recorded on the launch stream.
struct Profiler {
    sem_mesh *m = nullptr;
    size_t used = 0;
    std::vector<hipEvent_t> marks;  // 4 per iteration
    double ms_op = 0, ms_gs = 0, ms_up = 0;
    int launches = 0;
    hipEvent_t mark(hipStream_t s)
    {
        if (used == m->events.size()) {
            hipEvent_t e;
            SEM_HIP(hipEventCreate(&e));
            m->events.push_back(e);
        }
        hipEvent_t e = m->events[used++];
        SEM_HIP(hipEventRecord(e, s));
        marks.push_back(e);
        return e;
    }
    void flush(hipStream_t s)
    {
        if (marks.empty()) return;
        SEM_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q + 3 < marks.size(); q += 4) {
            float a = 0, b = 0, c = 0;
            SEM_HIP(hipEventElapsedTime(&a, marks[q], marks[q + 1]));
            SEM_HIP(hipEventElapsedTime(&b, marks[q + 1], marks[q + 2]));
            SEM_HIP(hipEventElapsedTime(&c, marks[q + 2], marks[q + 3]));
            ms_op += a; ms_gs += b; ms_up += c;
            launches++;
        }
        marks.clear();
        used = 0;
    }
};

// one CG iteration: w = A p (p updated from z and beta first), gs, alpha,
// x/r update with <r,z>, <r,r>, beta
template <typename T>
static void enqueue_iterations(sem_mesh *m, int k, hipStream_t s, Profiler *prof = nullptr)
{
    PcgState *st = Prec<T>::st(m);
    const bool coarse = coarse_cg<T>(m), schwarz = schwarz_cg<T>(m);
    const int mode = cg_mode<T>(m);
    const int64_t nL = m->h.nL;
    const int64_t ub = update_blocks(nL);
    // the Jacobi part of <r,z> comes from the update unless Schwarz supplies z
    const T *jinv = schwarz ? nullptr : Prec<T>::inv(m);
    T *zs = nullptr;
    if constexpr (sizeof(T) == 8) zs = schwarz ? m->schwarz->zs : nullptr;
    // the Jacobi iteration runs the fused operator and gather-scatter where it applies
    AxgsShape *fused = mode == 2 ? axgs_shape<T>(m) : nullptr;
    // Jacobi on a lattice mesh: the update sums w's copies itself
    const bool update_gs = mode == 2 && !fused && !coarse && !schwarz && m->h.N >= 3 && m->gs_lattice_ok &&
                           m->gs_kind != SEM_GS_PLAN && m->h.nL < INT32_MAX;
    for (int it = 0; it < k; ++it) {
        if (prof) prof->mark(s);
        int64_t axb = 0;
        if (fused) {
            axb = enqueue_axgs_fused<T>(m, *fused, 2, Prec<T>::r(m), Prec<T>::w(m), s);
            if (prof) prof->mark(s);
            enqueue_axgs_rest<T>(*fused, Prec<T>::w(m), st, s);
        } else {
            axb = enqueue_ax<T>(m, mode, schwarz ? zs : Prec<T>::r(m), Prec<T>::w(m), s);
            if (prof) prof->mark(s);
            if (!update_gs) enqueue_gs<T>(m, Prec<T>::w(m), st, s);
        }
        if (prof) prof->mark(s);
        SEM_HIP(launch_reduce_sigma(m->partials, axb, st, s));
        int64_t pairs = ub;
        if (coarse) {
            // restriction fused into the update; <r, P z0> = <P^T r, z0>: the
            // coarse solve's pairs follow the update's
            pairs = coarse_update<T>(m, Prec<T>::r(m), Prec<T>::w(m), Prec<T>::inv(m), st, m->partials, !schwarz, s);
            pairs += coarse_solve(m, m->partials + 2 * pairs, st, s);
        } else if (update_gs) {
            SEM_HIP(launch_pcg_update_gs<T>(m->gsl, m->h.N, m->h.E, st, Prec<T>::r(m), Prec<T>::w(m), Prec<T>::inv(m),
                                            m->mult, m->partials, s));
            pairs = update_elem_blocks(m->h.E);
        } else if (m->h.N >= 3 && (sizeof(T) == 8 || m->gs_lattice_ok)) {
            // element by element (the FP32 update of a non-lattice mesh keeps
            // the paired entries); on a lattice mesh the same workgroup
            // partials as the update with the gather-scatter folded in
            SEM_HIP(launch_pcg_update_elem<T>(m->h.N, m->h.E, st, Prec<T>::r(m), Prec<T>::w(m), jinv, m->mult,
                                              m->partials, s));
            pairs = update_elem_blocks(m->h.E);
        } else {
            SEM_HIP(launch_pcg_update<T>(nL, st, Prec<T>::r(m), Prec<T>::w(m), jinv, m->mult, m->partials, s));
        }
        if constexpr (sizeof(T) == 8) {
            // Schwarz local solves of the new r; their <r, z> pairs follow
            if (schwarz) pairs += schwarz_apply(m, m->r64, zs, m->partials + 2 * pairs, st, s);
        }
        SEM_HIP(launch_reduce_rho(m->partials, pairs, st, s));
        if (prof) prof->mark(s);
    }
    if (prof) prof->flush(s);
}

template <typename T>
static void run_iterations(sem_mesh *m, int k, bool use_graph, hipStream_t s, Profiler *prof = nullptr)
{
    if (prof || !use_graph) {
        enqueue_iterations<T>(m, k, s, prof);
        return;
    }
    const int slot = sizeof(T) == 8 ? 0 : 1;
    // graph key: tile shape and kernel (a change of the coarse space drops the graphs)
    const int epw = cg_epw<T>(m) + 1024 * (coarse_cg<T>(m) ? 2 : 0);
    if (!m->graph[slot] || m->graph_k[slot] != k || m->graph_epw[slot] != epw ||
        m->graph_grid[slot] != m->ax_grid_cap) {
        if (m->graph[slot]) {
            SEM_HIP(hipGraphExecDestroy(m->graph[slot]));
            m->graph[slot] = nullptr;
        }
        hipStream_t cs = cap_stream(m);
        hipGraph_t g = nullptr;
        SEM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_iterations<T>(m, k, cs);
        } catch (...) {
            hipStreamEndCapture(cs, &g);
            if (g) hipGraphDestroy(g);
            throw;
        }
        SEM_HIP(hipStreamEndCapture(cs, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        SEM_HIP(e);
        m->graph[slot] = ex;
        m->graph_k[slot] = k;
        m->graph_epw[slot] = epw;
        m->graph_grid[slot] = m->ax_grid_cap;
    }
    SEM_HIP(hipGraphLaunch(m->graph[slot], s));
}

// cached CG graphs launch the operator and preconditioner they were captured with
static void drop_graphs(sem_mesh *m, hipStream_t s)
{
    for (int q = 0; q < 2; ++q)
        if (m->graph[q]) {
            SEM_HIP(hipStreamSynchronize(s));
            SEM_HIP(hipGraphExecDestroy(m->graph[q]));
            m->graph[q] = nullptr;
        }
}

// the coarse space follows the operator: rebuilt with the same parameters
static void rebuild_coarse(sem_mesh *m, hipStream_t s)
{
    if (!m->coarse) return;
    drop_graphs(m, s);
    const int k = m->coarse->k;
    const double frac = m->coarse->frac;
    coarse_free(m->coarse);
    m->coarse = nullptr;
    m->coarse = coarse_build(m, k, frac, s);
}

static PcgState read_state(const PcgState *st, hipStream_t s)
{
    PcgState h;
    SEM_HIP(hipMemcpyAsync(&h, st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    return h;
}

static double read_scalar(const double *d, hipStream_t s)
{
    double h = 0.0;
    SEM_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    return h;
}

// r = b - A x (FP64), then rr = <r, r> into scal[slot]
static void true_residual(sem_mesh *m, const double *b, hipStream_t s, int slot)
{
    enqueue_ax_gs<double>(m, m->x64, m->w64, s);
    SEM_HIP(launch_residual(m->h.nL, b, m->w64, m->r64, s));
    SEM_HIP(launch_dot_unique<double>(m->h.nL, m->r64, m->r64, m->mult, m->partials, m->scal + slot, s));
}

// CG start from the current r: rho = <r, M^-1 r>, rr, flags; p = 0
template <typename T>
static void pcg_start(sem_mesh *m, double stop2, int limit, hipStream_t s)
{
    const int64_t nL = m->h.nL;
    const bool coarse = coarse_cg<T>(m), schwarz = schwarz_cg<T>(m);
    if (coarse || schwarz) {
        const int64_t vb = vec_blocks(nL);
        int64_t pairs = vb;
        SEM_HIP(launch_pcg_init_partials<T>(nL, Prec<T>::r(m), schwarz ? nullptr : Prec<T>::inv(m), m->mult,
                                            m->partials, s));
        if (coarse) {
            coarse_restrict<T>(m, Prec<T>::r(m), Prec<T>::inv(m), s);
            pairs += coarse_solve(m, m->partials + 2 * pairs, nullptr, s);
        }
        if constexpr (sizeof(T) == 8) {
            if (schwarz) pairs += schwarz_apply(m, m->r64, m->schwarz->zs, m->partials + 2 * pairs, nullptr, s);
        }
        SEM_HIP(launch_reduce_init(m->partials, pairs, Prec<T>::st(m), stop2, limit, s));
        SEM_HIP(hipMemsetAsync(Prec<T>::p(m), 0, sizeof(T) * nL, s));
        return;
    }
    SEM_HIP(launch_pcg_init<T>(nL, Prec<T>::r(m), Prec<T>::inv(m), m->mult, m->partials, Prec<T>::st(m), stop2,
                               limit, s));
    SEM_HIP(hipMemsetAsync(Prec<T>::p(m), 0, sizeof(T) * nL, s));
}

// Plain CG loop on precision T from the current r (x, p set by the caller);
// returns the final device state.
template <typename T>
static PcgState cg_loop(sem_mesh *m, double stop2, int limit, int poll, bool graph, hipStream_t s,
                        Profiler *prof = nullptr)
{
    pcg_start<T>(m, stop2, limit, s);
    PcgState hs = read_state(Prec<T>::st(m), s);
    while (!hs.done) {
        run_iterations<T>(m, poll, graph, s, prof);
        hs = read_state(Prec<T>::st(m), s);
    }
    SEM_HIP(launch_pcg_finish<T>(m->h.nL, Prec<T>::st(m), Prec<T>::x(m), Prec<T>::p(m), s));
    return hs;
}

static sem_status solve_fp64(sem_mesh *m, const double *b, double *x, const sem_solve_opts &o, sem_solve_stats &out,
                             hipStream_t s)
{
    const int64_t nL = m->h.nL;
    ensure_solve_space(m, false);
    SEM_HIP(launch_dot_unique<double>(nL, b, b, m->mult, m->partials, m->scal, s));
    const double bb = read_scalar(m->scal, s);
    out.bnorm = std::sqrt(bb);
    if (o.x0_given) SEM_HIP(hipMemcpyAsync(m->x64, x, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
    else SEM_HIP(hipMemsetAsync(m->x64, 0, sizeof(double) * nL, s));
    const int poll = std::max(1, o.poll_every);

    if (o.fixed_iters > 0) {
        // throughput mode: exactly fixed_iters iterations from the current x
        if (o.x0_given) true_residual(m, b, s, 1);
        else SEM_HIP(hipMemcpyAsync(m->r64, b, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
        pcg_start<double>(m, -1.0, o.fixed_iters, s);
        int left = o.fixed_iters;
        Profiler prof;
        prof.m = m;
        while (left > 0) {
            const int k = std::min(left, poll);
            run_iterations<double>(m, k, o.use_graph != 0, s, o.profile ? &prof : nullptr);
            left -= k;
        }
        out.ms_operator = prof.ms_op;
        out.ms_gather_scatter = prof.ms_gs;
        out.ms_update = prof.ms_up;
        out.operator_launches = prof.launches;
        SEM_HIP(launch_pcg_finish<double>(nL, m->state, m->x64, m->p64, s));
        const PcgState hs = read_state(m->state, s);
        SEM_HIP(hipMemcpyAsync(x, m->x64, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
        SEM_HIP(hipStreamSynchronize(s));
        out.iterations = hs.iters;
        out.outer_iterations = 1;
        out.rel_residual = bb > 0 ? std::sqrt(hs.rr / bb) : 0.0;
        return hs.done == 2 ? SEM_EBREAKDOWN : SEM_OK;
    }

    sem_status status = SEM_OK;
    if (bb == 0.0) {
        SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * nL, s));
        SEM_HIP(hipStreamSynchronize(s));
        out.iterations = 0;
        out.outer_iterations = 1;
        out.rel_residual = 0.0;
        return SEM_OK;
    }
    const double stop2 = o.tol * o.tol * bb;
    Profiler prof;
    prof.m = m;
    Profiler *pp = o.profile ? &prof : nullptr;
    int total = 0, restarts = 0;
    bool have_x = o.x0_given != 0;
    double rel = 0.0;
    for (;;) {
        if (have_x) true_residual(m, b, s, 1);
        else SEM_HIP(hipMemcpyAsync(m->r64, b, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
        const PcgState hs = cg_loop<double>(m, stop2, o.max_iter - total, poll, o.use_graph != 0, s, pp);
        total += hs.iters;
        have_x = true;
        if (hs.done == 2) {
            true_residual(m, b, s, 1);
            rel = std::sqrt(read_scalar(m->scal + 1, s) / bb);
            status = SEM_EBREAKDOWN;
            set_error("sem_pcg_solve: CG breakdown (p.Ap <= 0 or not finite)");
            break;
        }
        true_residual(m, b, s, 1);
        rel = std::sqrt(read_scalar(m->scal + 1, s) / bb);
        if (rel <= o.tol) break;
        if (total >= o.max_iter || restarts == 3) {
            status = SEM_ENOCONV;
            set_error("sem_pcg_solve: no convergence within max_iter");
            break;
        }
        restarts++;
    }
    SEM_HIP(hipMemcpyAsync(x, m->x64, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
    SEM_HIP(hipStreamSynchronize(s));
    out.iterations = total;
    out.outer_iterations = restarts + 1;
    out.rel_residual = rel;
    out.ms_operator = prof.ms_op;
    out.ms_gather_scatter = prof.ms_gs;
    out.ms_update = prof.ms_up;
    out.operator_launches = prof.launches;
    return status;
}

// Relative tolerance of the next FP32 inner solve when the FP64 residual is
// rel: inner_tol, but never tighter than the reduction still needed (with a
// factor 2 of margin) -- the last refinement step then stops early.
double inner_tolerance(const sem_solve_opts &o, double rel)
{
    return std::min(0.5, std::max(o.inner_tol, 0.5 * o.tol / rel));
}

static sem_status solve_mixed(sem_mesh *m, const double *b, double *x, const sem_solve_opts &o, sem_solve_stats &out,
                              hipStream_t s)
{
    if (!m->with_fp32) fail(SEM_EINVAL, "sem_pcg_solve: mixed precision needs SEM_WITH_FP32 at set-up");
    if (m->schwarz)
        fail(SEM_EUNSUPPORTED, "sem_pcg_solve: the Schwarz local solves run in FP64 solves only");
    const int64_t nL = m->h.nL;
    ensure_solve_space(m, true);
    SEM_HIP(launch_dot_unique<double>(nL, b, b, m->mult, m->partials, m->scal, s));
    const double bb = read_scalar(m->scal, s);
    out.bnorm = std::sqrt(bb);
    if (o.x0_given) SEM_HIP(hipMemcpyAsync(m->x64, x, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
    else SEM_HIP(hipMemsetAsync(m->x64, 0, sizeof(double) * nL, s));
    const int poll = std::max(1, o.poll_every);
    const int inner_max = o.inner_max_iter > 0 ? o.inner_max_iter : o.max_iter;
    sem_status status = SEM_OK;
    int total = 0, outer = 0;
    double rel = 0.0;
    Profiler prof;
    prof.m = m;
    Profiler *pp = o.profile ? &prof : nullptr;
    if (bb == 0.0) {
        SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * nL, s));
        SEM_HIP(hipStreamSynchronize(s));
        out.iterations = 0;
        out.outer_iterations = 0;
        out.rel_residual = 0.0;
        return SEM_OK;
    }
    for (;;) {
        // FP64: r = b - A x, rr -> scal[1]
        true_residual(m, b, s, 1);
        const double rr = read_scalar(m->scal + 1, s);
        rel = std::sqrt(rr / bb);
        if (rel <= o.tol) break;
        if (total >= o.max_iter || outer >= 100) {
            status = SEM_ENOCONV;
            set_error("sem_pcg_solve: mixed refinement did not converge within max_iter");
            break;
        }
        // FP32 inner solve of A d = r / ||r|| from d = 0
        SEM_HIP(launch_to_fp32_scaled(nL, m->r64, m->scal + 1, m->r32, s));
        SEM_HIP(hipMemsetAsync(m->x32, 0, sizeof(float) * nL, s));
        const int limit = std::min(inner_max, o.max_iter - total);
        const double eta = inner_tolerance(o, rel);
        const PcgState hs = cg_loop<float>(m, eta * eta, limit, poll, o.use_graph != 0, s, pp);
        total += hs.iters;
        outer++;
        if (hs.iters == 0 && hs.done == 2) {
            status = SEM_EBREAKDOWN;
            set_error("sem_pcg_solve: FP32 inner CG broke down at its first step");
            break;
        }
        // FP64: x += ||r|| d
        SEM_HIP(launch_axpy_fp32(nL, m->x32, m->scal + 1, m->x64, s));
    }
    SEM_HIP(hipMemcpyAsync(x, m->x64, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
    SEM_HIP(hipStreamSynchronize(s));
    out.iterations = total;
    out.outer_iterations = outer;
    out.rel_residual = rel;
    out.ms_operator = prof.ms_op;
    out.ms_gather_scatter = prof.ms_gs;
    out.ms_update = prof.ms_up;
    out.operator_launches = prof.launches;
    return status;
}

}  // namespace sem

using namespace sem;

// --- dot partials of the entry point that allocates nothing -----------------
// sem_ax_noalloc keeps the operator's per-workgroup dot partials in this fixed
// device array instead of the mesh's partials buffer.  Each device holds its
// own copy until the process ends; host code uses only the address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoallocPartials = 16384;  // 128 KiB per device
static __device__ __align__(256) double scratch[kNoallocPartials];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// once per device, with that device current (called by sem_setup)
static void init_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) fail(SEM_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void *p = nullptr;
    SEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double *>(p);
}

static double *scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

extern "C" {

const char *sem_last_error(void) { return g_err.c_str(); }
const char *sem_version(void) { return "sem-mi355x 0.1 (gfx950)"; }

sem_status sem_setup(const sem_mesh_desc *desc, void *stream, sem_mesh **out)
{
    return guarded([&]() -> sem_status {
        if (!desc || !out) fail(SEM_EINVAL, "sem_setup: null argument");
        *out = nullptr;
        require_device_gfx950();
        hipStream_t s = (hipStream_t)stream;
        sem_mesh *m = new sem_mesh();
        try {
            HostMesh &h = m->h;
            build_host_mesh(*desc, h);
            h.desc = *desc;
            if (desc->vertices) {
                const size_t nv = (size_t)(desc->nel[0] + 1) * (desc->nel[1] + 1) * (desc->nel[2] + 1) * 3;
                h.vertices.assign(desc->vertices, desc->vertices + nv);
            }
            h.desc.vertices = nullptr;
            SEM_HIP(hipGetDevice(&m->device));
            init_scratch(m->device);
            m->with_fp32 = (desc->precision_flags & SEM_WITH_FP32) ? 1 : 0;
            m->ax_epw = default_epw(h.N);
            m->ax_epw32 = default_epw(h.N, true);
            m->ax_epw_plain = default_plain_epw(h.N);
            m->axgs = new AxgsSpace();
            const int64_t nL = h.nL;
            ensure_dtables(s);
            m->G64 = dalloc<double>(m, 6 * nL);
            m->B64 = dalloc<double>(m, nL);
            m->inv64 = dalloc<double>(m, nL);
            m->mult = dalloc<uint8_t>(m, nL);
            m->gid = dalloc<int32_t>(m, nL);
            m->gsplan.n_sum = h.gs_n_sum;
            m->gsplan.n_ids = h.gs_n_ids;
            {
                int faces = desc->dirichlet_faces;  // resolved as the numbering resolves it
                if (faces < 0) {
                    faces = 0;
                    for (int a = 0; a < 3; ++a)
                        if (!desc->periodic[a]) faces |= 3 << (2 * a);
                }
                m->gs_lattice_ok = gs_lattice_make(h.N, h.nel, h.periodic, faces, m->gsl) ? 1 : 0;
                m->gs_kind = SEM_GS_AUTO;
            }
            m->gs_off = dalloc<int32_t>(m, h.gs_off.size());
            m->gs_idx = dalloc<int32_t>(m, h.gs_idx.size());
            m->ax_grid_cap = persistent_grid_cap();
            // + room for the coarse dot's and the Schwarz solves' pairs behind the
            // CG partial pairs
            const int64_t np = std::max<int64_t>(std::max<int64_t>(m->ax_grid_cap, 65536),
                                                2 * (int64_t)std::max(vec_blocks(nL), update_blocks(nL))) +
                               2 * (kMaxCoarseDotBlocks + kMaxSchwarzPairs) + 64;
            m->partials = dalloc<double>(m, np);
            m->n_partials = np;
            m->state = dalloc<PcgState>(m, 2);
            m->scal = dalloc<double>(m, 8);
            std::vector<uint8_t> lmult((size_t)nL);
            for (int64_t l = 0; l < nL; ++l) lmult[l] = h.gmult[h.gid[l]];
            upload(m->G64, h.G.data(), sizeof(double) * 6 * nL, s);
            upload(m->B64, h.B.data(), sizeof(double) * nL, s);
            upload(m->inv64, h.invdiag.data(), sizeof(double) * nL, s);
            upload(m->mult, lmult.data(), nL, s);
            upload(m->gid, h.gid.data(), sizeof(int32_t) * nL, s);
            upload(m->gs_off, h.gs_off.data(), sizeof(int32_t) * h.gs_off.size(), s);
            upload(m->gs_idx, h.gs_idx.data(), sizeof(int32_t) * h.gs_idx.size(), s);
            if (m->with_fp32) {
                m->G32 = dalloc<float>(m, 6 * nL);
                m->inv32 = dalloc<float>(m, nL);
                SEM_HIP(launch_fp64_to_fp32(6 * nL, m->G64, m->G32, s));
                SEM_HIP(launch_fp64_to_fp32(nL, m->inv64, m->inv32, s));
            }
            SEM_HIP(hipMemsetAsync(m->state, 0, 2 * sizeof(PcgState), s));
            SEM_HIP(hipStreamSynchronize(s));
            axgs_build(m);
            // the device holds these now; keep only what exports need
            std::vector<double>().swap(h.G);
            std::vector<double>().swap(h.B);
            std::vector<double>().swap(h.invdiag);
            std::vector<double>().swap(h.xyz);
        } catch (...) {
            sem_free(m);
            throw;
        }
        *out = m;
        return SEM_OK;
    });
}

sem_status sem_free(sem_mesh *m)
{
    if (!m) return SEM_OK;
    for (int q = 0; q < 2; ++q)
        if (m->graph[q]) hipGraphExecDestroy(m->graph[q]);
    if (m->capture_stream) hipStreamDestroy(m->capture_stream);
    coarse_free(m->coarse);
    schwarz_free(m->schwarz);
    axgs_reset(m);
    delete m->axgs;
    for (hipEvent_t e : m->events) hipEventDestroy(e);
    for (void *p : m->allocations) hipFree(p);
    delete m;
    return SEM_OK;
}

sem_status sem_info(const sem_mesh *m, sem_mesh_info *info)
{
    return guarded([&]() -> sem_status {
        if (!m || !info) fail(SEM_EINVAL, "sem_info: null argument");
        const HostMesh &h = m->h;
        info->N = h.N;
        info->E = h.E;
        info->n_local = h.nL;
        info->n_global = h.nG;
        info->n_shared_local = h.n_shared_local;
        info->n_shared_global = h.n_shared_global;
        info->n_masked_global = h.n_masked_global;
        info->n_unmasked_global = h.nG - h.n_masked_global;
        info->gs_plan_ids = h.gs_n_ids;
        info->gs_plan_sum_ids = h.gs_n_sum;
        info->gs_plan_len = h.gs_plan_len;
        info->device_bytes = m->device_bytes;
        return SEM_OK;
    });
}

sem_status sem_export_gll(int N, double *xi, double *w, double *D)
{
    return guarded([&]() -> sem_status {
        if (N < 1 || N > SEM_MAX_ORDER) fail(SEM_EINVAL, "sem_export_gll: N out of range");
        std::vector<double> x, wt, d;
        gll_rule(N, x, wt);
        lagrange_derivative(x, d);
        if (xi) std::copy(x.begin(), x.end(), xi);
        if (w) std::copy(wt.begin(), wt.end(), w);
        if (D) std::copy(d.begin(), d.end(), D);
        return SEM_OK;
    });
}

sem_status sem_export_maps(const sem_mesh *m, int64_t *glob_id, uint8_t *mult, uint8_t *mask)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_export_maps: null mesh");
        const HostMesh &h = m->h;
        for (int64_t l = 0; l < h.nL; ++l) {
            const int32_t g = h.gid[l];
            if (glob_id) glob_id[l] = g;
            if (mult) mult[l] = h.gmult[g];
            if (mask) mask[l] = h.gmask[g];
        }
        return SEM_OK;
    });
}

sem_status sem_export_geom(const sem_mesh *m, double *G, double *B, double *invdiag)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_export_geom: null mesh");
        const HostMesh &h = m->h;
        const int64_t nL = h.nL, P3 = (int64_t)h.P * h.P * h.P;
        if (G) {
            std::vector<double> tmp((size_t)6 * nL);
            SEM_HIP(hipMemcpy(tmp.data(), m->G64, sizeof(double) * 6 * nL, hipMemcpyDeviceToHost));
            for (int64_t e = 0; e < h.E; ++e)
                for (int c = 0; c < 6; ++c)
                    std::memcpy(G + c * nL + e * P3, tmp.data() + (e * 6 + c) * P3, sizeof(double) * P3);
        }
        if (B) SEM_HIP(hipMemcpy(B, m->B64, sizeof(double) * nL, hipMemcpyDeviceToHost));
        if (invdiag) SEM_HIP(hipMemcpy(invdiag, m->inv64, sizeof(double) * nL, hipMemcpyDeviceToHost));
        return SEM_OK;
    });
}

sem_status sem_export_coords(const sem_mesh *m, double *xyz)
{
    return guarded([&]() -> sem_status {
        if (!m || !xyz) fail(SEM_EINVAL, "sem_export_coords: null argument");
        HostMesh tmp;
        sem_mesh_desc d = m->h.desc;
        d.vertices = m->h.vertices.empty() ? nullptr : m->h.vertices.data();
        build_host_coords(d, tmp);
        std::memcpy(xyz, tmp.xyz.data(), sizeof(double) * 3 * tmp.nL);
        return SEM_OK;
    });
}

sem_status sem_host_setup(const sem_mesh_desc *desc, sem_mesh_info *info, int64_t *glob_id, uint8_t *mult,
                          uint8_t *mask, double *G, double *B, double *invdiag, int32_t *gs_off, int32_t *gs_idx)
{
    return guarded([&]() -> sem_status {
        if (!desc) fail(SEM_EINVAL, "sem_host_setup: null descriptor");
        HostMesh h;
        build_host_mesh(*desc, h);
        const int64_t nL = h.nL, P3 = (int64_t)h.P * h.P * h.P;
        if (info) {
            info->N = h.N;
            info->E = h.E;
            info->n_local = nL;
            info->n_global = h.nG;
            info->n_shared_local = h.n_shared_local;
            info->n_shared_global = h.n_shared_global;
            info->n_masked_global = h.n_masked_global;
            info->n_unmasked_global = h.nG - h.n_masked_global;
            info->gs_plan_ids = h.gs_n_ids;
            info->gs_plan_sum_ids = h.gs_n_sum;
            info->gs_plan_len = h.gs_plan_len;
            info->device_bytes = 0;
        }
        for (int64_t l = 0; l < nL; ++l) {
            const int32_t g = h.gid[l];
            if (glob_id) glob_id[l] = g;
            if (mult) mult[l] = h.gmult[g];
            if (mask) mask[l] = h.gmask[g];
        }
        if (G)
            for (int64_t e = 0; e < h.E; ++e)
                for (int c = 0; c < 6; ++c)
                    std::memcpy(G + c * nL + e * P3, h.G.data() + (e * 6 + c) * P3, sizeof(double) * P3);
        if (B) std::memcpy(B, h.B.data(), sizeof(double) * nL);
        if (invdiag) std::memcpy(invdiag, h.invdiag.data(), sizeof(double) * nL);
        if (gs_off) std::memcpy(gs_off, h.gs_off.data(), sizeof(int32_t) * h.gs_off.size());
        if (gs_idx) std::memcpy(gs_idx, h.gs_idx.data(), sizeof(int32_t) * h.gs_idx.size());
        return SEM_OK;
    });
}

sem_status sem_load_geometry(sem_mesh *m, const double *G, const double *B, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !G || !B) fail(SEM_EINVAL, "sem_load_geometry: null argument");
        hipStream_t s = (hipStream_t)stream;
        HostMesh &h = m->h;
        const int64_t nL = h.nL, P3 = (int64_t)h.P * h.P * h.P;
        try {
            h.G.assign((size_t)6 * nL, 0.0);
            for (int64_t e = 0; e < h.E; ++e)
                for (int c = 0; c < 6; ++c)
                    std::memcpy(h.G.data() + (e * 6 + c) * P3, G + c * nL + e * P3, sizeof(double) * P3);
            build_jacobi(h);
            upload(m->G64, h.G.data(), sizeof(double) * 6 * nL, s);
            upload(m->B64, B, sizeof(double) * nL, s);
            upload(m->inv64, h.invdiag.data(), sizeof(double) * nL, s);
            if (m->with_fp32) {
                SEM_HIP(launch_fp64_to_fp32(6 * nL, m->G64, m->G32, s));
                SEM_HIP(launch_fp64_to_fp32(nL, m->inv64, m->inv32, s));
            }
            SEM_HIP(hipStreamSynchronize(s));
        } catch (...) {
            std::vector<double>().swap(h.G);
            std::vector<double>().swap(h.invdiag);
            throw;
        }
        std::vector<double>().swap(h.G);
        std::vector<double>().swap(h.invdiag);
        m->op_version++;
        if (m->helm) {
            // h2*B was formed with the old B: back to the Poisson form
            drop_graphs(m, s);
            m->helm = 0;
        }
        rebuild_coarse(m, s);
        return SEM_OK;
    });
}

sem_status sem_set_operator_config(sem_mesh *m, int epw, int grid)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_set_operator_config: null mesh");
        const int P2 = m->h.P * m->h.P;
        if (epw < 1 || epw * P2 > 512) fail(SEM_EINVAL, "sem_set_operator_config: epw out of range");
        if (grid < 0) fail(SEM_EINVAL, "sem_set_operator_config: negative grid");
        const int cap = grid > 0 ? grid : persistent_grid_cap();
        if (cap > m->n_partials - 64) fail(SEM_EINVAL, "sem_set_operator_config: grid larger than the partials buffer");
        m->ax_epw = epw;
        m->ax_epw32 = epw;
        m->ax_epw_plain = epw;
        m->ax_grid_cap = cap;
        return SEM_OK;
    });
}

sem_status sem_get_operator_config(const sem_mesh *m, int *epw, int *grid)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_get_operator_config: null mesh");
        if (epw) *epw = m->ax_epw;
        if (grid) *grid = m->ax_grid_cap;
        return SEM_OK;
    });
}

sem_status sem_set_gs_config(sem_mesh *m, int kind)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_set_gs_config: null mesh");
        if (kind != SEM_GS_AUTO && kind != SEM_GS_PLAN && kind != SEM_GS_STREAM)
            fail(SEM_EINVAL, "sem_set_gs_config: unknown kind");
        if (kind != m->gs_kind) {
            drop_graphs(m, nullptr);  // captured iterations hold the old kernel
            m->gs_kind = kind;
        }
        return SEM_OK;
    });
}

sem_status sem_get_gs_config(const sem_mesh *m, int *kind, int *lattice_in_use)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_get_gs_config: null mesh");
        if (kind) *kind = m->gs_kind;
        if (lattice_in_use) *lattice_in_use = m->gs_lattice_ok && m->gs_kind != SEM_GS_PLAN;
        return SEM_OK;
    });
}

sem_status sem_set_helmholtz(sem_mesh *m, const double *h1, const double *h2, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_set_helmholtz: null mesh");
        hipStream_t s = (hipStream_t)stream;
        const int64_t nL = m->h.nL;
        drop_graphs(m, s);
        const bool helm = h1 || h2;
        if (helm && !m->h1_64) {
            m->h1_64 = dalloc<double>(m, nL);
            m->h2b64 = dalloc<double>(m, nL);
            if (m->with_fp32) {
                m->h1_32 = dalloc<float>(m, nL);
                m->h2b32 = dalloc<float>(m, nL);
            }
        }
        if (helm) {
            if (h1) SEM_HIP(hipMemcpyAsync(m->h1_64, h1, sizeof(double) * nL, hipMemcpyDeviceToDevice, s));
            else SEM_HIP(launch_fill(nL, 1.0, m->h1_64, s));
            if (h2) SEM_HIP(launch_scale(nL, h2, m->B64, m->h2b64, s));
            else SEM_HIP(launch_fill(nL, 0.0, m->h2b64, s));
            if (m->with_fp32) {
                SEM_HIP(launch_fp64_to_fp32(nL, m->h1_64, m->h1_32, s));
                SEM_HIP(launch_fp64_to_fp32(nL, m->h2b64, m->h2b32, s));
            }
        }
        // Jacobi: assembled diagonal of the new operator, inverted (0 on masked nodes)
        double *diag = nullptr;
        SEM_HIP(hipMalloc(&diag, sizeof(double) * std::max<int64_t>(nL, 1)));
        try {
            SEM_HIP(launch_helm_diag(m->h.N, m->h.E, m->G64, helm ? m->h1_64 : nullptr, helm ? m->h2b64 : nullptr,
                                     diag, s));
            SEM_HIP(launch_gs<double>(m->gsplan, m->gs_off, m->gs_idx, diag, false, nullptr, s));
            SEM_HIP(launch_invert_positive(nL, diag, m->inv64, s));
            if (m->with_fp32) SEM_HIP(launch_fp64_to_fp32(nL, m->inv64, m->inv32, s));
            SEM_HIP(hipStreamSynchronize(s));
        } catch (...) {
            hipFree(diag);
            throw;
        }
        SEM_HIP(hipFree(diag));
        m->helm = helm ? 1 : 0;
        m->op_version++;
        rebuild_coarse(m, s);
        return SEM_OK;
    });
}

static void check_dtype(const sem_mesh *m, int dtype)
{
    if (dtype != SEM_FP64 && dtype != SEM_FP32) fail(SEM_EINVAL, "unknown dtype");
    if (dtype == SEM_FP32 && !m->with_fp32) fail(SEM_EINVAL, "FP32 operators need SEM_WITH_FP32 at set-up");
}

sem_status sem_ax(sem_mesh *m, int dtype, const void *u, void *w, double *opt_dot, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !u || !w) fail(SEM_EINVAL, "sem_ax: null argument");
        if (u == w) fail(SEM_EINVAL, "sem_ax: u and w must not overlap");
        check_dtype(m, dtype);
        hipStream_t s = (hipStream_t)stream;
        const int mode = opt_dot ? 1 : 0;
        const int64_t grid = dtype == SEM_FP64 ? enqueue_ax<double>(m, mode, (const double *)u, (double *)w, s)
                                               : enqueue_ax<float>(m, mode, (const float *)u, (float *)w, s);
        if (opt_dot) SEM_HIP(launch_reduce_scalar(m->partials, grid, opt_dot, s));
        return SEM_OK;
    });
}

sem_status sem_ax_noalloc(sem_mesh *m, int dtype, const void *u, void *w, double *dot, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !u || !w || !dot) fail(SEM_EINVAL, "sem_ax_noalloc: null argument");
        if (u == w) fail(SEM_EINVAL, "sem_ax_noalloc: u and w must not overlap");
        check_dtype(m, dtype);
        int dev = -1;
        SEM_HIP(hipGetDevice(&dev));
        if (dev != m->device) fail(SEM_EINVAL, "sem_ax_noalloc: the mesh lives on another device");
        double *part = scratch_of(dev);
        if (!part) fail(SEM_EHIP, "sem_ax_noalloc: no scratch address for this device");
        // the operator launches min(tiles, grid cap) workgroups, one partial each
        const int epw = dtype == SEM_FP64 ? op_epw<double>(m) : op_epw<float>(m);
        const int64_t tiles = (m->h.E + epw - 1) / epw;
        const int64_t grid = std::min<int64_t>(tiles, m->ax_grid_cap);
        if (grid > kNoallocPartials)
            fail(SEM_EINVAL, "sem_ax_noalloc: " + std::to_string(grid) + " operator workgroups exceed the " +
                                 std::to_string(kNoallocPartials) + " dot partials of the fixed scratch");
        hipStream_t s = (hipStream_t)stream;
        const int64_t launched =
            dtype == SEM_FP64 ? enqueue_ax<double>(m, 1, (const double *)u, (double *)w, s, part, kNoallocPartials)
                              : enqueue_ax<float>(m, 1, (const float *)u, (float *)w, s, part, kNoallocPartials);
        SEM_HIP(launch_reduce_scalar(part, launched, dot, s));
        return SEM_OK;
    });
}

sem_status sem_gs(sem_mesh *m, int dtype, void *v, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !v) fail(SEM_EINVAL, "sem_gs: null argument");
        check_dtype(m, dtype);
        hipStream_t s = (hipStream_t)stream;
        if (dtype == SEM_FP64) enqueue_gs<double>(m, (double *)v, nullptr, s);
        else enqueue_gs<float>(m, (float *)v, nullptr, s);
        return SEM_OK;
    });
}

sem_status sem_axgs(sem_mesh *m, int dtype, const void *u, void *w, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !u || !w) fail(SEM_EINVAL, "sem_axgs: null argument");
        if (u == w) fail(SEM_EINVAL, "sem_axgs: u and w must not overlap");
        check_dtype(m, dtype);
        hipStream_t s = (hipStream_t)stream;
        if (dtype == SEM_FP64) enqueue_ax_gs<double>(m, (const double *)u, (double *)w, s);
        else enqueue_ax_gs<float>(m, (const float *)u, (float *)w, s);
        return SEM_OK;
    });
}

sem_status sem_set_axgs_config(sem_mesh *m, int enable, int epw, int lines_per_wg)
{
    return guarded([&]() -> sem_status {
        if (!m || !m->axgs) fail(SEM_EINVAL, "sem_set_axgs_config: null mesh");
        if (enable != 0 && enable != 1) fail(SEM_EINVAL, "sem_set_axgs_config: enable must be 0 or 1");
        if (epw < 0 || lines_per_wg < 0) fail(SEM_EINVAL, "sem_set_axgs_config: negative count");
        if (epw * m->h.P * m->h.P > 512) fail(SEM_EINVAL, "sem_set_axgs_config: epw (N+1)^2 > 512");
        const int64_t n_lines = (int64_t)m->h.nel[1] * m->h.nel[2];
        if (lines_per_wg > 0 && (n_lines + lines_per_wg - 1) / lines_per_wg > m->n_partials - 64)
            fail(SEM_EINVAL, "sem_set_axgs_config: more workgroups than dot partials");
        SEM_HIP(hipDeviceSynchronize());  // launches in flight may still read the residual plans
        drop_graphs(m, nullptr);
        axgs_reset(m);
        m->axgs->enabled = enable;
        m->axgs->req_epw = epw;
        m->axgs->req_lines = lines_per_wg;
        axgs_build(m);
        return SEM_OK;
    });
}

sem_status sem_host_axgs_residual(const sem_mesh_desc *desc, int lines_per_wg, int y_onchip, int64_t *n_ids,
                                  int64_t *n_copies, int32_t *off, int32_t *idx)
{
    return guarded([&]() -> sem_status {
        if (!desc || !n_ids || !n_copies || lines_per_wg < 1 || (y_onchip != 0 && y_onchip != 1))
            fail(SEM_EINVAL, "sem_host_axgs_residual: bad arguments");
        HostMesh h;
        build_host_mesh(*desc, h);
        h.desc = *desc;
        std::vector<int32_t> o, x;
        axgs_residual_plan(h, lines_per_wg, y_onchip != 0, o, x);
        *n_ids = (int64_t)o.size() - 1;
        *n_copies = (int64_t)x.size();
        if (off) std::memcpy(off, o.data(), sizeof(int32_t) * o.size());
        if (idx && !x.empty()) std::memcpy(idx, x.data(), sizeof(int32_t) * x.size());
        return SEM_OK;
    });
}

sem_status sem_get_axgs_info(sem_mesh *m, int dtype, sem_axgs_info *info)
{
    return guarded([&]() -> sem_status {
        if (!m || !info || !m->axgs) fail(SEM_EINVAL, "sem_get_axgs_info: null argument");
        check_dtype(m, dtype);
        std::memset(info, 0, sizeof(*info));
        AxgsShape *sh = dtype == SEM_FP64 ? axgs_shape<double>(m) : axgs_shape<float>(m);
        if (!sh) return SEM_OK;
        info->enabled = 1;
        info->epw = sh->epw;
        info->lines_per_wg = sh->lines_per_wg;
        info->y_onchip = sh->y_onchip;
        info->grid = sh->grid;
        info->residual_ids = sh->res.n_ids;
        info->residual_copies = sh->res_copies;
        return SEM_OK;
    });
}

sem_status sem_mass(sem_mesh *m, const double *f, double *b, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !f || !b) fail(SEM_EINVAL, "sem_mass: null argument");
        hipStream_t s = (hipStream_t)stream;
        SEM_HIP(launch_scale(m->h.nL, m->B64, f, b, s));
        enqueue_gs<double>(m, b, nullptr, s);
        return SEM_OK;
    });
}

sem_status sem_scatter(sem_mesh *m, const double *v_global, double *u_local, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !v_global || !u_local) fail(SEM_EINVAL, "sem_scatter: null argument");
        hipStream_t s = (hipStream_t)stream;
        SEM_HIP(launch_scatter(m->h.nL, m->gid, v_global, u_local, s));
        // masked ids only: every copy set to 0
        SEM_HIP(launch_gs<double>(m->gsplan, m->gs_off, m->gs_idx, u_local, true, nullptr, s));
        return SEM_OK;
    });
}

sem_status sem_set_coarse(sem_mesh *m, int steps, double fraction, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_set_coarse: null mesh");
        if (steps < 0 || steps > 1000) fail(SEM_EINVAL, "sem_set_coarse: chebyshev_steps must be 0..1000");
        if (steps > 0 && m->h.N > kMaxPrecondOrder)
            fail(SEM_EUNSUPPORTED, "sem_set_coarse: the coarse term is built for N <= 12");
        if (steps > 0 && !(fraction > 0.0 && fraction < 1.0))
            fail(SEM_EINVAL, "sem_set_coarse: fraction must be in (0, 1)");
        hipStream_t s = (hipStream_t)stream;
        drop_graphs(m, s);
        SEM_HIP(hipStreamSynchronize(s));
        coarse_free(m->coarse);
        m->coarse = nullptr;
        if (steps > 0) m->coarse = coarse_build(m, steps, fraction, s);
        return SEM_OK;
    });
}

sem_status sem_set_schwarz(sem_mesh *m, int enable, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_set_schwarz: null mesh");
        if (enable && m->h.N > kMaxPrecondOrder)
            fail(SEM_EUNSUPPORTED, "sem_set_schwarz: the local solves are built for N <= 12");
        if (enable && m->h.N < 2)
            fail(SEM_EUNSUPPORTED, "sem_set_schwarz: N = 1 (the overlap spans the neighbours; singular local problems)");
        hipStream_t s = (hipStream_t)stream;
        drop_graphs(m, s);
        SEM_HIP(hipStreamSynchronize(s));
        schwarz_free(m->schwarz);
        m->schwarz = nullptr;
        if (enable) m->schwarz = schwarz_build(m, s);
        return SEM_OK;
    });
}

sem_status sem_get_schwarz_info(const sem_mesh *m, int *enabled, int64_t *n_factors)
{
    return guarded([&]() -> sem_status {
        if (!m) fail(SEM_EINVAL, "sem_get_schwarz_info: null mesh");
        if (enabled) *enabled = m->schwarz ? 1 : 0;
        if (n_factors) *n_factors = m->schwarz ? m->schwarz->n_table : 0;
        return SEM_OK;
    });
}

sem_status sem_get_coarse_info(const sem_mesh *m, sem_coarse_info *info)
{
    return guarded([&]() -> sem_status {
        if (!m || !info) fail(SEM_EINVAL, "sem_get_coarse_info: null argument");
        std::memset(info, 0, sizeof(*info));
        if (const CoarseSpace *C = m->coarse) {
            info->n_vertices = C->nvert;
            info->n_coarse = C->n_coarse;
            info->nnz = C->nnz;
            info->chebyshev_steps = C->k;
            info->a = C->a;
            info->b = C->b;
        }
        return SEM_OK;
    });
}

sem_status sem_precond_apply(sem_mesh *m, const double *r, double *z, void *stream)
{
    return guarded([&]() -> sem_status {
        if (!m || !r || !z) fail(SEM_EINVAL, "sem_precond_apply: null argument");
        if (r == z) fail(SEM_EINVAL, "sem_precond_apply: r and z must be distinct");
        hipStream_t s = (hipStream_t)stream;
        if (m->schwarz) schwarz_apply(m, r, z, nullptr, nullptr, s);
        else launch_jacobi(m->h.nL, m->inv64, r, z, s);
        if (m->coarse) {
            coarse_restrict<double>(m, r, m->inv64, s);
            coarse_solve(m, nullptr, nullptr, s);
            coarse_prolong_add(m, z, s);
        }
        return SEM_OK;
    });
}

void sem_solve_opts_default(sem_solve_opts *o)
{
    if (!o) return;
    o->tol = 1e-10;
    o->max_iter = 5000;
    o->precision = SEM_PREC_FP64;
    o->inner_tol = 1e-4;
    o->inner_max_iter = 0;
    o->poll_every = 16;
    o->use_graph = 1;
    o->fixed_iters = 0;
    o->x0_given = 0;
    o->profile = 0;
}

sem_status sem_pcg_solve(sem_mesh *m, const double *b, double *x, const sem_solve_opts *opts, sem_solve_stats *stats,
                         void *stream)
{
    sem_solve_stats local{};
    sem_solve_stats &out = stats ? *stats : local;
    std::memset(&out, 0, sizeof(out));
    const auto t0 = std::chrono::steady_clock::now();
    const sem_status st = guarded([&]() -> sem_status {
        if (!m || !b || !x) fail(SEM_EINVAL, "sem_pcg_solve: null argument");
        sem_solve_opts o;
        sem_solve_opts_default(&o);
        if (opts) o = *opts;
        if (!(o.tol > 0.0) && o.fixed_iters <= 0) fail(SEM_EINVAL, "sem_pcg_solve: tol must be positive");
        if (o.max_iter < 0) fail(SEM_EINVAL, "sem_pcg_solve: negative max_iter");
        hipStream_t s = (hipStream_t)stream;
        if (o.precision == SEM_PREC_MIXED) return solve_mixed(m, b, x, o, out, s);
        if (o.precision != SEM_PREC_FP64) fail(SEM_EINVAL, "sem_pcg_solve: unknown precision");
        return solve_fp64(m, b, x, o, out, s);
    });
    out.status = st;
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

}  // extern "C"
