// batch.hip -- persistent batched kernels: every CG phase of many solves of
// different orders and sizes in one launch (the paper's remedy for small
// kernels called in loops is to move the loop inside the kernel, section 3).
// Each workgroup walks the group's work table; the slot descriptor and the
// item are uniform per workgroup and come through scalar loads.
#include "batch.hpp"
#include "operator.hpp"

namespace sem {

// read-only views through the constant address space (scalar loads for
// uniform addresses); the host compilation pass only needs the types
#if defined(__HIP_DEVICE_COMPILE__)
template <typename X>
using cptr = const __attribute__((address_space(4))) X *;
#else
template <typename X>
using cptr = const X *;
#endif

// orders compiled into the batched operator
#define SEM_BATCH_ORDERS(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

bool batch_order_supported(int N)
{
    switch (N) {
#define SEM_BO(n) case n:
        SEM_BATCH_ORDERS(SEM_BO)
#undef SEM_BO
        return true;
    default:
        return false;
    }
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T>
__device__ inline int prec_of() { return sizeof(T) == 8 ? 0 : 1; }
template <typename T>
static inline int prec_of_host() { return sizeof(T) == 8 ? 0 : 1; }

// Operator of one order N over that order's items of the group.  MODE 0:
// w[0] = A x64 (FP64).  MODE 2: CG operator with the p update and per-item
// p.Ap partials.  A workgroup is epw elements x (N+1)^2 lanes, as in the
// single-mesh kernel; the derivative rows are loaded once per workgroup.
template <typename T, int N, int MODE>
__global__ __launch_bounds__(512) void batch_ax_kernel(const SlotDesc *slots_, GroupDev g, int epw)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.ax_items;
    const int64_t first = ((cptr<int64_t>)g.counts)[kCountAxRange + 2 * N];
    const int64_t n = ((cptr<int64_t>)g.counts)[kCountAxRange + 2 * N + 1];
    const int prec = prec_of<T>();
    const int tid = threadIdx.x;
    const int el = tid / P2;
    const int ij = tid - el * P2;
    const int i = ij % P, j = ij / P;
    const bool inblk = el < epw;
    constexpr bool kPlanes = plane_tile<T, N, MODE>();  // the single-mesh operator's tile
    T *su = sm + (size_t)(inblk ? el : epw - 1) * 3 * (kPlanes ? P2 : P3);
    const T *__restrict__ D = dtable<T>(N);
    __shared__ T sDt[lane_rows_lds<T, N>()];
    LaneRows<T, N> R;
    R.load(D, i, j, sDt);
    for (int64_t it = first + blockIdx.x; it < first + n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        const int64_t e = (int64_t)item.local * epw + el;
        const bool active = inblk && e < sd.E;
        double dot = 0.0;
        if (MODE == 0) {
            if constexpr (kPlanes)
                ax_tile_planes<T, N, 0>(R, D, su, e, active, inblk, i, j, static_cast<const T *>(sd.G[0]),
                                        reinterpret_cast<const T *>(sd.x64), static_cast<T *>(sd.w[0]), nullptr,
                                        nullptr, T(0), nullptr, T(0), dot);
            else
                ax_tile<T, N, 0>(R, D, su, e, active, inblk, i, j, static_cast<const T *>(sd.G[0]),
                                 reinterpret_cast<const T *>(sd.x64), static_cast<T *>(sd.w[0]), nullptr, nullptr,
                                 T(0), nullptr, T(0), dot);
        } else {
            if (uniform_int(sd.st[prec].done) == 0) {
                const T beta = (T)sd.st[prec].beta, alpha = (T)sd.st[prec].alpha;
                const T *zc = sd.zc_prec == prec ? static_cast<const T *>(sd.zc) : nullptr;
                if constexpr (kPlanes)
                    ax_tile_planes<T, N, 2>(R, D, su, e, active, inblk, i, j, static_cast<const T *>(sd.G[prec]),
                                            static_cast<const T *>(sd.r[prec]), static_cast<T *>(sd.w[prec]),
                                            static_cast<const T *>(sd.inv[prec]), static_cast<T *>(sd.p[prec]),
                                            beta, static_cast<T *>(sd.x[prec]), alpha, dot, nullptr, nullptr,
                                            NoSink(), zc);
                else
                    ax_tile<T, N, 2>(R, D, su, e, active, inblk, i, j, static_cast<const T *>(sd.G[prec]),
                                     static_cast<const T *>(sd.r[prec]), static_cast<T *>(sd.w[prec]),
                                     static_cast<const T *>(sd.inv[prec]), static_cast<T *>(sd.p[prec]), beta,
                                     static_cast<T *>(sd.x[prec]), alpha, dot, nullptr, nullptr, nullptr, nullptr,
                                     NoSink(), zc);
            }
            double v[1] = {dot};
            block_reduce_store<1>(v, g.ax_partial + it, 0);
            __syncthreads();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBatchBlock) void batch_gs_kernel(const SlotDesc *slots_, GroupDev g, int check_done,
                                                               int which)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.gs_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[2];
    const int prec = prec_of<T>();
    // the workgroups of one XCD (blockIdx mod 8) walk one contiguous eighth of
    // the items, so the lines that neighbouring chunks share stay in its L2
    // (with fewer than 8 workgroups, each walks its own contiguous range)
    const int64_t nb = gridDim.x, groups = nb < 8 ? nb : 8;
    const int64_t grp = blockIdx.x % groups, kb = blockIdx.x / groups;
    const int64_t per_g = nb / groups + (grp < nb % groups ? 1 : 0);  // workgroups of this group, >= 1
    const int64_t lo = n * grp / groups, hi = n * (grp + 1) / groups;
    for (int64_t it = lo + kb; it < hi; it += per_g) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        if (check_done && uniform_int(sd.st[prec].done)) continue;
        T *v = static_cast<T *>(which == 0 ? sd.w[prec] : sd.w[0]);
        const int64_t t = (int64_t)item.local * kGsChunk + threadIdx.x;
        if (sd.gs_lattice) {
            if (t < sd.gsl.n_nodes) gs_lattice_node<T>(sd.gsl, t, v);
            continue;
        }
        if (t >= sd.gs_n_ids) continue;
        gs_id<T>(t, sd.gs_n_sum, sd.gs_off, sd.gs_idx, v);
    }
}

__device__ inline double inv_mult_b(uint8_t m) { return 1.0 / (double)m; }

// CG update after the gather-scatter: r -= alpha w; per-item partials of
// <r,r>, <r, invdiag r>.  The x step is applied by the next operator launch.
template <typename T>
__global__ __launch_bounds__(kBatchBlock) void batch_update_kernel(const SlotDesc *slots_, GroupDev g)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    const int prec = prec_of<T>();
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        double rr = 0.0, rz = 0.0;
        if (!uniform_int(sd.st[prec].done)) {
            constexpr int U = kVecChunk / kBatchBlock;
            const T alpha = (T)sd.st[prec].alpha;
            T *r = static_cast<T *>(sd.r[prec]);
            const T *w = static_cast<const T *>(sd.w[prec]);
            const T *iv = static_cast<const T *>(sd.inv[prec]);
            const int64_t q0 = (int64_t)item.local * kVecChunk;
            const int64_t qlast = min(q0 + kVecChunk, sd.nL) - 1;
            // all loads of the chunk in flight at once (past the end: re-read the last entry)
            T rv[U], wv[U], ivv[U];
            uint8_t mv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = min(q0 + u * kBatchBlock + threadIdx.x, qlast);
                rv[u] = ld_stream(r + q);
                wv[u] = ld_stream(w + q);
                ivv[u] = ld_stream(iv + q);
                mv[u] = ld_stream(sd.mult + q);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
                if (q > qlast) break;
                const T rq = rv[u] - alpha * wv[u];
                st_stream(rq, r + q);
                const double rd = (double)rq, im = inv_mult_b(mv[u]);
                rr += rd * rd * im;
                rz += rd * (double)(ivv[u] * rq) * im;
            }
        }
        double v[2] = {rr, rz};
        block_reduce_store<2>(v, g.vec_partial + 2 * it, 0);
        __syncthreads();
    }
}

// CG start from r: p = 0, partials of <r,r>, <r, invdiag r>
template <typename T>
__global__ __launch_bounds__(kBatchBlock) void batch_init_kernel(const SlotDesc *slots_, GroupDev g)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    const int prec = prec_of<T>();
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        const T *r = static_cast<const T *>(sd.r[prec]);
        T *p = static_cast<T *>(sd.p[prec]);
        const T *iv = static_cast<const T *>(sd.inv[prec]);
        double rr = 0.0, rz = 0.0;
        const int64_t q0 = (int64_t)item.local * kVecChunk;
        for (int u = 0; u < kVecChunk / kBatchBlock; ++u) {
            const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
            if (q >= sd.nL) break;
            p[q] = T(0);
            const double rd = (double)r[q], im = inv_mult_b(sd.mult[q]);
            rr += rd * rd * im;
            rz += rd * (double)(iv[q] * r[q]) * im;
        }
        double v[2] = {rr, rz};
        block_reduce_store<2>(v, g.vec_partial + 2 * it, 0);
        __syncthreads();
    }
}

// FP64 residual: r = b - w (copy_b: r = b, x = 0); partials of <r,r> (slot 0)
__global__ __launch_bounds__(kBatchBlock) void batch_residual_kernel(const SlotDesc *slots_, GroupDev g, int copy_b)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        double *r = static_cast<double *>(sd.r[0]);
        const double *w = static_cast<const double *>(sd.w[0]);
        double rr = 0.0, bb = 0.0;
        const int64_t q0 = (int64_t)item.local * kVecChunk;
        for (int u = 0; u < kVecChunk / kBatchBlock; ++u) {
            const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
            if (q >= sd.nL) break;
            const double bq = sd.b[q];
            double rq;
            if (copy_b) {
                rq = bq;
                sd.x64[q] = 0.0;
            } else {
                rq = bq - w[q];
            }
            r[q] = rq;
            const double im = inv_mult_b(sd.mult[q]);
            rr += rq * rq * im;
            bb += bq * bq * im;
        }
        double v[2] = {rr, bb};
        block_reduce_store<2>(v, g.vec_partial + 2 * it, 0);
        __syncthreads();
    }
}

// mixed: r32 = r64 / ||r||, x32 = 0
__global__ __launch_bounds__(kBatchBlock) void batch_to_fp32_kernel(const SlotDesc *slots_, GroupDev g)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        const double s = 1.0 / sqrt(sd.scal[1]);
        const double *r = static_cast<const double *>(sd.r[0]);
        float *r32 = static_cast<float *>(sd.r[1]);
        float *x32 = static_cast<float *>(sd.x[1]);
        const int64_t q0 = (int64_t)item.local * kVecChunk;
        for (int u = 0; u < kVecChunk / kBatchBlock; ++u) {
            const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
            if (q >= sd.nL) break;
            r32[q] = (float)(r[q] * s);
            x32[q] = 0.0f;
        }
    }
}

// end of a slot's CG run: the last deferred x step (none after a breakdown)
template <typename T>
__global__ __launch_bounds__(kBatchBlock) void batch_finish_kernel(const SlotDesc *slots_, GroupDev g)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    const int prec = prec_of<T>();
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        const PcgState *st = sd.st + prec;
        if (uniform_int(st->done) == 2 || uniform_int(st->iters) == 0) continue;
        const T alpha = (T)st->alpha;
        T *x = static_cast<T *>(sd.x[prec]);
        const T *p = static_cast<const T *>(sd.p[prec]);
        const int64_t q0 = (int64_t)item.local * kVecChunk;
        for (int u = 0; u < kVecChunk / kBatchBlock; ++u) {
            const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
            if (q >= sd.nL) break;
            x[q] = x[q] + alpha * p[q];
        }
    }
}

// mixed: x64 += ||r|| x32
__global__ __launch_bounds__(kBatchBlock) void batch_axpy_kernel(const SlotDesc *slots_, GroupDev g)
{
    cptr<SlotDesc> slots = (cptr<SlotDesc>)slots_;
    cptr<Item> items = (cptr<Item>)g.vec_items;
    const int64_t n = ((cptr<int64_t>)g.counts)[3];
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item item = items[it];
        const SlotDesc sd = slots[item.slot];
        const double s = sqrt(sd.scal[1]);
        const float *x32 = static_cast<const float *>(sd.x[1]);
        const int64_t q0 = (int64_t)item.local * kVecChunk;
        for (int u = 0; u < kVecChunk / kBatchBlock; ++u) {
            const int64_t q = q0 + u * kBatchBlock + threadIdx.x;
            if (q >= sd.nL) break;
            sd.x64[q] += s * (double)x32[q];
        }
    }
}

// ---------------------------------------------------------------------------
// per-slot reductions: workgroup b takes the group's b-th slot and sums that
// slot's item partials in item order (fixed order, independent of the rest)
template <int NV>
__device__ inline void slot_sum(const double *__restrict__ part, int64_t first, int64_t count, double (&out)[NV])
{
    __shared__ double red[NV][kBatchBlock];
    double s[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = 0.0;
    for (int64_t b = threadIdx.x; b < count; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) s[q] += part[(first + b) * NV + q];
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = red[q][0];
}

__device__ inline int group_slot(const GroupDev &g)
{
    const int64_t ns = g.counts[0];
    if ((int64_t)blockIdx.x >= ns) return -1;
    return g.slots[blockIdx.x];
}

__global__ __launch_bounds__(kBatchBlock) void batch_reduce_sigma_kernel(SlotDesc *slots, GroupDev g, int prec)
{
    const int sl = group_slot(g);
    if (sl < 0) return;
    PcgState *st = slots[sl].st + prec;
    if (st->done) return;
    double s[1];
    slot_sum<1>(g.ax_partial, g.ax_first[sl], g.ax_count[sl], s);
    if (threadIdx.x == 0) {
        st->sigma = s[0];
        if (!(s[0] > 0.0) || !isfinite(s[0])) st->done = 2;
        else st->alpha = st->rho / s[0];
    }
}

__global__ __launch_bounds__(kBatchBlock) void batch_reduce_rho_kernel(SlotDesc *slots, GroupDev g, int prec)
{
    const int sl = group_slot(g);
    if (sl < 0) return;
    PcgState *st = slots[sl].st + prec;
    if (st->done) return;
    double s[2];
    slot_sum<2>(g.vec_partial, g.vec_first[sl], g.vec_count[sl], s);
    if (slots[sl].crz && slots[sl].zc_prec == prec) s[1] += *slots[sl].crz;  // <r, P z0> = r0.z0
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = s[0];
        st->rho_new = s[1];
        st->beta = s[1] / st->rho;
        st->rho = s[1];
        if (s[0] <= st->stop2) st->done = 1;
        else if (!isfinite(s[0])) st->done = 2;
        else if (st->iters >= st->limit) st->done = 3;
    }
}

__global__ __launch_bounds__(kBatchBlock) void batch_reduce_init_kernel(SlotDesc *slots, GroupDev g, int prec)
{
    const int sl = group_slot(g);
    if (sl < 0) return;
    const SlotDesc &sd = slots[sl];
    PcgState *st = sd.st + prec;
    double s[2];
    slot_sum<2>(g.vec_partial, g.vec_first[sl], g.vec_count[sl], s);
    if (sd.crz && sd.zc_prec == prec) s[1] += *sd.crz;
    if (threadIdx.x == 0) {
        st->rr = s[0];
        st->rho = s[1];
        st->rho_new = s[1];
        st->beta = 0.0;
        st->alpha = 0.0;
        st->sigma = 0.0;
        st->iters = 0;
        st->limit = sd.limit[prec];
        st->stop2 = sd.stop2[prec];
        st->done = (s[0] <= st->stop2) ? 1 : (st->limit <= 0 ? 3 : 0);
    }
}

// scal[1] = <r,r>, scal[0] = <b,b> after batch_residual
__global__ __launch_bounds__(kBatchBlock) void batch_reduce_residual_kernel(SlotDesc *slots, GroupDev g)
{
    const int sl = group_slot(g);
    if (sl < 0) return;
    double s[2];
    slot_sum<2>(g.vec_partial, g.vec_first[sl], g.vec_count[sl], s);
    if (threadIdx.x == 0) {
        slots[sl].scal[1] = s[0];
        slots[sl].scal[0] = s[1];
    }
}

// ---------------------------------------------------------------------------
size_t batch_ax_lds(int N, int epw, int prec, int mode)
{
    const size_t P2 = (size_t)(N + 1) * (N + 1), P3 = P2 * (N + 1);
    const int bytes = prec == 0 ? 8 : 4;
    return (size_t)epw * 3 * (plane_tile_use(N, mode, bytes) ? P2 : P3) * bytes;
}

template <typename T, int MODE>
static hipError_t batch_ax_order(int N, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    const int epw = L.epw[N];
    const int threads = ax_block_threads(N, epw);
    if (epw < 1 || threads > 512) return hipErrorInvalidConfiguration;
    const size_t lds = batch_ax_lds(N, epw, prec_of_host<T>(), MODE);
    switch (N) {
#define SEM_BCASE(n) \
    case n: hipLaunchKernelGGL((batch_ax_kernel<T, n, MODE>), dim3(L.ax_grid), dim3(threads), lds, s, slots, g, epw); break;
        SEM_BATCH_ORDERS(SEM_BCASE)
#undef SEM_BCASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t batch_ax(int prec, int mode, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    for (int N = 1; N <= SEM_MAX_ORDER; ++N) {
        if (!(L.orders & (1u << N))) continue;
        hipError_t e;
        if (mode == 0) e = batch_ax_order<double, 0>(N, slots, g, L, s);
        else if (prec == 0) e = batch_ax_order<double, 2>(N, slots, g, L, s);
        else e = batch_ax_order<float, 2>(N, slots, g, L, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t batch_gs(int prec, int check_done, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L,
                    hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((batch_gs_kernel<double>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g, check_done, 0);
    else
        hipLaunchKernelGGL((batch_gs_kernel<float>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g, check_done, 0);
    return hipGetLastError();
}

hipError_t batch_reduce_sigma(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reduce_sigma_kernel, dim3(L.max_slots), dim3(kBatchBlock), 0, s,
                       const_cast<SlotDesc *>(slots), g, prec);
    return hipGetLastError();
}

hipError_t batch_update(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((batch_update_kernel<double>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    else
        hipLaunchKernelGGL((batch_update_kernel<float>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    return hipGetLastError();
}

hipError_t batch_reduce_rho(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reduce_rho_kernel, dim3(L.max_slots), dim3(kBatchBlock), 0, s,
                       const_cast<SlotDesc *>(slots), g, prec);
    return hipGetLastError();
}

hipError_t batch_cg_init(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((batch_init_kernel<double>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    else
        hipLaunchKernelGGL((batch_init_kernel<float>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    hipLaunchKernelGGL(batch_reduce_init_kernel, dim3(L.max_slots), dim3(kBatchBlock), 0, s,
                       const_cast<SlotDesc *>(slots), g, prec);
    return hipGetLastError();
}

hipError_t batch_residual(int copy_b, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(batch_residual_kernel, dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g, copy_b);
    hipLaunchKernelGGL(batch_reduce_residual_kernel, dim3(L.max_slots), dim3(kBatchBlock), 0, s,
                       const_cast<SlotDesc *>(slots), g);
    return hipGetLastError();
}

hipError_t batch_to_fp32(const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(batch_to_fp32_kernel, dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    return hipGetLastError();
}

hipError_t batch_finish(int prec, const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((batch_finish_kernel<double>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    else
        hipLaunchKernelGGL((batch_finish_kernel<float>), dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    return hipGetLastError();
}

hipError_t batch_axpy(const SlotDesc *slots, const GroupDev &g, const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(batch_axpy_kernel, dim3(L.vec_grid), dim3(kBatchBlock), 0, s, slots, g);
    return hipGetLastError();
}

hipError_t upload_batch_dtables(const double *d64, const float *d32, hipStream_t s)
{
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D64), d64, sizeof(double) * kDTableSize, 0,
                                          hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D32), d32, sizeof(float) * kDTableSize, 0, hipMemcpyHostToDevice, s);
}

}  // namespace sem
