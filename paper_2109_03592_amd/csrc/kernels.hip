// kernels.hip -- gfx950 kernels of the SEM hot path.
//
//  * ax_kernel: the local operator of Algorithm 1 (axhelm).  One lane per
//    (i,j) column of an element holds the column u(i,j,0..N) in registers, so
//    the t-derivative never touches LDS; r- and s-derivatives read the element
//    staged in LDS.  The derivative matrix rows a lane needs live in VGPRs,
//    the uniform D[k][l] of the t-direction comes through scalar loads.  The
//    six geometric factors stream from HBM, one coalesced plane per k.  An
//    epilogue reduces u.w per workgroup for CG (p.Ap is taken before the
//    gather-scatter, which is exact for continuous p).
//  * gs_kernel: direct-stiffness summation from a plan sorted by global id:
//    one lane per global id, copies summed in ascending local index and
//    written back; masked ids get 0.  No atomics.
//  * PCG update / reductions: fused x, r update with the Jacobi-weighted
//    <r,z> and <r,r>, per-workgroup partials reduced in a fixed order by a
//    single-workgroup kernel that also forms alpha and beta on the device.
#include "kernels.hpp"

namespace sem {

// ---------------------------------------------------------------------------
// block reductions (fixed order => deterministic)
template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double *dst, int stride)
{
    __shared__ double red[NV][32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < nwave; ++w) s += red[q][w];
            dst[(size_t)blockIdx.x * stride + q] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Local operator (Algorithm 1, h1 = 1).  MODE 0: w = A_L u.  MODE 1: also
// per-workgroup partial of u.w.  MODE 2 (CG): p <- invdiag*r + beta*p first,
// then w = A_L p and the partial of p.w.
template <typename T, int N, int MODE>
__global__ __launch_bounds__(256) void ax_kernel(AxParams<T> a)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);

    if (MODE == 2 && a.st->done) return;

    const int tid = threadIdx.x;
    const int el = tid / P2;
    const int ij = tid - el * P2;
    const int i = ij % P, j = ij / P;
    const bool inblk = el < a.epw;
    const int slot = inblk ? el : a.epw - 1;  // padding lanes read a valid slot
    const int64_t e = (int64_t)blockIdx.x * a.epw + el;
    const bool active = inblk && e < a.E;
    T *su = sm + (size_t)slot * 3 * P3;
    T *sr = su + P3;
    T *ss = sr + P3;
    const T *__restrict__ D = a.D;

    T Di[P], Dj[P], Dti[P], Dtj[P];
#pragma unroll
    for (int l = 0; l < P; ++l) {
        Di[l] = D[i * P + l];
        Dj[l] = D[j * P + l];
        Dti[l] = D[l * P + i];
        Dtj[l] = D[l * P + j];
    }

    const int64_t base = (active ? e : 0) * P3 + ij;
    T uc[P];
    if (MODE == 2) {
        const T beta = (T)a.st->beta;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T v = 0;
            if (active) {
                const int64_t o = base + k * P2;
                v = a.invdiag[o] * a.in[o] + beta * a.p[o];
                a.p[o] = v;
            }
            uc[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) uc[k] = active ? a.in[base + k * P2] : T(0);
    }
    if (inblk) {
#pragma unroll
        for (int k = 0; k < P; ++k) su[k * P2 + ij] = uc[k];
    }
    __syncthreads();

    const T *__restrict__ Ge = a.G + (active ? e : 0) * 6 * P3 + ij;
    T wt[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        T ur = 0, us = 0, ut = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            ur += Di[l] * su[k * P2 + j * P + l];
            us += Dj[l] * su[k * P2 + l * P + i];
            ut += D[k * P + l] * uc[l];
        }
        T g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0, g6 = 0;
        if (active) {
            const T *g = Ge + k * P2;
            g1 = g[0 * P3]; g2 = g[1 * P3]; g3 = g[2 * P3];
            g4 = g[3 * P3]; g5 = g[4 * P3]; g6 = g[5 * P3];
        }
        const T wr = g1 * ur + g4 * us + g5 * ut;
        const T ws = g2 * us + g4 * ur + g6 * ut;
        wt[k] = g3 * ut + g5 * ur + g6 * us;
        if (inblk) {
            sr[k * P2 + ij] = wr;
            ss[k * P2 + ij] = ws;
        }
    }
    __syncthreads();

    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        T acc = 0;
#pragma unroll
        for (int l = 0; l < P; ++l)
            acc += Dti[l] * sr[k * P2 + j * P + l] + Dtj[l] * ss[k * P2 + l * P + i] + D[l * P + k] * wt[l];
        if (active) a.out[base + k * P2] = acc;
        if (MODE != 0) dot += (double)uc[k] * (double)acc;
    }
    if (MODE != 0) {
        double v[1] = {dot};
        block_reduce_store<1>(v, a.partial, 1);
    }
}

// ---------------------------------------------------------------------------
// Gather-scatter from the sorted plan.  Ids [0, n_sum): sum of copies in plan
// order written to every copy.  Ids [n_sum, n_ids): copies set to 0 (mask).
template <typename T>
__global__ __launch_bounds__(256) void gs_kernel(int64_t first, int64_t n_sum, int64_t n_ids,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ idx, T *__restrict__ v,
                                                 const PcgState *__restrict__ st)
{
    if (st && st->done) return;
    const int64_t t = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ids) return;
    const int32_t q0 = off[t], q1 = off[t + 1];
    if (t < n_sum) {
        T s = 0;
        for (int32_t q = q0; q < q1; ++q) s += v[idx[q]];
        for (int32_t q = q0; q < q1; ++q) v[idx[q]] = s;
    } else {
        for (int32_t q = q0; q < q1; ++q) v[idx[q]] = T(0);
    }
}

// ---------------------------------------------------------------------------
// elementwise helpers
__global__ void scale_kernel(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                             double *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = a[q] * b[q];
}

__global__ void scatter_kernel(int64_t n, const int32_t *__restrict__ gid, const double *__restrict__ vg,
                               double *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = vg[gid[q]];
}

__global__ void residual_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w,
                                double *__restrict__ r)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        r[q] = b[q] - w[q];
}

// r32 = FP32(r * scale)
__global__ void to_fp32_kernel(int64_t n, const double *__restrict__ r, const double *__restrict__ scal,
                               float *__restrict__ out)
{
    const double s = 1.0 / sqrt(scal[0]);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = (float)(r[q] * s);
}

// x += sqrt(scal) * FP64(d)
__global__ void axpy_fp32_kernel(int64_t n, const float *__restrict__ d, const double *__restrict__ scal,
                                 double *__restrict__ x)
{
    const double s = sqrt(scal[0]);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        x[q] += s * (double)d[q];
}

__global__ void fp64_to_fp32_kernel(int64_t n, const double *__restrict__ a, float *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = (float)a[q];
}

__device__ inline double inv_mult(uint8_t m) { return 1.0 / (double)m; }

// partial of sum a*b/mult (unique-dof inner product)
template <typename T>
__global__ __launch_bounds__(256) void dot_unique_kernel(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                                                         const uint8_t *__restrict__ mult, double *__restrict__ partial)
{
    double s = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        s += (double)a[q] * (double)b[q] * inv_mult(mult[q]);
    double v[1] = {s};
    block_reduce_store<1>(v, partial, 1);
}

// CG start: partials of <r, invdiag r> and <r, r>
template <typename T>
__global__ __launch_bounds__(256) void pcg_init_kernel(int64_t n, const T *__restrict__ r, const T *__restrict__ inv,
                                                       const uint8_t *__restrict__ mult, double *__restrict__ partial)
{
    double rr = 0.0, rz = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const double rd = (double)r[q], im = inv_mult(mult[q]);
        rr += rd * rd * im;
        rz += rd * (double)(inv[q] * r[q]) * im;
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// x += alpha p, r -= alpha w; partials of <r, r> and <r, invdiag r>
template <typename T>
__global__ __launch_bounds__(256) void pcg_update_kernel(int64_t n, const PcgState *__restrict__ st, T *__restrict__ x,
                                                         T *__restrict__ r, const T *__restrict__ p,
                                                         const T *__restrict__ w, const T *__restrict__ inv,
                                                         const uint8_t *__restrict__ mult, double *__restrict__ partial)
{
    if (st->done) return;
    const T alpha = (T)st->alpha;
    double rr = 0.0, rz = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        x[q] = x[q] + alpha * p[q];
        const T rq = r[q] - alpha * w[q];
        r[q] = rq;
        const double rd = (double)rq, im = inv_mult(mult[q]);
        rr += rd * rd * im;
        rz += rd * (double)(inv[q] * rq) * im;
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// ---------------------------------------------------------------------------
// single-workgroup reductions of partials (fixed order)
template <int NV>
__device__ inline void sum_partials(const double *__restrict__ partial, int64_t n, double (&out)[NV])
{
    __shared__ double red[NV][1024];
    double s[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) s[q] += partial[b * NV + q];
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

__global__ __launch_bounds__(1024) void reduce_scalar_kernel(const double *__restrict__ partial, int64_t n,
                                                             double *__restrict__ out)
{
    double s[1];
    sum_partials<1>(partial, n, s);
    if (threadIdx.x == 0) out[0] = s[0];
}

// sigma = <p, A p>; alpha = rho / sigma (breakdown when sigma <= 0 or not finite)
__global__ __launch_bounds__(1024) void reduce_sigma_kernel(const double *__restrict__ partial, int64_t n,
                                                            PcgState *__restrict__ st)
{
    if (st->done) return;
    double s[1];
    sum_partials<1>(partial, n, s);
    if (threadIdx.x == 0) {
        st->sigma = s[0];
        if (!(s[0] > 0.0) || !isfinite(s[0])) st->done = 2;
        else st->alpha = st->rho / s[0];
    }
}

// rho' = <r, z>, rr = <r, r>; beta = rho'/rho; convergence / limit flags
__global__ __launch_bounds__(1024) void reduce_rho_kernel(const double *__restrict__ partial, int64_t n,
                                                          PcgState *__restrict__ st)
{
    if (st->done) return;
    double s[2];
    sum_partials<2>(partial, n, s);
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

// CG start: rho = <r, z>, rr = <r, r>, beta = 0
__global__ __launch_bounds__(1024) void reduce_init_kernel(const double *__restrict__ partial, int64_t n,
                                                           PcgState *__restrict__ st, double stop2, int limit)
{
    double s[2];
    sum_partials<2>(partial, n, s);
    if (threadIdx.x == 0) {
        st->rr = s[0];
        st->rho = s[1];
        st->rho_new = s[1];
        st->beta = 0.0;
        st->alpha = 0.0;
        st->sigma = 0.0;
        st->iters = 0;
        st->limit = limit;
        st->stop2 = stop2;
        st->done = (s[0] <= stop2) ? 1 : (limit <= 0 ? 3 : 0);
    }
}

// ---------------------------------------------------------------------------
// host launchers
static inline int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

int ax_block_threads(int N, int epw)
{
    const int P2 = (N + 1) * (N + 1);
    const int t = epw * P2;
    return (t + 63) / 64 * 64;
}

size_t ax_lds_bytes(int N, int epw, size_t elem)
{
    const size_t P3 = (size_t)(N + 1) * (N + 1) * (N + 1);
    return (size_t)epw * 3 * P3 * elem;
}

int64_t ax_blocks(int64_t E, int epw) { return (E + epw - 1) / epw; }

template <typename T, int MODE>
static hipError_t launch_ax_mode(int N, const AxParams<T> &a, hipStream_t s)
{
    const int threads = ax_block_threads(N, a.epw);
    const size_t lds = ax_lds_bytes(N, a.epw, sizeof(T));
    const int64_t blocks = ax_blocks(a.E, a.epw);
    if (threads > 256 || blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    switch (N) {
#define SEM_AX_CASE(n) \
    case n: hipLaunchKernelGGL((ax_kernel<T, n, MODE>), dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
        SEM_AX_CASE(1) SEM_AX_CASE(2) SEM_AX_CASE(3) SEM_AX_CASE(4) SEM_AX_CASE(5) SEM_AX_CASE(6)
        SEM_AX_CASE(7) SEM_AX_CASE(8) SEM_AX_CASE(9) SEM_AX_CASE(10) SEM_AX_CASE(11) SEM_AX_CASE(12)
#undef SEM_AX_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ax(int N, int mode, const AxParams<T> &a, hipStream_t s)
{
    if (mode == 0) return launch_ax_mode<T, 0>(N, a, s);
    if (mode == 1) return launch_ax_mode<T, 1>(N, a, s);
    return launch_ax_mode<T, 2>(N, a, s);
}
template hipError_t launch_ax<double>(int, int, const AxParams<double> &, hipStream_t);
template hipError_t launch_ax<float>(int, int, const AxParams<float> &, hipStream_t);

template <typename T>
hipError_t launch_gs(int64_t first, int64_t n_sum, int64_t n_ids, const int32_t *off, const int32_t *idx, T *v,
                     const PcgState *st, hipStream_t s)
{
    const int64_t n = n_ids - first;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL((gs_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, first, n_sum, n_ids, off, idx, v, st);
    return hipGetLastError();
}
template hipError_t launch_gs<double>(int64_t, int64_t, int64_t, const int32_t *, const int32_t *, double *,
                                      const PcgState *, hipStream_t);
template hipError_t launch_gs<float>(int64_t, int64_t, int64_t, const int32_t *, const int32_t *, float *,
                                     const PcgState *, hipStream_t);

int vec_blocks(int64_t n) { return grid_for(n, 256, 4096); }

hipError_t launch_scale(int64_t n, const double *a, const double *b, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(scale_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, a, b, out);
    return hipGetLastError();
}
hipError_t launch_scatter(int64_t n, const int32_t *gid, const double *vg, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(scatter_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, gid, vg, out);
    return hipGetLastError();
}
hipError_t launch_residual(int64_t n, const double *b, const double *w, double *r, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, b, w, r);
    return hipGetLastError();
}
hipError_t launch_to_fp32_scaled(int64_t n, const double *r, const double *scal, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(to_fp32_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, r, scal, out);
    return hipGetLastError();
}
hipError_t launch_axpy_fp32(int64_t n, const float *d, const double *scal, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(axpy_fp32_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, d, scal, x);
    return hipGetLastError();
}
hipError_t launch_fp64_to_fp32(int64_t n, const double *a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(fp64_to_fp32_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, a, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dot_unique(int64_t n, const T *a, const T *b, const uint8_t *mult, double *partial,
                             double *out, hipStream_t s)
{
    const int blocks = vec_blocks(n);
    hipLaunchKernelGGL((dot_unique_kernel<T>), dim3(blocks), dim3(256), 0, s, n, a, b, mult, partial);
    hipLaunchKernelGGL(reduce_scalar_kernel, dim3(1), dim3(1024), 0, s, partial, (int64_t)blocks, out);
    return hipGetLastError();
}
template hipError_t launch_dot_unique<double>(int64_t, const double *, const double *, const uint8_t *, double *,
                                              double *, hipStream_t);
template hipError_t launch_dot_unique<float>(int64_t, const float *, const float *, const uint8_t *, double *,
                                             double *, hipStream_t);

template <typename T>
hipError_t launch_pcg_init(int64_t n, const T *r, const T *inv, const uint8_t *mult, double *partial,
                           PcgState *st, double stop2, int limit, hipStream_t s)
{
    const int blocks = vec_blocks(n);
    hipLaunchKernelGGL((pcg_init_kernel<T>), dim3(blocks), dim3(256), 0, s, n, r, inv, mult, partial);
    hipLaunchKernelGGL(reduce_init_kernel, dim3(1), dim3(1024), 0, s, partial, (int64_t)blocks, st, stop2, limit);
    return hipGetLastError();
}
template hipError_t launch_pcg_init<double>(int64_t, const double *, const double *, const uint8_t *, double *,
                                            PcgState *, double, int, hipStream_t);
template hipError_t launch_pcg_init<float>(int64_t, const float *, const float *, const uint8_t *, double *,
                                           PcgState *, double, int, hipStream_t);

template <typename T>
hipError_t launch_pcg_update(int64_t n, const PcgState *st, T *x, T *r, const T *p, const T *w, const T *inv,
                             const uint8_t *mult, double *partial, hipStream_t s)
{
    const int blocks = vec_blocks(n);
    hipLaunchKernelGGL((pcg_update_kernel<T>), dim3(blocks), dim3(256), 0, s, n, st, x, r, p, w, inv, mult, partial);
    return hipGetLastError();
}
template hipError_t launch_pcg_update<double>(int64_t, const PcgState *, double *, double *, const double *,
                                              const double *, const double *, const uint8_t *, double *, hipStream_t);
template hipError_t launch_pcg_update<float>(int64_t, const PcgState *, float *, float *, const float *,
                                             const float *, const float *, const uint8_t *, double *, hipStream_t);

hipError_t launch_reduce_sigma(const double *partial, int64_t n, PcgState *st, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_sigma_kernel, dim3(1), dim3(1024), 0, s, partial, n, st);
    return hipGetLastError();
}
hipError_t launch_reduce_rho(const double *partial, int64_t n, PcgState *st, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_rho_kernel, dim3(1), dim3(1024), 0, s, partial, n, st);
    return hipGetLastError();
}
hipError_t launch_reduce_scalar(const double *partial, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_scalar_kernel, dim3(1), dim3(1024), 0, s, partial, n, out);
    return hipGetLastError();
}

}  // namespace sem
