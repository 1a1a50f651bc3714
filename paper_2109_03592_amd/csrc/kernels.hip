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
//  * gs_lattice_kernel: the same summation with no plan read: a node's
//    copies follow from its position on the element lattice (GsLattice).
//  * PCG update / reductions: fused x, r update with the Jacobi-weighted
//    <r,z> and <r,r>, per-workgroup partials reduced in a fixed order by a
//    single-workgroup kernel that also forms alpha and beta on the device.
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.hpp"
#include "operator.hpp"

namespace sem {

// Single mesh, persistent: each workgroup walks element tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... and stores its dot partial (modes 1, 2).
template <typename T, int N, int MODE, bool HELM>
__global__ __launch_bounds__(512) void ax_kernel(AxParams<T> a)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);

    if (MODE >= 2 && a.st->done) return;

    const int tid = threadIdx.x;
    const int el = tid / P2;
    const int ij = tid - el * P2;
    const int i = ij % P, j = ij / P;
    const bool inblk = el < a.epw;
    const int slot = inblk ? el : a.epw - 1;  // padding lanes read a valid slot
    constexpr bool kPlanes = plane_tile<T, N, MODE>();
    T *su = sm + (size_t)slot * 3 * (kPlanes ? P2 : P3);
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
    const int64_t ntiles = (a.E + a.epw - 1) / a.epw;
    // coarse modes: the tile's corner values of z0 come from LDS, staged one
    // tile ahead (their vertex indices two tiles ahead), so the dependent
    // evert -> z0 loads never sit on a tile's critical path
    constexpr bool kCoarse = MODE == 3 || MODE == 5;
    constexpr int kZB = kCoarse ? (512 / P2) * 8 : 1;  // corner values of one tile
    constexpr int kPer = (8 + P2 - 1) / P2;            // staged values per lane
    __shared__ double szb[2 * kZB];
    int32_t evn[kPer];
    double zp[kPer];
    int cur = 0;
    const int nz = a.epw * 8;
    auto vert_of = [&](int64_t t, int q) -> int32_t {
        const int64_t e2 = t * a.epw + q / 8;
        return (q < nz && t < ntiles && e2 < a.E) ? a.evert[e2 * 8 + (q & 7)] : -1;
    };
    if constexpr (kCoarse) {
        const int64_t t0 = blockIdx.x;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = tid + u * (int)blockDim.x;
            const int32_t v0 = vert_of(t0, q);
            if (q < nz) szb[q] = v0 >= 0 ? a.z0[v0] : 0.0;
            evn[u] = vert_of(t0 + gridDim.x, q);
        }
        __syncthreads();
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t e = tile * a.epw + el;
        const bool active = inblk && e < a.E;
        if constexpr (kCoarse) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int q = tid + u * (int)blockDim.x;
                zp[u] = evn[u] >= 0 ? a.z0[evn[u]] : 0.0;          // next tile
                evn[u] = vert_of(tile + 2 * (int64_t)gridDim.x, q);  // the tile after
            }
        }
        if constexpr (kPlanes)
            ax_tile_planes<T, N, MODE, HELM>(R, D, su, e, active, inblk, i, j, a.G, a.in, a.out, a.invdiag, a.p,
                                             beta, a.x, alpha, dot, a.h1, a.h2b);
        else
            ax_tile<T, N, MODE, HELM>(R, D, su, e, active, inblk, i, j, a.G, a.in, a.out, a.invdiag, a.p, beta,
                                         a.x, alpha, dot, a.h1, a.h2b,
                                         kCoarse ? szb + cur * kZB + slot * 8 : nullptr, a.cq);
        if constexpr (kCoarse) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int q = tid + u * (int)blockDim.x;
                if (q < nz) szb[(cur ^ 1) * kZB + q] = zp[u];
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    if (MODE != 0) {
        double v[1] = {dot};
        block_reduce_store<1>(v, a.partial, 1);
    }
}

// ---------------------------------------------------------------------------
// Gather-scatter from the plan sorted by global id (lattice order, so that
// neighbouring lanes touch neighbouring rows of neighbouring elements).  One
// lane per global id: ids [0, n_sum) sum their copies (ascending local index,
// from 0) and write the sum to every copy; ids [n_sum, n_ids) are Dirichlet
// ids whose copies are set to 0.
template <typename T>
__global__ __launch_bounds__(256) void gs_kernel(GsPlan plan, int64_t first, const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ idx, T *__restrict__ v,
                                                 const PcgState *__restrict__ st)
{
    if (st && st->done) return;
    // workgroups go to the 8 XCDs round-robin; remap so that each XCD walks
    // one contiguous range of ids and its L2 sees neighbouring rows together
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned per = nb / 8, rem = nb % 8, xcd = b % 8, k = b / 8;
    const unsigned lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k;
    const int64_t t = first + (int64_t)lb * blockDim.x + threadIdx.x;
    if (t >= plan.n_ids) return;
    gs_id<T>(t, plan.n_sum, off, idx, v);
}

template <typename T>
__global__ __launch_bounds__(256) void gs_lattice_kernel(GsLattice L, T *__restrict__ v,
                                                         const PcgState *__restrict__ st)
{
    if (st && st->done) return;
    // the XCD-aware remap of gs_kernel: each XCD walks one contiguous range
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned per = nb / 8, rem = nb % 8, xcd = b % 8, kb = b / 8;
    const unsigned lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + kb;
    const int64_t t = (int64_t)lb * blockDim.x + threadIdx.x;
    if (t < L.n_nodes) gs_lattice_node<T>(L, t, v);
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
        if (inv) rz += rd * (double)(inv[q] * r[q]) * im;
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// CG update after the gather-scatter: r -= alpha w; partials of <r,r> and
// <r, invdiag r> (0 when inv is null: another preconditioner forms <r,z>).  (x += alpha p is applied by the next operator launch, or
// by pcg_finish_kernel at the end of the run.)  Two consecutive entries per
// lane and step over a wide grid (more waves in flight beat more steps in
// flight per lane here).
template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

template <typename T>
__global__ __launch_bounds__(256) void pcg_update_kernel(int64_t n, const PcgState *__restrict__ st,
                                                         T *__restrict__ r, const T *__restrict__ w,
                                                         const T *__restrict__ inv,
                                                         const uint8_t *__restrict__ mult,
                                                         double *__restrict__ partial)
{
    using V = typename Pair<T>::type;
    constexpr int U = 1;
    if (st->done) return;
    const T alpha = (T)st->alpha;
    double rr = 0.0, rz = 0.0;
    const int64_t n2 = n >> 1;
    const int64_t S = (int64_t)gridDim.x * blockDim.x;
    V *__restrict__ r2 = reinterpret_cast<V *>(r);
    const V *__restrict__ w2 = reinterpret_cast<const V *>(w);
    const V *__restrict__ i2 = reinterpret_cast<const V *>(inv);
    const uint16_t *__restrict__ m2 = reinterpret_cast<const uint16_t *>(mult);
    for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q0 < n2; q0 += U * S) {
        V rv[U], wv[U], iv[U];
        uint16_t mm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + u * S;
            if (q < n2) {
                rv[u] = ld_stream(r2 + q); wv[u] = ld_stream(w2 + q);
                if (inv) iv[u] = ld_stream(i2 + q);
                else iv[u].x = iv[u].y = T(0);
                mm[u] = ld_stream(m2 + q);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + u * S;
            if (q >= n2) break;
            rv[u].x = rv[u].x - alpha * wv[u].x;
            rv[u].y = rv[u].y - alpha * wv[u].y;
            st_stream(rv[u], r2 + q);
            const double ima = inv_mult((uint8_t)(mm[u] & 0xff)), imb = inv_mult((uint8_t)(mm[u] >> 8));
            const double ra = (double)rv[u].x, rb = (double)rv[u].y;
            rr += ra * ra * ima + rb * rb * imb;
            rz += ra * (double)(iv[u].x * rv[u].x) * ima + rb * (double)(iv[u].y * rv[u].y) * imb;
        }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t q = n - 1;
        const T rq = r[q] - alpha * w[q];
        r[q] = rq;
        const double rd = (double)rq, im = inv_mult(mult[q]);
        rr += rd * rd * im;
        if (inv) rz += rd * (double)(inv[q] * rq) * im;
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// Elements [e0, e1) of the workgroup in the element-wise update: the
// workgroups split the elements into contiguous chunks, and the workgroups
// that run on one XCD (blockIdx mod 8) take neighbouring chunks.
__device__ inline void update_chunk(int64_t E, int64_t &e0, int64_t &e1)
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned per = nb / 8, rem = nb % 8, xcd = b % 8, kb = b / 8;
    const unsigned lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + kb;
    const int64_t chunk = (E + nb - 1) / nb;
    e0 = (int64_t)lb * chunk;
    e1 = e0 + chunk < E ? e0 + chunk : E;
}

// The same update element by element: one wavefront per element, each lane
// P^3/64 nodes at stride 64 (all their loads in flight together); the
// partial pairs per workgroup of four wavefronts.
template <typename T, int N>
__global__ __launch_bounds__(256) void pcg_update_elem_kernel(int64_t E, const PcgState *__restrict__ st,
                                                              T *__restrict__ r, const T *__restrict__ w,
                                                              const T *__restrict__ inv,
                                                              const uint8_t *__restrict__ mult,
                                                              double *__restrict__ partial)
{
    constexpr int P = N + 1, P3 = P * P * P;
    if (st->done) return;
    const T alpha = (T)st->alpha;
    const int lane = threadIdx.x & 63;
    double rr = 0.0, rz = 0.0;
    int64_t e0, e1;
    update_chunk(E, e0, e1);
    for (int64_t e = e0 + (threadIdx.x >> 6); e < e1; e += 4) {
        const int64_t base = e * P3;
#pragma unroll
        for (int q = lane; q < P3; q += 64) {
            const int64_t o = base + q;
            const T rv = ld_stream(r + o) - alpha * ld_stream(w + o);
            st_stream(rv, r + o);
            const double im = inv_mult(ld_stream(mult + o));
            const double rd = (double)rv;
            rr += rd * rd * im;
            if (inv) rz += rd * (double)(ld_stream(inv + o) * rv) * im;
        }
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// The element-wise update with the gather-scatter of w folded in (lattice
// meshes, Jacobi iteration): a node on an element face sums its copies of w
// itself -- from 0, in ascending local index, as the gather-scatter would --
// and uses the sum, so the assembled w is never written and the separate
// gather-scatter pass disappears; the result is bit-identical to gather-
// scatter then update.  Each block walks a contiguous chunk of elements
// (blocks XCD-contiguous; update_chunk), so the neighbours whose faces it
// reads are being read on the same XCD at about the same time.  A
// wavefront's element is uniform across its lanes, so each axis's copy rule
// is formed once per element and a lane only selects its side.
template <typename T, int N>
__global__ __launch_bounds__(256) void pcg_update_gs_kernel(GsLattice L, int64_t E, const PcgState *__restrict__ st,
                                                            T *__restrict__ r, const T *__restrict__ w,
                                                            const T *__restrict__ inv,
                                                            const uint8_t *__restrict__ mult,
                                                            double *__restrict__ partial)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    if (st->done) return;
    const T alpha = (T)st->alpha;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t e0, e1;
    update_chunk(E, e0, e1);  // the same elements per workgroup as pcg_update_elem_kernel: the same partials
    const int nx = L.nel[0], ny = L.nel[1];
    const int sy = nx * P3, sz = nx * ny * P3;  // E P3 < 2^31 (launch_pcg_update_gs)
    double rr = 0.0, rz = 0.0;
    for (int64_t e = e0 + wave; e < e1; e += 4) {
        const int ex = (int)(e % nx);
        const int64_t eyz = e / nx;
        const int ey = (int)(eyz % ny), ez = (int)(eyz / ny);
        const ElemAxis ax = elem_axis<N>(ex, nx, L.periodic[0], L.faces & 1, L.faces & 2);
        const ElemAxis ay = elem_axis<N>(ey, ny, L.periodic[1], L.faces & 4, L.faces & 8);
        const ElemAxis az = elem_axis<N>(ez, L.nel[2], L.periodic[2], L.faces & 16, L.faces & 32);
        const int64_t base = e * P3;
#pragma unroll
        for (int q = lane; q < P3; q += 64) {
            const int i = q % P, j = (q / P) % P, k = q / P2;
            const int64_t o = base + q;
            T ws = w[o];
            if (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N) {
                const LaneAxis cx = lane_axis<N>(ax, i, P3, 1);
                const LaneAxis cy = lane_axis<N>(ay, j, sy, P);
                const LaneAxis cz = lane_axis<N>(az, k, sz, P2);
                if (cx.masked || cy.masked || cz.masked) {
                    ws = T(0);
                } else if (cx.c * cy.c * cz.c > 1) {
                    T val[8];
#pragma unroll
                    for (int c8 = 0; c8 < 8; ++c8) {
                        const int qz = c8 >> 2, qy = (c8 >> 1) & 1, qx = c8 & 1;
                        const int64_t a = o + (cz.d[qz] + cy.d[qy] + cx.d[qx]);
                        val[c8] = (qz < cz.c && qy < cy.c && qx < cx.c) ? w[a] : T(0);
                    }
                    T sum = T(0);
#pragma unroll
                    for (int c8 = 0; c8 < 8; ++c8) {
                        const int qz = c8 >> 2, qy = (c8 >> 1) & 1, qx = c8 & 1;
                        if (qz < cz.c && qy < cy.c && qx < cx.c) sum = sum + val[c8];
                    }
                    ws = sum;
                }
            }
            const T rv = ld_stream(r + o) - alpha * ws;
            st_stream(rv, r + o);
            const double im = inv_mult(ld_stream(mult + o));
            const double rd = (double)rv;
            rr += rd * rd * im;
            rz += rd * (double)(ld_stream(inv + o) * rv) * im;
        }
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
    // eight partial sums per thread (eight loads in flight), combined in order
    constexpr int K = 8;
    double s[NV], acc[K][NV];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[c][q] = 0.0;
    const int64_t B = blockDim.x;
    int64_t b = threadIdx.x;
    for (; b + (K - 1) * B < n; b += K * B)
#pragma unroll
        for (int c = 0; c < K; ++c)
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[c][q] += partial[(b + c * B) * NV + q];
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (b + c * B < n)
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[c][q] += partial[(b + c * B) * NV + q];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        s[q] = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) s[q] += acc[c][q];
    }
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
// Diagonal of the local Helmholtz operator, one lane per local point
// (i,j,k) of element e.  The basis function of the point has an r-derivative
// only on its r-line, so the diagonal is the h1*g1-weighted sum of D[l][i]^2
// along that line, likewise for s and t, plus the cross terms at the point
// itself (2 h1 (g4 D_ii D_jj + g5 D_ii D_kk + g6 D_jj D_kk)) and h2*B.
__global__ __launch_bounds__(256) void helm_diag_kernel(int N, int64_t E, const double *__restrict__ G,
                                                        const double *__restrict__ h1,
                                                        const double *__restrict__ h2b, double *__restrict__ diag)
{
    const int P = N + 1, P2 = P * P, P3 = P2 * P;
    const double *D = c_D64 + dtable_offset(N);
    const int64_t n = E * P3;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q / P3;
        const int pt = (int)(q - e * P3);
        const int k = pt / P2, j = (pt / P) % P, i = pt % P;
        const double *Ge = G + e * 6 * P3;
        const double *he = h1 ? h1 + e * P3 : nullptr;
        double d = 0.0;
        for (int l = 0; l < P; ++l) {
            const int pr = l + P * j + P2 * k, ps = i + P * l + P2 * k, pt3 = i + P * j + P2 * l;
            const double hr = he ? he[pr] : 1.0, hs = he ? he[ps] : 1.0, ht = he ? he[pt3] : 1.0;
            const double dr = D[l * P + i], ds = D[l * P + j], dt = D[l * P + k];
            d += hr * Ge[0 * P3 + pr] * dr * dr + hs * Ge[1 * P3 + ps] * ds * ds + ht * Ge[2 * P3 + pt3] * dt * dt;
        }
        const double h = he ? he[pt] : 1.0;
        const double dii = D[i * P + i], djj = D[j * P + j], dkk = D[k * P + k];
        d += 2.0 * h * (Ge[3 * P3 + pt] * dii * djj + Ge[4 * P3 + pt] * dii * dkk + Ge[5 * P3 + pt] * djj * dkk);
        if (h2b) d += h2b[q];
        diag[q] = d;
    }
}

__global__ void invert_positive_kernel(int64_t n, const double *__restrict__ v, double *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = v[q] > 0.0 ? 1.0 / v[q] : 0.0;
}

__global__ void fill_kernel(int64_t n, double value, double *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        out[q] = value;
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

size_t ax_lds_bytes(int N, int epw, size_t elem, int mode)
{
    const size_t P2 = (size_t)(N + 1) * (N + 1), P3 = P2 * (N + 1);
    const bool planes = plane_tile_use(N, mode, (int)elem);
    return (size_t)epw * 3 * (planes ? P2 : P3) * elem;
}


// Workgroups of a persistent operator launch: at most cap (the partials
// buffer holds that many) and at most one per tile.  With `whole_rounds`,
// when fewer than cap workgroups of this kernel fit on the device at once,
// the largest multiple of that resident count, so that no partial last round
// leaves SIMDs idle.  Measured on the 48x48x96 pipe this pays for the
// coarse-corrected FP32 operator (three waves per SIMD, one-wave
// workgroups: 1.60 -> 1.19 ms) but not for the plain ones (FP32 at N = 9
// lost 12%), so only the coarse modes ask for it.
static int64_t resident_grid(const void *fn, int threads, size_t lds, int64_t tiles, int cap, bool whole_rounds)
{
    if (!whole_rounds) return tiles < cap ? tiles : cap;
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int64_t> resident;
    int dev = 0;
    int64_t res = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> lock(mu);
        const auto key = std::make_tuple(fn, threads, lds, dev);
        auto it = resident.find(key);
        if (it == resident.end()) {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) per_cu = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
            it = resident.emplace(key, (int64_t)per_cu * cus).first;
        }
        res = it->second;
    }
    int64_t c = cap;
    if (res > 0 && res < c) c = (c / res) * res;
    return tiles < c ? tiles : c;
}

// dynamic LDS a workgroup may request on the current device
static size_t max_dynamic_lds()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 65536;
    return (size_t)v - 4096;  // static LDS of the kernel (reduction, D copy)
}

template <typename T, int MODE, bool HELM>
static hipError_t launch_ax_mode(int N, const AxParams<T> &a, hipStream_t s, int64_t *grid)
{
    if constexpr (MODE == 3 || MODE == 5) {
        if (!a.evert || !a.z0 || !a.cq) return hipErrorInvalidValue;
    }
    static const size_t lds_cap = max_dynamic_lds();
    const int threads = ax_block_threads(N, a.epw);
    const size_t lds = ax_lds_bytes(N, a.epw, sizeof(T), MODE);
    const int64_t tiles = (a.E + a.epw - 1) / a.epw;
    int64_t blocks = 0;
    if (threads > 512 || lds > lds_cap || tiles < 1 || a.grid_cap < 1) return hipErrorInvalidConfiguration;
    switch (N) {
#define SEM_AX_CASE(n)                                                                                       \
    case n:                                                                                                  \
        blocks = resident_grid(reinterpret_cast<const void *>(&ax_kernel<T, n, MODE, HELM>), threads, lds,   \
                               tiles, a.grid_cap, MODE == 3 || MODE == 5);                                   \
        hipLaunchKernelGGL((ax_kernel<T, n, MODE, HELM>), dim3((unsigned)blocks), dim3(threads), lds, s, a); \
        break;
        SEM_AX_CASE(1) SEM_AX_CASE(2) SEM_AX_CASE(3) SEM_AX_CASE(4) SEM_AX_CASE(5) SEM_AX_CASE(6)
        SEM_AX_CASE(7) SEM_AX_CASE(8) SEM_AX_CASE(9) SEM_AX_CASE(10) SEM_AX_CASE(11) SEM_AX_CASE(12)
    default:
        // orders 13..17 (up to the LDS of one element per workgroup): the plain
        // and CG modes only
        if constexpr (MODE <= 2) {
            switch (N) {
                SEM_AX_CASE(13) SEM_AX_CASE(14) SEM_AX_CASE(15) SEM_AX_CASE(16) SEM_AX_CASE(17)
            default: return hipErrorInvalidValue;
            }
        } else {
            return hipErrorInvalidValue;
        }
    }
#undef SEM_AX_CASE
    if (grid) *grid = blocks;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ax(int N, int mode, const AxParams<T> &a, hipStream_t s, int64_t *grid)
{
    if (mode == 3) {
        if (a.h1) return launch_ax_mode<T, 3, true>(N, a, s, grid);
        return launch_ax_mode<T, 3, false>(N, a, s, grid);
    }
    if (mode == 4 || mode == 5) {
        // the preconditioned residual is given (FP64 solves)
        if constexpr (sizeof(T) == 8) {
            if (mode == 4)
                return a.h1 ? launch_ax_mode<T, 4, true>(N, a, s, grid) : launch_ax_mode<T, 4, false>(N, a, s, grid);
            return a.h1 ? launch_ax_mode<T, 5, true>(N, a, s, grid) : launch_ax_mode<T, 5, false>(N, a, s, grid);
        }
        return hipErrorInvalidValue;
    }
    if (a.h1) {
        if (mode == 0) return launch_ax_mode<T, 0, true>(N, a, s, grid);
        if (mode == 1) return launch_ax_mode<T, 1, true>(N, a, s, grid);
        return launch_ax_mode<T, 2, true>(N, a, s, grid);
    }
    if (mode == 0) return launch_ax_mode<T, 0, false>(N, a, s, grid);
    if (mode == 1) return launch_ax_mode<T, 1, false>(N, a, s, grid);
    return launch_ax_mode<T, 2, false>(N, a, s, grid);
}
template hipError_t launch_ax<double>(int, int, const AxParams<double> &, hipStream_t, int64_t *);
template hipError_t launch_ax<float>(int, int, const AxParams<float> &, hipStream_t, int64_t *);

template <typename T>
hipError_t launch_gs(const GsPlan &plan, const int32_t *off, const int32_t *idx, T *v, bool zero_only,
                     const PcgState *st, hipStream_t s)
{
    const int64_t first = zero_only ? plan.n_sum : 0;
    const int64_t n = plan.n_ids - first;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((gs_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, plan, first, off, idx, v, st);
    return hipGetLastError();
}
template hipError_t launch_gs<double>(const GsPlan &, const int32_t *, const int32_t *, double *, bool,
                                      const PcgState *, hipStream_t);
template hipError_t launch_gs<float>(const GsPlan &, const int32_t *, const int32_t *, float *, bool,
                                     const PcgState *, hipStream_t);

// Row-streaming gather-scatter of the nodes off the z-planes (orders 2..7,
// (N+1)^2 <= 64 lanes).  One wavefront per (element row yg in y, interior
// plane k, element layer ez) walks the row along x.  Its lanes hold the N+1
// rows of the lattice lines Y = yg N .. yg N + N - 1 at plane k of the
// current element: slot 0 the row j = N of element row yg - 1 (the other
// copy of the line Y = yg N), slots 1..N the rows j = 0..N-1 of element row
// yg; lane (slot, i) holds GLL index i.  Rows are loaded and stored whole
// (coalesced).  Every lane that holds a copy of a shared node forms the
// node's sum itself from the copies' values (cross-lane shuffles), from 0 in
// ascending local index -- y copies outer, x copies inner, as the lattice
// rule orders them -- so all copies get the same bits as the per-node
// kernel writes.  The x-face X = ex N is formed at step ex from the
// previous element's i = N and the current element's i = 0; the previous
// element's rows are then final and stored.  On a periodic x axis the face
// X = 0 waits for the last element.  For a non-periodic y axis the group
// yg = nel[1] holds only slot 0 (the top boundary line).
template <typename T, int N>
__device__ inline void gs_stream_wave(const GsLattice &L, int64_t wv, T *__restrict__ v)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    const int nx = L.nel[0], ny = L.nel[1];
    const bool px = L.periodic[0] != 0, py = L.periodic[1] != 0;
    const int ngy = py ? ny : ny + 1;
    const int yg = (int)(wv % ngy);
    const int64_t rest = wv / ngy;
    const int k = 1 + (int)(rest % (N - 1));
    const int ez = (int)(rest / (N - 1));
    const int lane = threadIdx.x & 63;
    const int sl = lane / P, i = lane - sl * P;
    bool act = lane < P2;
    int eys = 0, js = 0;
    if (sl == 0) {
        js = N;
        if (yg > 0) eys = yg - 1;
        else if (py) eys = ny - 1;
        else act = false;
    } else {
        js = sl - 1;
        if (yg < ny) eys = yg;
        else act = false;
    }
    if (!act) { eys = 0; js = 0; }
    // the y copies of this lane's line, in ascending element order
    int cy = 1, ys0 = sl, ys1 = sl;
    bool ymask = false;
    if (sl <= 1) {
        const bool has0 = yg > 0 || py, has1 = yg < ny;
        if (has0 && has1) {
            cy = 2;
            if (py && yg == 0) { ys0 = 1; ys1 = 0; }  // element row 0 before the wrapped last one
            else { ys0 = 0; ys1 = 1; }
        } else {
            cy = 1; ys0 = ys1 = has1 ? 1 : 0;
            ymask = has1 ? (L.faces & 4) != 0 : (L.faces & 8) != 0;
        }
    }
    const bool yline = sl <= 1;
    const int64_t rowoff = (int64_t)k * P2 + (int64_t)js * P + i;
    const int64_t rowbase = ((int64_t)ez * ny + eys) * nx;  // element index of ex = 0 in this lane's row
    auto addr = [&](int ex) { return (rowbase + ex) * P3 + rowoff; };
    // sum over y copies (outer) and x copies (inner) of values drawn from
    // lanes: x copy q takes register a (q = 0) or b (q = 1) at GLL index xi[q]
    auto node_sum = [&](T a, T b, int cx, int xi0, int xi1) {
        T s = T(0);
#pragma unroll
        for (int qy = 0; qy < 2; ++qy) {
            const int ysl = qy == 0 ? ys0 : ys1;
#pragma unroll
            for (int qx = 0; qx < 2; ++qx) {
                const int src = ysl * P + (qx == 0 ? xi0 : xi1);
                const T va = __shfl(a, src, 64), vb = __shfl(b, src, 64);
                if (qy < cy && qx < cx) s = s + (qx == 0 ? va : vb);
            }
        }
        return s;
    };
    T first = T(0), prev = T(0);
    T n1 = act ? v[addr(0)] : T(0);
    T n2 = (act && nx > 1) ? v[addr(1)] : T(0);
    for (int ex = 0; ex < nx; ++ex) {
        T cur = n1;
        n1 = n2;
        if (act && ex + 2 < nx) n2 = v[addr(ex + 2)];
        // the line nodes off the x-faces (1 <= i <= N-1): y copies only
        T curn = cur;
        {
            const T sy = node_sum(cur, cur, 1, i, i);
            if (yline && i >= 1 && i <= N - 1) {
                if (ymask) curn = T(0);
                else if (cy == 2) curn = sy;
            }
        }
        if (ex > 0) {
            // x-face X = ex N: copies (ex - 1, N) in prev, (ex, 0) in cur
            const T sf = node_sum(prev, cur, 2, N, 0);
            const T f = (yline && ymask) ? T(0) : sf;
            if (i == 0) curn = f;
            T prevn = prev;
            if (i == N) prevn = f;
            if (act) v[addr(ex - 1)] = prevn;
        } else {
            // X = 0: a boundary face, or on a periodic axis the wrap with the last element
            const T sb = node_sum(cur, cur, 1, 0, 0);
            if (!px && i == 0) {
                if ((L.faces & 1) || (yline && ymask)) curn = T(0);
                else if (yline && cy == 2) curn = sb;
            }
            first = cur;
        }
        prev = curn;
    }
    // the last face X = nx N
    if (px) {
        // copies (0, 0) in first (its raw value), (nx - 1, N) in prev
        const T sw = node_sum(first, prev, 2, 0, N);
        const T f = (yline && ymask) ? T(0) : sw;
        if (i == N) prev = f;
        if (act && i == 0) v[addr(0)] = f;
    } else {
        const T sb = node_sum(prev, prev, 1, N, N);
        if (i == N) {
            if ((L.faces & 2) || (yline && ymask)) prev = T(0);
            else if (yline && cy == 2) prev = sb;
        }
    }
    if (act) v[addr(nx - 1)] = prev;
}

template <typename T, int N>
__global__ __launch_bounds__(256) void gs_stream_kernel(GsLattice L, GsLattice Lz, T *__restrict__ v,
                                                        const PcgState *__restrict__ st, int64_t nwaves,
                                                        unsigned sblocks)
{
    if (st && st->done) return;
    const unsigned b = blockIdx.x;
    if (b < sblocks) {
        const int64_t wv = (int64_t)b * 4 + (threadIdx.x >> 6);
        if (wv < nwaves) gs_stream_wave<T, N>(L, wv, v);
        return;
    }
    // the z-planes: one lane per node, XCD-contiguous (sblocks is a multiple of 8)
    const unsigned nb = gridDim.x - sblocks, bb = b - sblocks;
    const unsigned per = nb / 8, rem = nb % 8, xcd = bb % 8, kb = bb / 8;
    const unsigned lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + kb;
    const int64_t t = (int64_t)lb * blockDim.x + threadIdx.x;
    if (t < Lz.n_nodes) gs_lattice_node<T>(Lz, t, v);
}

template <typename T>
hipError_t launch_gs_lattice(const GsLattice &L, T *v, const PcgState *st, hipStream_t s, bool force_stream)
{
    const int64_t ngy = L.periodic[1] ? L.nel[1] : L.nel[1] + 1;
    const int64_t nwaves = ngy * (L.N - 1) * L.nel[2];
    // measured: the row walks win at N = 7 once there are enough of them to
    // fill the device; at lower orders most lanes of a wave are idle and on
    // small meshes the walks are too few, and the per-node kernel is faster
    const bool stream = L.N >= 2 && L.N <= 7 && (force_stream || (L.N == 7 && nwaves >= 2048));
    if (stream) {
        GsLattice Lz{};
        if (!gs_lattice_make(L.N, L.nel, L.periodic, L.faces, Lz, true)) return hipErrorInvalidValue;
        const int64_t sblocks = ((nwaves + 3) / 4 + 7) / 8 * 8;
        const int64_t zblocks = (Lz.n_nodes + 255) / 256;
        const dim3 grid((unsigned)(sblocks + zblocks));
        switch (L.N) {
#define SEM_GSS_CASE(n)                                                                                      \
    case n:                                                                                                  \
        hipLaunchKernelGGL((gs_stream_kernel<T, n>), grid, dim3(256), 0, s, L, Lz, v, st, nwaves,           \
                           (unsigned)sblocks);                                                               \
        break;
            SEM_GSS_CASE(2) SEM_GSS_CASE(3) SEM_GSS_CASE(4) SEM_GSS_CASE(5) SEM_GSS_CASE(6) SEM_GSS_CASE(7)
#undef SEM_GSS_CASE
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int64_t n = L.n_nodes;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL((gs_lattice_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, L, v, st);
    return hipGetLastError();
}
template hipError_t launch_gs_lattice<double>(const GsLattice &, double *, const PcgState *, hipStream_t, bool);
template hipError_t launch_gs_lattice<float>(const GsLattice &, float *, const PcgState *, hipStream_t, bool);

int vec_blocks(int64_t n) { return grid_for(n, 256, 8192); }

hipError_t launch_helm_diag(int N, int64_t E, const double *G, const double *h1, const double *h2b, double *diag,
                            hipStream_t s)
{
    if (N < 1 || N > SEM_MAX_ORDER) return hipErrorInvalidValue;
    const int64_t n = E * (int64_t)(N + 1) * (N + 1) * (N + 1);
    hipLaunchKernelGGL(helm_diag_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, N, E, G, h1, h2b, diag);
    return hipGetLastError();
}
hipError_t launch_invert_positive(int64_t n, const double *v, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(invert_positive_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, v, out);
    return hipGetLastError();
}
hipError_t launch_fill(int64_t n, double value, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, value, out);
    return hipGetLastError();
}
int update_blocks(int64_t n) { return grid_for((n + 1) / 2, 256, 65536); }

hipError_t upload_dtables(const double *d64, const float *d32, hipStream_t s)
{
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D64), d64, sizeof(double) * kDTableSize, 0,
                                          hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_D32), d32, sizeof(float) * kDTableSize, 0, hipMemcpyHostToDevice, s);
}

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
template <typename T>
hipError_t launch_pcg_init_partials(int64_t n, const T *r, const T *inv, const uint8_t *mult, double *partial,
                                    hipStream_t s)
{
    hipLaunchKernelGGL((pcg_init_kernel<T>), dim3(vec_blocks(n)), dim3(256), 0, s, n, r, inv, mult, partial);
    return hipGetLastError();
}
template hipError_t launch_pcg_init_partials<double>(int64_t, const double *, const double *, const uint8_t *,
                                                     double *, hipStream_t);
template hipError_t launch_pcg_init_partials<float>(int64_t, const float *, const float *, const uint8_t *, double *,
                                                    hipStream_t);
hipError_t launch_reduce_init(const double *partial, int64_t pairs, PcgState *st, double stop2, int limit,
                              hipStream_t s)
{
    hipLaunchKernelGGL(reduce_init_kernel, dim3(1), dim3(1024), 0, s, partial, pairs, st, stop2, limit);
    return hipGetLastError();
}
template hipError_t launch_pcg_init<float>(int64_t, const float *, const float *, const uint8_t *, double *,
                                           PcgState *, double, int, hipStream_t);

template <typename T>
hipError_t launch_pcg_update(int64_t n, const PcgState *st, T *r, const T *w, const T *inv, const uint8_t *mult,
                             double *partial, hipStream_t s)
{
    const int blocks = update_blocks(n);
    hipLaunchKernelGGL((pcg_update_kernel<T>), dim3(blocks), dim3(256), 0, s, n, st, r, w, inv, mult, partial);
    return hipGetLastError();
}
template hipError_t launch_pcg_update<double>(int64_t, const PcgState *, double *, const double *, const double *,
                                              const uint8_t *, double *, hipStream_t);

int update_elem_blocks(int64_t E) { return (int)std::max<int64_t>(1, std::min<int64_t>((E + 3) / 4, 8192)); }

template <typename T>
hipError_t launch_pcg_update_elem(int N, int64_t E, const PcgState *st, T *r, const T *w, const T *inv,
                                  const uint8_t *mult, double *partial, hipStream_t s)
{
    const int blocks = update_elem_blocks(E);
    switch (N) {
#define SEM_UPD_CASE(n)                                                                                           \
    case n:                                                                                                       \
        hipLaunchKernelGGL((pcg_update_elem_kernel<T, n>), dim3(blocks), dim3(256), 0, s, E, st, r, w, inv, mult, \
                           partial);                                                                              \
        break;
        SEM_UPD_CASE(3) SEM_UPD_CASE(4) SEM_UPD_CASE(5) SEM_UPD_CASE(6) SEM_UPD_CASE(7) SEM_UPD_CASE(8)
        SEM_UPD_CASE(9) SEM_UPD_CASE(10) SEM_UPD_CASE(11) SEM_UPD_CASE(12) SEM_UPD_CASE(13) SEM_UPD_CASE(14)
        SEM_UPD_CASE(15) SEM_UPD_CASE(16) SEM_UPD_CASE(17)
#undef SEM_UPD_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_pcg_update_gs(const GsLattice &L, int N, int64_t E, const PcgState *st, T *r, const T *w,
                                const T *inv, const uint8_t *mult, double *partial, hipStream_t s)
{
    // copy offsets are formed in 32 bits
    if (E * (int64_t)(N + 1) * (N + 1) * (N + 1) >= INT32_MAX) return hipErrorInvalidValue;
    const int blocks = update_elem_blocks(E);
    switch (N) {
#define SEM_UPDGS_CASE(n)                                                                                       \
    case n:                                                                                                     \
        hipLaunchKernelGGL((pcg_update_gs_kernel<T, n>), dim3(blocks), dim3(256), 0, s, L, E, st, r, w, inv,     \
                           mult, partial);                                                                      \
        break;
        SEM_UPDGS_CASE(3) SEM_UPDGS_CASE(4) SEM_UPDGS_CASE(5) SEM_UPDGS_CASE(6) SEM_UPDGS_CASE(7)
        SEM_UPDGS_CASE(8) SEM_UPDGS_CASE(9) SEM_UPDGS_CASE(10) SEM_UPDGS_CASE(11) SEM_UPDGS_CASE(12)
        SEM_UPDGS_CASE(13) SEM_UPDGS_CASE(14) SEM_UPDGS_CASE(15) SEM_UPDGS_CASE(16) SEM_UPDGS_CASE(17)
#undef SEM_UPDGS_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_pcg_update_gs<double>(const GsLattice &, int, int64_t, const PcgState *, double *,
                                                 const double *, const double *, const uint8_t *, double *,
                                                 hipStream_t);
template hipError_t launch_pcg_update_gs<float>(const GsLattice &, int, int64_t, const PcgState *, float *,
                                                const float *, const float *, const uint8_t *, double *, hipStream_t);

template hipError_t launch_pcg_update_elem<double>(int, int64_t, const PcgState *, double *, const double *,
                                                   const double *, const uint8_t *, double *, hipStream_t);
template hipError_t launch_pcg_update_elem<float>(int, int64_t, const PcgState *, float *, const float *,
                                                  const float *, const uint8_t *, double *, hipStream_t);
template hipError_t launch_pcg_update<float>(int64_t, const PcgState *, float *, const float *, const float *,
                                             const uint8_t *, double *, hipStream_t);

// End of a CG run: apply the last x step (not after a breakdown, whose alpha
// was never formed).
template <typename T>
__global__ __launch_bounds__(256) void pcg_finish_kernel(int64_t n, const PcgState *__restrict__ st,
                                                         T *__restrict__ x, const T *__restrict__ p)
{
    if (st->done == 2 || st->iters == 0) return;
    const T alpha = (T)st->alpha;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        x[q] = x[q] + alpha * p[q];
}

template <typename T>
hipError_t launch_pcg_finish(int64_t n, const PcgState *st, T *x, const T *p, hipStream_t s)
{
    hipLaunchKernelGGL((pcg_finish_kernel<T>), dim3(vec_blocks(n)), dim3(256), 0, s, n, st, x, p);
    return hipGetLastError();
}
template hipError_t launch_pcg_finish<double>(int64_t, const PcgState *, double *, const double *, hipStream_t);
template hipError_t launch_pcg_finish<float>(int64_t, const PcgState *, float *, const float *, hipStream_t);

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
