// coarse.hip -- the coarse term of Eq. 6 on the GPU: a two-level
// preconditioner M^{-1} r = D^{-1} r + P C(A0) P^T r for FP64 CG.
//
//  * P: trilinear hat functions of the element vertices at the GLL nodes (in
//    each element's reference coordinates), zero at Dirichlet nodes.
//  * A0 = P^T A P, assembled on the host from per-element 8x8 blocks
//    P_e^T A_e P_e; each block column is the local operator applied to one
//    masked hat function, tested against the eight hats.
//  * C(A0): k steps of Chebyshev iteration for D0^-1 A0 z = D0^-1 r0 from 0
//    on [frac b, b], b the largest absolute row sum of D0^-1 A0 -- a fixed
//    polynomial, so M stays linear and symmetric positive definite.
//  * Restriction P^T r: per element, eight weighted sums over its nodes
//    (1/mult for unique-node sums), then per vertex the sum of its element
//    corners in a fixed order.  Prolongation: folded into the CG operator's
//    prologue (p = D^-1 r + P z0 + beta p), or added to a vector.
//  * The coarse part of <r, z> is r0 . z0, appended to the CG partials.
// Dirichlet nodes are the nodes whose inverse diagonal is 0.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "coarse.hpp"
#include "kernels.hpp"
#include "operator.hpp"

namespace sem {

// ---------------------------------------------------------------------------
// device kernels

// node q of an element: (i, j, k) and the eight hat weights
__device__ inline void hat_weights(const double *__restrict__ qw, int P, int q, double (&phi)[8])
{
    const int i = q % P, j = (q / P) % P, k = q / (P * P);
    const double ai[2] = {qw[i], qw[P + i]}, aj[2] = {qw[j], qw[P + j]}, ak[2] = {qw[k], qw[P + k]};
#pragma unroll
    for (int c = 0; c < 8; ++c) phi[c] = ai[c & 1] * aj[(c >> 1) & 1] * ak[(c >> 2) & 1];
}

// u = masked hat function of corner c on every element (element-local vector)
__global__ __launch_bounds__(256) void hat_kernel(int64_t E, int P, const double *__restrict__ qw, int c,
                                                  const double *__restrict__ inv, double *__restrict__ u)
{
    const int P3 = P * P * P;
    const int64_t n = E * P3;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double phi[8];
        hat_weights(qw, P, (int)(q % P3), phi);
        u[q] = inv[q] > 0.0 ? phi[c] : 0.0;
    }
}

// One wavefront per element: s[c] = sum over the element's live nodes of
// phi_c * f (f = the element's slice of a vector, scaled by w when given);
// every lane ends with the eight totals (butterfly, fixed order).
__device__ inline void wave_hat_sums(int P, const double *__restrict__ sqw, const double *__restrict__ f,
                                     const uint8_t *__restrict__ mult, const double *__restrict__ inv,
                                     double (&s)[8])
{
    const int P3 = P * P * P, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = 0.0;
    for (int q = lane; q < P3; q += 64) {
        double v = inv[q] > 0.0 ? f[q] : 0.0;
        if (mult) v /= (double)mult[q];
        double phi[8];
        hat_weights(sqw, P, q, phi);
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] += phi[c] * v;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
        for (int off = 32; off > 0; off >>= 1) s[c] += __shfl_xor(s[c], off, 64);
}

__device__ inline double pick8(const double (&s)[8], int c)
{
    double out = s[0];
#pragma unroll
    for (int q = 1; q < 8; ++q)
        if (c == q) out = s[q];
    return out;
}

// E8[e][c'][c] = sum over element e's live nodes of phi_c' * w, w = A_e u_c
__global__ __launch_bounds__(256) void elem_coarse_kernel(int64_t E, int P, const double *__restrict__ w,
                                                          const double *__restrict__ qw,
                                                          const double *__restrict__ inv, int c,
                                                          double *__restrict__ E8)
{
    __shared__ double sqw[2 * (SEM_MAX_ORDER + 1)];
    if (threadIdx.x < 2 * P) sqw[threadIdx.x] = qw[threadIdx.x];
    __syncthreads();
    const int P3 = P * P * P, lane = threadIdx.x & 63;
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < E; e += (int64_t)gridDim.x * 4) {
        double s[8];
        wave_hat_sums(P, sqw, w + e * P3, nullptr, inv + e * P3, s);
        const double v = pick8(s, lane);
        if (lane < 8) E8[e * 64 + lane * 8 + c] = v;
    }
}

// Hat-function sums at compile-time order: node q = i + P j + P^2 k of an
// element adds v phi_c(q) to s[c], phi_c = a[cx][i] a[cy][j] a[cz][k]
// (c = cx + 2 cy + 4 cz, a[side][.] the 1-D weights in LDS).
template <int N>
__device__ inline void hat_add(const double *__restrict__ sqw, int q, double v, double (&s)[8])
{
    constexpr int P = N + 1, P2 = P * P;
    const int i = q % P, j = (q / P) % P, k = q / P2;
    const double ai0 = sqw[i], ai1 = sqw[P + i];
    const double aj0 = sqw[j], aj1 = sqw[P + j], ak0 = sqw[k], ak1 = sqw[P + k];
    const double t00 = aj0 * ak0 * v, t10 = aj1 * ak0 * v, t01 = aj0 * ak1 * v, t11 = aj1 * ak1 * v;
    s[0] += ai0 * t00; s[1] += ai1 * t00; s[2] += ai0 * t10; s[3] += ai1 * t10;
    s[4] += ai0 * t01; s[5] += ai1 * t01; s[6] += ai0 * t11; s[7] += ai1 * t11;
}

// butterfly over the wavefront: every lane ends with the eight totals
__device__ inline void wave_sum8(double (&s)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c)
        for (int off = 32; off > 0; off >>= 1) s[c] += __shfl_xor(s[c], off, 64);
}

// partial8[e*8 + c] = sum over element e's live nodes of phi_c r / mult;
// one wavefront per element
template <typename T, int N>
__global__ __launch_bounds__(256) void restrict_elem_kernel(int64_t E, const T *__restrict__ r,
                                                            const uint8_t *__restrict__ mult,
                                                            const T *__restrict__ inv,
                                                            const double *__restrict__ qw,
                                                            double *__restrict__ partial8)
{
    constexpr int P = N + 1, P3 = P * P * P;
    __shared__ double sqw[2 * P];
    if (threadIdx.x < 2 * P) sqw[threadIdx.x] = qw[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < E; e += (int64_t)gridDim.x * 4) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int64_t base = e * P3;
#pragma unroll
        for (int q = lane; q < P3; q += 64) {
            const T iv = ld_stream(inv + base + q);
            const double v = iv > T(0) ? (double)ld_stream(r + base + q) / (double)mult[base + q] : 0.0;
            hat_add<N>(sqw, q, v, s);
        }
        wave_sum8(s);
        const double out = pick8(s, lane);
        if (lane < 8) partial8[e * 8 + lane] = out;
    }
}

// CG update with the coarse restriction fused in: r -= alpha w, the partial
// pairs of <r,r> and <r, invdiag r> per workgroup (FP64 sums, the products
// as in the plain update; the second 0 unless with_rz), and the element
// restriction sums of the new r; one wavefront per element.
template <typename T, int N>
__global__ __launch_bounds__(256) void update_restrict_kernel(int64_t E, const PcgState *__restrict__ st,
                                                              T *__restrict__ r, const T *__restrict__ w,
                                                              const T *__restrict__ inv,
                                                              const uint8_t *__restrict__ mult,
                                                              const double *__restrict__ qw,
                                                              double *__restrict__ partial,
                                                              double *__restrict__ partial8, int with_rz)
{
    constexpr int P = N + 1, P3 = P * P * P;
    if (st->done) return;
    __shared__ double sqw[2 * P];
    if (threadIdx.x < 2 * P) sqw[threadIdx.x] = qw[threadIdx.x];
    __syncthreads();
    const T alpha = (T)st->alpha;
    const int lane = threadIdx.x & 63;
    double rr = 0.0, rz = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < E; e += (int64_t)gridDim.x * 4) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int64_t base = e * P3;
        if constexpr (sizeof(T) == 4 && P3 % 2 == 0) {
            // FP32, N odd: two adjacent nodes of one element row per lane
            // (paired 8-byte loads), in the same per-node arithmetic
            const float2 *r2 = reinterpret_cast<const float2 *>(r + base);
            const float2 *w2 = reinterpret_cast<const float2 *>(w + base);
            const float2 *i2 = reinterpret_cast<const float2 *>(inv + base);
            const uint16_t *m2 = reinterpret_cast<const uint16_t *>(mult + base);
#pragma unroll
            for (int h = lane; h < P3 / 2; h += 64) {
                float2 rv = ld_stream(r2 + h);
                const float2 wv = ld_stream(w2 + h), iv = ld_stream(i2 + h);
                const uint16_t mm = ld_stream(m2 + h);
                rv.x = rv.x - (float)alpha * wv.x;
                rv.y = rv.y - (float)alpha * wv.y;
                st_stream(rv, reinterpret_cast<float2 *>(r + base) + h);
                const double ima = 1.0 / (double)(mm & 0xff), imb = 1.0 / (double)(mm >> 8);
                const double ra = (double)rv.x, rb = (double)rv.y;
                rr += ra * ra * ima;
                rr += rb * rb * imb;
                if (with_rz) {
                    rz += ra * (double)(iv.x * rv.x) * ima;
                    rz += rb * (double)(iv.y * rv.y) * imb;
                }
                hat_add<N>(sqw, 2 * h, iv.x > 0.0f ? ra * ima : 0.0, s);
                hat_add<N>(sqw, 2 * h + 1, iv.y > 0.0f ? rb * imb : 0.0, s);
            }
        } else {
#pragma unroll
            for (int q = lane; q < P3; q += 64) {
                const int64_t o = base + q;
                const T rv = ld_stream(r + o) - alpha * ld_stream(w + o);
                st_stream(rv, r + o);
                const T iv = ld_stream(inv + o);
                const double im = 1.0 / (double)ld_stream(mult + o);
                const double rd = (double)rv;
                rr += rd * rd * im;
                if (with_rz) rz += rd * (double)(iv * rv) * im;
                hat_add<N>(sqw, q, iv > T(0) ? rd * im : 0.0, s);
            }
        }
        wave_sum8(s);
        const double out = pick8(s, lane);
        if (lane < 8) partial8[e * 8 + lane] = out;
    }
    double v[2] = {rr, rz};
    block_reduce_store<2>(v, partial, 2);
}

// r0[v] = sum of v's element corners (ascending element, corner); then the
// Chebyshev start: z = 0, res = r0, d = D0^-1 r0 / theta
__global__ __launch_bounds__(256) void restrict_vert_kernel(int64_t nv, const int32_t *__restrict__ v_off,
                                                            const int32_t *__restrict__ v_idx,
                                                            const double *__restrict__ partial8,
                                                            const double *__restrict__ d0inv, double inv_theta,
                                                            double *__restrict__ r0, double *__restrict__ z,
                                                            double *__restrict__ res, double *__restrict__ d,
                                                            const PcgState *__restrict__ st)
{
    if (st && st->done) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t q = v_off[v]; q < v_off[v + 1]; ++q) s += partial8[v_idx[q]];
        r0[v] = s;
        z[v] = 0.0;
        res[v] = s;
        d[v] = s * d0inv[v] * inv_theta;
    }
}

// One Chebyshev step, eight lanes per row of A0 (its entries read
// contiguously, summed by a fixed butterfly):
//   z += d_in; res -= A0 d_in; d_out = c1 d_in + c2 D0^-1 res.
// LAST: no d_out; (0, sum r0 z) pairs per workgroup into `partial` when given.
template <bool LAST>
__global__ __launch_bounds__(256) void cheb_kernel(int64_t nv, const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                                   double c1, double c2, const double *__restrict__ d0inv,
                                                   const double *__restrict__ din, double *__restrict__ dout,
                                                   double *__restrict__ z, double *__restrict__ res,
                                                   const double *__restrict__ r0, double *__restrict__ partial,
                                                   const PcgState *__restrict__ st)
{
    if (st && st->done) return;
    const int sub = threadIdx.x & 7;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double dot = 0.0;
    // wave-uniform trip count: the butterfly runs on full wavefronts
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < nv * 8; t0 += stride) {
        const int64_t v = (t0 + (threadIdx.x & 63)) >> 3;
        double s = 0.0;
        if (v < nv)
            for (int32_t q = off[v] + sub; q < off[v + 1]; q += 8) s += val[q] * din[col[q]];
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 1, 64);
        if (v < nv && sub == 0) {
            const double dv = din[v];
            const double zv = z[v] + dv;
            z[v] = zv;
            const double rv = res[v] - s;
            res[v] = rv;
            if (!LAST) dout[v] = c1 * dv + c2 * rv * d0inv[v];
            else dot += r0[v] * zv;
        }
    }
    if (LAST && partial) {
        double p[2] = {0.0, dot};
        block_reduce_store<2>(p, partial, 2);
    }
}

// ADD: z += masked P z0; else z = masked P z0 (0 on masked nodes), rounded
// to the precision of z
template <bool ADD, typename TZ>
__global__ __launch_bounds__(256) void prolong_kernel(int64_t E, int P, const int32_t *__restrict__ evert,
                                                      const double *__restrict__ z0, const double *__restrict__ qw,
                                                      const double *__restrict__ inv, TZ *__restrict__ z)
{
    const int P3 = P * P * P;
    const int64_t n = E * P3;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (!(inv[q] > 0.0)) {
            if (!ADD) z[q] = TZ(0);
            continue;
        }
        const int64_t e = q / P3;
        double phi[8];
        hat_weights(qw, P, (int)(q - e * P3), phi);
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += phi[c] * z0[evert[e * 8 + c]];
        z[q] = ADD ? (TZ)(z[q] + s) : (TZ)s;
    }
}

__global__ void jacobi_kernel(int64_t n, const double *__restrict__ inv, const double *__restrict__ r,
                              double *__restrict__ z)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        z[q] = inv[q] * r[q];
}

// ---------------------------------------------------------------------------
// host side

static int cgrid(int64_t n, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap)); }

template <typename X>
static X *cmalloc(CoarseSpace *C, size_t count)
{
    void *p = nullptr;
    SEM_HIP(hipMalloc(&p, std::max<size_t>(count * sizeof(X), 16)));
    C->allocations.push_back(p);
    return static_cast<X *>(p);
}

void coarse_free(CoarseSpace *C)
{
    if (!C) return;
    for (void *p : C->allocations) (void)hipFree(p);
    delete C;
}

CoarseSpace *coarse_build(sem_mesh *m, int k, double frac, hipStream_t s)
{
    const HostMesh &h = m->h;
    const int N = h.N, P = N + 1;
    const int64_t E = h.E, P3 = (int64_t)P * P * P, nL = h.nL;
    if (k < 1 || k > 1000) fail(SEM_EINVAL, "sem_set_coarse: chebyshev_steps must be 1..1000");
    if (!(frac > 0.0 && frac < 1.0)) fail(SEM_EINVAL, "sem_set_coarse: fraction must be in (0, 1)");
    if (E * 8 >= INT32_MAX) fail(SEM_EUNSUPPORTED, "sem_set_coarse: too many elements");
    CoarseSpace *C = new CoarseSpace();
    try {
        C->k = k;
        C->frac = frac;
        const int nx = h.nel[0], ny = h.nel[1], nz = h.nel[2];
        const int vd[3] = {nx + 1 - h.periodic[0], ny + 1 - h.periodic[1], nz + 1 - h.periodic[2]};
        C->nvert = (int64_t)vd[0] * vd[1] * vd[2];
        // element corners -> vertices
        std::vector<int32_t> evert((size_t)E * 8);
        for (int64_t e = 0; e < E; ++e) {
            const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
            for (int c = 0; c < 8; ++c) {
                const int64_t a = (ex + (c & 1)) % vd[0], b = (ey + ((c >> 1) & 1)) % vd[1],
                              cc = (ez + ((c >> 2) & 1)) % vd[2];
                evert[e * 8 + c] = (int32_t)(a + vd[0] * (b + (int64_t)vd[1] * cc));
            }
        }
        // vertex -> (element, corner) entries, ascending
        std::vector<int32_t> v_off((size_t)C->nvert + 1, 0), v_idx((size_t)E * 8);
        for (int64_t q = 0; q < E * 8; ++q) v_off[evert[q] + 1]++;
        for (int64_t v = 0; v < C->nvert; ++v) v_off[v + 1] += v_off[v];
        {
            std::vector<int32_t> cur(v_off.begin(), v_off.end() - 1);
            for (int64_t q = 0; q < E * 8; ++q) v_idx[cur[evert[q]]++] = (int32_t)q;
        }
        // 1-D hat weights at the GLL nodes
        std::vector<double> qw(2 * P);
        for (int i = 0; i < P; ++i) {
            qw[i] = 0.5 * (1.0 - h.xi[i]);
            qw[P + i] = 0.5 * (1.0 + h.xi[i]);
        }
        C->evert = cmalloc<int32_t>(C, evert.size());
        C->v_off = cmalloc<int32_t>(C, v_off.size());
        C->v_idx = cmalloc<int32_t>(C, v_idx.size());
        C->qw = cmalloc<double>(C, qw.size());
        SEM_HIP(hipMemcpyAsync(C->evert, evert.data(), sizeof(int32_t) * evert.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipMemcpyAsync(C->v_off, v_off.data(), sizeof(int32_t) * v_off.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipMemcpyAsync(C->v_idx, v_idx.data(), sizeof(int32_t) * v_idx.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipMemcpyAsync(C->qw, qw.data(), sizeof(double) * qw.size(), hipMemcpyHostToDevice, s));
        // element blocks P_e^T A_e P_e with the mesh's current operator
        std::vector<double> E8((size_t)E * 64);
        {
            double *u = nullptr, *w = nullptr, *dE8 = nullptr;
            SEM_HIP(hipMalloc(&u, sizeof(double) * nL));
            SEM_HIP(hipMalloc(&w, sizeof(double) * nL));
            SEM_HIP(hipMalloc(&dE8, sizeof(double) * E * 64));
            try {
                for (int c = 0; c < 8; ++c) {
                    hipLaunchKernelGGL(hat_kernel, dim3(vec_blocks(nL)), dim3(256), 0, s, E, P, C->qw, c, m->inv64, u);
                    SEM_HIP(hipGetLastError());
                    const sem_status st = sem_ax(m, SEM_FP64, u, w, nullptr, s);
                    if (st != SEM_OK) fail(st, "sem_set_coarse: operator apply failed");
                    hipLaunchKernelGGL(elem_coarse_kernel, dim3(cgrid(E * 64, 8192)), dim3(256), 0, s, E, P, w,
                                       C->qw, m->inv64, c, dE8);
                    SEM_HIP(hipGetLastError());
                }
                SEM_HIP(hipMemcpyAsync(E8.data(), dE8, sizeof(double) * E * 64, hipMemcpyDeviceToHost, s));
                SEM_HIP(hipStreamSynchronize(s));
            } catch (...) {
                hipFree(u);
                hipFree(w);
                hipFree(dE8);
                throw;
            }
            SEM_HIP(hipFree(u));
            SEM_HIP(hipFree(w));
            SEM_HIP(hipFree(dE8));
        }
        // A0 rows: sum of the element blocks of the vertex's corners, ascending
        std::vector<int32_t> off((size_t)C->nvert + 1, 0), col;
        std::vector<double> val, diag((size_t)C->nvert, 0.0);
        col.reserve((size_t)C->nvert * 27);
        val.reserve((size_t)C->nvert * 27);
        // entries of a row are summed in the order of its element corners
        std::vector<std::pair<int32_t, double>> row;
        row.reserve(64);
        for (int64_t v = 0; v < C->nvert; ++v) {
            row.clear();
            for (int32_t q = v_off[v]; q < v_off[v + 1]; ++q) {
                const int64_t e = v_idx[q] / 8, cr = v_idx[q] % 8;
                for (int c = 0; c < 8; ++c) row.emplace_back(evert[e * 8 + c], E8[e * 64 + cr * 8 + c]);
            }
            std::stable_sort(row.begin(), row.end(),
                             [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                                 return x.first < y.first;
                             });
            const size_t start = col.size();
            for (size_t q = 0; q < row.size(); ++q) {
                if (q == 0 || row[q].first != row[q - 1].first) {
                    col.push_back(row[q].first);
                    val.push_back(row[q].second);
                } else {
                    val.back() += row[q].second;
                }
                if (row[q].first == (int32_t)v) diag[v] = val.back();
            }
            if (!(diag[v] > 0.0)) {  // not a coarse unknown: empty row
                col.resize(start);
                val.resize(start);
            }
            off[v + 1] = (int32_t)col.size();
        }
        // vertices whose masked hat is zero are not coarse unknowns: drop their columns
        std::vector<double> d0inv((size_t)C->nvert, 0.0);
        for (int64_t v = 0; v < C->nvert; ++v)
            if (diag[v] > 0.0) d0inv[v] = 1.0 / diag[v];
        double bmax = 0.0;
        for (int64_t v = 0; v < C->nvert; ++v) {
            if (!(diag[v] > 0.0)) continue;
            double sabs = 0.0;
            for (int32_t q = off[v]; q < off[v + 1]; ++q) {
                if (!(diag[col[q]] > 0.0)) val[q] = 0.0;
                sabs += std::fabs(val[q]);
            }
            bmax = std::max(bmax, sabs * d0inv[v]);
        }
        if (!(bmax > 0.0)) fail(SEM_EINVAL, "sem_set_coarse: the coarse operator is zero");
        C->b = bmax;
        C->a = frac * bmax;
        C->n_coarse = 0;
        for (int64_t v = 0; v < C->nvert; ++v) C->n_coarse += diag[v] > 0.0;
        C->nnz = (int64_t)col.size();
        C->a_off = cmalloc<int32_t>(C, off.size());
        C->a_col = cmalloc<int32_t>(C, std::max<size_t>(col.size(), 1));
        C->a_val = cmalloc<double>(C, std::max<size_t>(val.size(), 1));
        C->d0inv = cmalloc<double>(C, d0inv.size());
        SEM_HIP(hipMemcpyAsync(C->a_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s));
        if (!col.empty()) {
            SEM_HIP(hipMemcpyAsync(C->a_col, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, s));
            SEM_HIP(hipMemcpyAsync(C->a_val, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, s));
        }
        SEM_HIP(hipMemcpyAsync(C->d0inv, d0inv.data(), sizeof(double) * d0inv.size(), hipMemcpyHostToDevice, s));
        // Chebyshev coefficients
        const double theta = 0.5 * (C->b + C->a), delta = 0.5 * (C->b - C->a), sigma = theta / delta;
        C->inv_theta = 1.0 / theta;
        double rho = 1.0 / sigma;
        C->c1.resize(k);
        C->c2.resize(k);
        for (int j = 0; j < k; ++j) {
            const double rho_new = 1.0 / (2.0 * sigma - rho);
            C->c1[j] = rho_new * rho;
            C->c2[j] = 2.0 * rho_new / delta;
            rho = rho_new;
        }
        C->r0 = cmalloc<double>(C, C->nvert);
        C->z0 = cmalloc<double>(C, C->nvert);
        C->res = cmalloc<double>(C, C->nvert);
        C->d = cmalloc<double>(C, C->nvert);
        C->tmp = cmalloc<double>(C, C->nvert);
        C->partial8 = cmalloc<double>(C, (size_t)E * 8);
        C->dot_blocks = cgrid(C->nvert * 8, kMaxCoarseDotBlocks);
        SEM_HIP(hipMemsetAsync(C->z0, 0, sizeof(double) * C->nvert, s));
        SEM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        coarse_free(C);
        throw;
    }
    return C;
}

// launches F<N> for the mesh's order
#define SEM_COARSE_ORDER_SWITCH(N, CALL)                                                                  \
    switch (N) {                                                                                       \
    case 1: CALL(1); break;  case 2: CALL(2); break;   case 3: CALL(3); break;   case 4: CALL(4); break;  \
    case 5: CALL(5); break;  case 6: CALL(6); break;   case 7: CALL(7); break;   case 8: CALL(8); break;  \
    case 9: CALL(9); break;  case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break; \
    default: fail(SEM_EUNSUPPORTED, "coarse term: order out of range");                               \
    }

static int elem_blocks(int64_t E) { return (int)std::max<int64_t>(1, std::min<int64_t>((E + 3) / 4, 8192)); }

template <typename T>
int coarse_update(sem_mesh *m, T *r, const T *w, const T *inv, const PcgState *st, double *partial, bool with_rz,
                  hipStream_t s)
{
    CoarseSpace *C = m->coarse;
    const int64_t E = m->h.E;
    const int blocks = elem_blocks(E);
    const int rz = with_rz ? 1 : 0;
#define SEM_UPD(n)                                                                                              \
    hipLaunchKernelGGL((update_restrict_kernel<T, n>), dim3(blocks), dim3(256), 0, s, E, st, r, w, inv, m->mult, \
                       C->qw, partial, C->partial8, rz)
    SEM_COARSE_ORDER_SWITCH(m->h.N, SEM_UPD)
#undef SEM_UPD
    SEM_HIP(hipGetLastError());
    return blocks;
}
template int coarse_update<double>(sem_mesh *, double *, const double *, const double *, const PcgState *, double *,
                                   bool, hipStream_t);
template int coarse_update<float>(sem_mesh *, float *, const float *, const float *, const PcgState *, double *,
                                  bool, hipStream_t);

static int64_t round32(int64_t n) { return (n + 31) / 32 * 32; }

int64_t coarse_work_doubles(const CoarseSpace *C, int64_t E)
{
    return round32(E * 8) + 5 * round32(C->nvert) + round32(2 * (int64_t)C->dot_blocks) + 32;
}

CoarseWork coarse_work_carve(const CoarseSpace *C, int64_t E, double *base)
{
    CoarseWork W;
    double *q = base;
    auto take = [&](int64_t n) {
        double *r = q;
        q += round32(n);
        return r;
    };
    W.partial8 = take(E * 8);
    W.r0 = take(C->nvert);
    W.z0 = take(C->nvert);
    W.res = take(C->nvert);
    W.d = take(C->nvert);
    W.tmp = take(C->nvert);
    W.dot = take(2 * (int64_t)C->dot_blocks);
    W.rz = take(1);
    return W;
}

CoarseWork coarse_work_own(const CoarseSpace *C)
{
    CoarseWork W;
    W.partial8 = C->partial8;
    W.r0 = C->r0;
    W.z0 = C->z0;
    W.res = C->res;
    W.d = C->d;
    W.tmp = C->tmp;
    W.dot = nullptr;
    W.rz = nullptr;
    return W;
}

template <typename T>
void coarse_restrict_w(sem_mesh *m, const CoarseWork &W, const T *r, const T *inv, hipStream_t s)
{
    CoarseSpace *C = m->coarse;
    const int64_t E = m->h.E;
#define SEM_RES(n)                                                                                                  \
    hipLaunchKernelGGL((restrict_elem_kernel<T, n>), dim3(elem_blocks(E)), dim3(256), 0, s, E, r, m->mult, inv, \
                       C->qw, W.partial8)
    SEM_COARSE_ORDER_SWITCH(m->h.N, SEM_RES)
#undef SEM_RES
    SEM_HIP(hipGetLastError());
}
template void coarse_restrict_w<double>(sem_mesh *, const CoarseWork &, const double *, const double *, hipStream_t);
template void coarse_restrict_w<float>(sem_mesh *, const CoarseWork &, const float *, const float *, hipStream_t);

template <typename T>
void coarse_restrict(sem_mesh *m, const T *r, const T *inv, hipStream_t s)
{
    coarse_restrict_w<T>(m, coarse_work_own(m->coarse), r, inv, s);
}
template void coarse_restrict<double>(sem_mesh *, const double *, const double *, hipStream_t);
template void coarse_restrict<float>(sem_mesh *, const float *, const float *, hipStream_t);

int coarse_solve_w(sem_mesh *m, const CoarseWork &W, double *dot_pairs, const PcgState *st, hipStream_t s)
{
    CoarseSpace *C = m->coarse;
    const int64_t nv = C->nvert;
    hipLaunchKernelGGL(restrict_vert_kernel, dim3(cgrid(nv, 4096)), dim3(256), 0, s, nv, C->v_off, C->v_idx,
                       W.partial8, C->d0inv, C->inv_theta, W.r0, W.z0, W.res, W.d, st);
    SEM_HIP(hipGetLastError());
    double *din = W.d, *dout = W.tmp;
    for (int j = 0; j < C->k; ++j) {
        if (j + 1 < C->k) {
            hipLaunchKernelGGL(cheb_kernel<false>, dim3(C->dot_blocks), dim3(256), 0, s, nv, C->a_off, C->a_col,
                               C->a_val, C->c1[j], C->c2[j], C->d0inv, din, dout, W.z0, W.res, W.r0, nullptr, st);
            std::swap(din, dout);
        } else {
            hipLaunchKernelGGL(cheb_kernel<true>, dim3(C->dot_blocks), dim3(256), 0, s, nv, C->a_off, C->a_col,
                               C->a_val, C->c1[j], C->c2[j], C->d0inv, din, dout, W.z0, W.res, W.r0, dot_pairs,
                               st);
        }
    }
    SEM_HIP(hipGetLastError());
    return C->dot_blocks;
}

int coarse_solve(sem_mesh *m, double *dot_pairs, const PcgState *st, hipStream_t s)
{
    return coarse_solve_w(m, coarse_work_own(m->coarse), dot_pairs, st, s);
}

void coarse_prolong_w(sem_mesh *m, const CoarseWork &W, double *z, bool add, hipStream_t s)
{
    CoarseSpace *C = m->coarse;
    const int64_t nL = m->h.nL;
    if (add)
        hipLaunchKernelGGL((prolong_kernel<true, double>), dim3(vec_blocks(nL)), dim3(256), 0, s, m->h.E, m->h.N + 1,
                           C->evert, W.z0, C->qw, m->inv64, z);
    else
        hipLaunchKernelGGL((prolong_kernel<false, double>), dim3(vec_blocks(nL)), dim3(256), 0, s, m->h.E,
                           m->h.N + 1, C->evert, W.z0, C->qw, m->inv64, z);
    SEM_HIP(hipGetLastError());
}

void coarse_prolong_w32(sem_mesh *m, const CoarseWork &W, float *z, hipStream_t s)
{
    CoarseSpace *C = m->coarse;
    const int64_t nL = m->h.nL;
    hipLaunchKernelGGL((prolong_kernel<false, float>), dim3(vec_blocks(nL)), dim3(256), 0, s, m->h.E, m->h.N + 1,
                       C->evert, W.z0, C->qw, m->inv64, z);
    SEM_HIP(hipGetLastError());
}

void coarse_prolong_add(sem_mesh *m, double *z, hipStream_t s)
{
    coarse_prolong_w(m, coarse_work_own(m->coarse), z, true, s);
}

void launch_jacobi(int64_t n, const double *inv, const double *r, double *z, hipStream_t s)
{
    hipLaunchKernelGGL(jacobi_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, inv, r, z);
    SEM_HIP(hipGetLastError());
}

}  // namespace sem
