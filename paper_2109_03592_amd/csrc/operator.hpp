// operator.hpp -- device building blocks shared by the single-mesh and the
// batched kernels: fixed-order block reductions, the constant table of GLL
// derivative matrices and the Algorithm 1 operator on one tile of elements.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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
// Streaming accesses: data read or written once per launch bypass the caches
// (non-temporal), which keeps them from evicting what is reused.
template <typename T>
__device__ inline T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ inline void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }
// pairs go through the compiler's native two-element vectors
typedef double native_double2 __attribute__((ext_vector_type(2)));
typedef float native_float2 __attribute__((ext_vector_type(2)));
template <>
__device__ inline double2 ld_stream(const double2 *p)
{
    const native_double2 v = __builtin_nontemporal_load(reinterpret_cast<const native_double2 *>(p));
    return double2(v.x, v.y);
}
template <>
__device__ inline float2 ld_stream(const float2 *p)
{
    const native_float2 v = __builtin_nontemporal_load(reinterpret_cast<const native_float2 *>(p));
    return float2(v.x, v.y);
}
template <>
__device__ inline void st_stream(double2 v, double2 *p)
{
    native_double2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<native_double2 *>(p));
}
template <>
__device__ inline void st_stream(float2 v, float2 *p)
{
    native_float2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<native_float2 *>(p));
}

// ---------------------------------------------------------------------------
// Direct-stiffness summation of one global id t of a plan (offsets `off` into
// local indices `idx`, every id has at least one copy): ids below n_sum get
// the sum of their copies, added in ascending local index starting from 0,
// written back to every copy; the other ids are Dirichlet ids whose copies
// are set to 0.  Copies are loaded four at a time without branches --
// positions past the id's last copy re-read that copy -- so the index loads,
// then the value loads, of a face id (2 copies) or an edge id (4) are in
// flight together; a vertex id (8) takes a second group.
template <typename T>
__device__ inline void gs_id(int64_t t, int64_t n_sum, const int32_t *__restrict__ off,
                             const int32_t *__restrict__ idx, T *__restrict__ v)
{
    const int32_t q0 = ld_stream(off + t), q1 = ld_stream(off + t + 1);
    const int32_t last = q1 - 1, cnt = q1 - q0;
    int32_t ix[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) ix[c] = idx[min(q0 + c, last)];
    if (cnt > 4) {
#pragma unroll
        for (int c = 4; c < 8; ++c) ix[c] = idx[min(q0 + c, last)];
    }
    if (t < n_sum) {
        T val[8];
#pragma unroll
        for (int c = 0; c < 4; ++c) val[c] = v[ix[c]];
        T s = T(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) s = c < cnt ? s + val[c] : s;
        if (cnt > 4) {
#pragma unroll
            for (int c = 4; c < 8; ++c) val[c] = v[ix[c]];
#pragma unroll
            for (int c = 4; c < 8; ++c) s = c < cnt ? s + val[c] : s;
            for (int32_t q = q0 + 8; q < q1; ++q) s += v[idx[q]];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < cnt) v[ix[c]] = s;
        for (int32_t q = q0 + 8; q < q1; ++q) v[idx[q]] = s;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < cnt) v[ix[c]] = T(0);
        for (int32_t q = q0 + 8; q < q1; ++q) v[idx[q]] = T(0);
    }
}

// Node t of the face lattice (enumerated as GsLattice describes): its
// copies summed from 0 in ascending local index and written back, 0 on a
// Dirichlet node, an unmasked single copy left alone.  Requires
// t < L.n_nodes.
template <typename T>
__device__ inline void gs_lattice_node(const GsLattice &L, int64_t t, T *__restrict__ v)
{
    unsigned X, Y, Z;
    gs_lattice_pos(L, (unsigned)t, X, Y, Z);
    const LatticeCopies c = gs_lattice_copies(L, X, Y, Z);
    const AxisCopies &cx = c.cx, &cy = c.cy, &cz = c.cz;
    const bool masked = c.masked;
    if (!masked && c.cnt < 2) return;
    if (masked) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
            if (qz < cz.c && qy < cy.c && qx < cx.c) v[c.a[q]] = T(0);
        }
        return;
    }
    T val[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
        val[q] = (qz < cz.c && qy < cy.c && qx < cx.c) ? v[c.a[q]] : T(0);
    }
    T s = T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
        if (qz < cz.c && qy < cy.c && qx < cx.c) s = s + val[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
        if (qz < cz.c && qy < cy.c && qx < cx.c) v[c.a[q]] = s;
    }
}

// ---------------------------------------------------------------------------
// GLL derivative matrices of every order in constant memory: the uniform
// D[k][l] of the t-direction become scalar loads, the per-lane rows vector
// loads.  Order N lives at offset sum_{n<N} (n+1)^2.
// (static: every code object that includes this header holds and fills its
// own copy)
static __constant__ double c_D64[kDTableSize];
static __constant__ float c_D32[kDTableSize];

template <typename T>
__device__ inline const T *dtable(int N);
template <>
__device__ inline const double *dtable<double>(int N) { return c_D64 + dtable_offset(N); }
template <>
__device__ inline const float *dtable<float>(int N) { return c_D32 + dtable_offset(N); }

// ---------------------------------------------------------------------------
// Local operator (Algorithm 1, h1 = 1) on one tile of `epw` elements.  Lane
// (el, i, j) owns column (i,j) of element tile*epw + el.  MODE 0: w = A_L u.
// MODE 1: also accumulates u.w into `dot`.  MODE 2 (CG): first x <- x +
// alpha*p (the previous iteration's step) and p <- invdiag*r + beta*p, then
// w = A_L p and p.w into `dot`.  The caller provides the
// LDS slot of this lane's element (3 (N+1)^3 values), the lane's rows of D
// and of D^T, and ends the tile with a barrier before LDS is reused.
template <typename T, int N>
struct LaneRows {
    static constexpr int P = N + 1;
    // at high order the D^T rows (and above that the D rows too) come from
    // an LDS copy of D instead of VGPRs (keeps the FP64 kernels at two waves
    // per SIMD)
    static constexpr bool kDtLds = sizeof(T) == 8 ? N >= 8 : N >= 11;
    static constexpr bool kDLds = sizeof(T) == 8 ? N >= 10 : false;
    static constexpr int kDtLen = kDtLds ? 1 : P;
    static constexpr int kDLen = kDLds ? 1 : P;
    T Di_[kDLen], Dj_[kDLen], Dti_[kDtLen], Dtj_[kDtLen];
    const T *sD;
    int ci, cj;
    // sDbuf: P*P values of LDS (used when kDtLds); the caller's first barrier
    // after load() publishes it
    __device__ inline void load(const T *__restrict__ D, int i, int j, T *sDbuf)
    {
        if constexpr (!kDLds) {
#pragma unroll
            for (int l = 0; l < P; ++l) {
                Di_[l] = D[i * P + l];
                Dj_[l] = D[j * P + l];
            }
        }
        if constexpr (kDtLds) {
            for (int q = threadIdx.x; q < P * P; q += blockDim.x) sDbuf[q] = D[q];
            sD = sDbuf;
        } else {
#pragma unroll
            for (int l = 0; l < P; ++l) {
                Dti_[l] = D[l * P + i];
                Dtj_[l] = D[l * P + j];
            }
            sD = nullptr;
        }
        ci = i;
        cj = j;
    }
    __device__ inline T di(int l) const
    {
        if constexpr (kDLds) return sD[ci * P + l];
        else return Di_[l];
    }
    __device__ inline T dj(int l) const
    {
        if constexpr (kDLds) return sD[cj * P + l];
        else return Dj_[l];
    }
    // uniform D[k][l] of the t-direction: constant memory (scalar loads), or
    // the LDS copy where the constant table would not fit the SGPRs
    static constexpr bool kTLds = kDLds;
    __device__ inline T dk(const T *__restrict__ D, int k, int l) const
    {
        if constexpr (kTLds) return sD[k * P + l];
        else return D[k * P + l];
    }
    __device__ inline T dti(int l) const
    {
        if constexpr (kDtLds) return sD[l * P + ci];
        else return Dti_[l];
    }
    __device__ inline T dtj(int l) const
    {
        if constexpr (kDtLds) return sD[l * P + cj];
        else return Dtj_[l];
    }
};

// LDS values a kernel reserves for LaneRows::load
template <typename T, int N>
constexpr int lane_rows_lds() { return LaneRows<T, N>::kDtLds ? (N + 1) * (N + 1) : 1; }

// HELM: Helmholtz form -- the three products of the combine step are scaled
// by h1 at the point (Algorithm 1's h1) and h2*B*u is added to the output
// (the h2 term of Eq. 4); h2b holds h2*B per point.
// MODE 3 (CG with the coarse term of Eq. 6): MODE 2 with the coarse
// correction added to the preconditioned residual, p <- invdiag*r +
// sum_c phi_c zcl[c] + beta*p at live nodes (invdiag > 0), phi_c the
// trilinear hat of corner c (c = cx + 2cy + 4cz) with 1-D weights cq[side][i]
// and zcl the coarse solution at the element's corners (staged in LDS by the
// caller).
// MODE 4 (CG with a preconditioned residual given, e.g. by the Schwarz local
// solves): p <- in + beta*p.  MODE 5: MODE 4 plus the coarse correction.
// addv (MODE 2): a correction added to invdiag*r + beta*p at every node, the
// coarse term a batched slot has prolonged beforehand (0 on masked nodes).
// Sink: with a callable other than NoSink, each output w(i,j,k) of the lane
// goes to sink(k, w) as it is formed instead of to `out`, and the tile ends
// without the trailing barrier (the caller's epilogue barrier orders the LDS
// reuse).
struct NoSink {
    template <typename T>
    __device__ void operator()(int, T) const {}
};
template <typename T, int N, int MODE, bool HELM = false, typename Sink = NoSink>
__device__ inline void ax_tile(const LaneRows<T, N> &R, const T *__restrict__ D, T *su, int64_t e, bool active,
                               bool inblk, int i, int j, const T *__restrict__ G, const T *__restrict__ in,
                               T *__restrict__ out, const T *__restrict__ invdiag, T *__restrict__ p, T beta,
                               T *__restrict__ x, T alpha, double &dot, const T *__restrict__ h1 = nullptr,
                               const T *__restrict__ h2b = nullptr, const double *zcl = nullptr,
                               const double *__restrict__ cq = nullptr, const Sink &sink = Sink(),
                               const T *__restrict__ addv = nullptr)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    T *sr = su + P3;
    T *ss = sr + P3;
    const int ij = i + P * j;
    const int64_t eb = (active ? e : 0) * P3;
    T uc[P];
    constexpr bool kCoarse = MODE == 3 || MODE == 5;
    if (MODE >= 2) {
        // coarse correction of this column (FP64): bilinear in (i,j) per t-side
        double cs0 = 0, cs1 = 0;
        if (kCoarse && active) {
            double zc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) zc[c] = zcl[c];
            const double ai0 = cq[i], ai1 = cq[P + i], aj0 = cq[j], aj1 = cq[P + j];
            cs0 = aj0 * (ai0 * zc[0] + ai1 * zc[1]) + aj1 * (ai0 * zc[2] + ai1 * zc[3]);
            cs1 = aj0 * (ai0 * zc[4] + ai1 * zc[5]) + aj1 * (ai0 * zc[6] + ai1 * zc[7]);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T v = 0;
            if (active) {
                const int64_t o = eb + ij + k * P2;
                const T pold = ld_stream(p + o);
                // the previous iteration's x step, deferred to here where p is read anyway
                st_stream(ld_stream(x + o) + alpha * pold, x + o);
                if (MODE >= 4) {
                    v = ld_stream(in + o) + beta * pold;
                    if (kCoarse && ld_stream(invdiag + o) > T(0)) v += (T)(cq[k] * cs0 + cq[P + k] * cs1);
                } else {
                    const T iv = ld_stream(invdiag + o);
                    v = iv * ld_stream(in + o) + beta * pold;
                    if (kCoarse && iv > T(0)) v += (T)(cq[k] * cs0 + cq[P + k] * cs1);
                    // MODE 2 with a precomputed correction (a batched slot's P z0)
                    if (MODE == 2 && addv) v += ld_stream(addv + o);
                }
                st_stream(v, p + o);
            }
            uc[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) uc[k] = active ? ld_stream(in + eb + ij + k * P2) : T(0);
    }
    if (inblk) {
#pragma unroll
        for (int k = 0; k < P; ++k) su[k * P2 + ij] = uc[k];
    }
    __syncthreads();

    const T *__restrict__ Ge = G + (active ? e : 0) * 6 * P3 + ij;
    T wt[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        T ur = 0, us = 0, ut = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            ur += R.di(l) * su[k * P2 + j * P + l];
            us += R.dj(l) * su[k * P2 + l * P + i];
            ut += R.dk(D, k, l) * uc[l];
        }
        T g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0, g6 = 0;
        if (active) {
            const T *g = Ge + k * P2;
            g1 = ld_stream(g + 0 * P3); g2 = ld_stream(g + 1 * P3); g3 = ld_stream(g + 2 * P3);
            g4 = ld_stream(g + 3 * P3); g5 = ld_stream(g + 4 * P3); g6 = ld_stream(g + 5 * P3);
        }
        T wr = g1 * ur + g4 * us + g5 * ut;
        T ws = g2 * us + g4 * ur + g6 * ut;
        wt[k] = g3 * ut + g5 * ur + g6 * us;
        if (HELM) {
            const T h = active ? ld_stream(h1 + eb + ij + k * P2) : T(0);
            wr *= h;
            ws *= h;
            wt[k] *= h;
        }
        if (inblk) {
            sr[k * P2 + ij] = wr;
            ss[k * P2 + ij] = ws;
        }
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < P; ++k) {
        T acc = 0;
#pragma unroll
        for (int l = 0; l < P; ++l)
            acc += R.dti(l) * sr[k * P2 + j * P + l] + R.dtj(l) * ss[k * P2 + l * P + i] + R.dk(D, l, k) * wt[l];
        if (HELM && active) acc += ld_stream(h2b + eb + ij + k * P2) * uc[k];
        constexpr bool kSink = !std::is_same<Sink, NoSink>::value;
        if constexpr (kSink) sink(k, acc);
        else if (active) st_stream(acc, out + eb + ij + k * P2);
        if (MODE != 0) dot += (double)uc[k] * (double)acc;
    }
    if constexpr (std::is_same<Sink, NoSink>::value) __syncthreads();  // the LDS slot is rewritten by the next tile
}


// Which tile an operator launch runs (mode 0-2, values of value_bytes).  At
// high order the whole-element tile's LDS (3 (N+1)^3 values per element)
// leaves room for one or two workgroups per compute unit, so from order 8 on
// the operator runs plane by plane; at N = 7 the plane tile is the faster one
// for the FP64 plain operator (modes 0, 1) only.
constexpr bool plane_tile_use(int N, int mode, int value_bytes)
{
    return mode <= 2 && (N >= 8 || (N == 7 && mode <= 1 && value_bytes == 8));
}
template <typename T, int N, int MODE>
constexpr bool plane_tile() { return plane_tile_use(N, MODE, (int)sizeof(T)); }

// The local operator tile plane by plane (MODE 0-2; the same operator as
// ax_tile).  LDS holds three planes of the element -- u(., ., k) and the two
// in-plane fluxes -- instead of three whole elements: per plane k the lanes
// stage u(i,j,k), form the r-, s- and t-derivatives and the fluxes of the
// combine step, stage the r- and s-fluxes, and apply the in-plane transposed
// derivatives; the t-direction part of the transposed derivative is
// accumulated in registers as the planes pass.  Two barriers per plane; the
// plane loop is not unrolled (unrolled, the compiler hoists every plane's
// factor loads above the barriers and spills); instead the factors of the
// next plane are loaded one plane ahead.  The caller provides the LDS
// slot of this lane's element (3 (N+1)^2 values at least).  Sink as for
// ax_tile: outputs go to sink(k, w) in ascending k once all planes have
// passed, and the tile then ends without the trailing barrier.  addv as for
// ax_tile (MODE 2).
template <typename T, int N, int MODE, bool HELM = false, typename Sink = NoSink>
__device__ inline void ax_tile_planes(const LaneRows<T, N> &R, const T *__restrict__ D, T *sp, int64_t e,
                                      bool active, bool inblk, int i, int j, const T *__restrict__ G,
                                      const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ invdiag,
                                      T *__restrict__ p, T beta, T *__restrict__ x, T alpha, double &dot,
                                      const T *__restrict__ h1 = nullptr, const T *__restrict__ h2b = nullptr,
                                      const Sink &sink = Sink(), const T *__restrict__ addv = nullptr)
{
    static_assert(MODE <= 2, "plane tile: the plain and CG modes");
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    T *su = sp;
    T *sr = sp + P2;
    T *ss = sr + P2;
    const int ij = i + P * j;
    const int64_t eb = (active ? e : 0) * P3;
    T uc[P];
    if (MODE >= 2) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T v = 0;
            if (active) {
                const int64_t o = eb + ij + k * P2;
                const T pold = ld_stream(p + o);
                // the previous iteration's x step, deferred to here where p is read anyway
                st_stream(ld_stream(x + o) + alpha * pold, x + o);
                v = ld_stream(invdiag + o) * ld_stream(in + o) + beta * pold;
                if (MODE == 2 && addv) v += ld_stream(addv + o);  // as ax_tile's addv
                st_stream(v, p + o);
            }
            uc[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) uc[k] = active ? ld_stream(in + eb + ij + k * P2) : T(0);
    }
    const T *__restrict__ Ge = G + (active ? e : 0) * 6 * P3 + ij;
    T acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = 0;
    // the factors of plane k + 1 are loaded while plane k is worked on, so
    // that their latency overlaps a whole plane's barriers and LDS products
    T gn[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) gn[c] = active ? ld_stream(Ge + c * P3) : T(0);
#pragma unroll 1
    for (int k = 0; k < P; ++k) {
        const T g1 = gn[0], g2 = gn[1], g3 = gn[2], g4 = gn[3], g5 = gn[4], g6 = gn[5];
        if (active && k + 1 < P) {
            const T *g = Ge + (k + 1) * P2;
#pragma unroll
            for (int c = 0; c < 6; ++c) gn[c] = ld_stream(g + c * P3);
        }
        T uk = uc[0];
#pragma unroll
        for (int l = 1; l < P; ++l) uk = l == k ? uc[l] : uk;
        if (inblk) su[ij] = uk;
        __syncthreads();
        T ur = 0, us = 0, ut = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            ur += R.di(l) * su[j * P + l];
            us += R.dj(l) * su[l * P + i];
            ut += R.dk(D, k, l) * uc[l];
        }
        T wr = g1 * ur + g4 * us + g5 * ut;
        T ws = g2 * us + g4 * ur + g6 * ut;
        T wt = g3 * ut + g5 * ur + g6 * us;
        if (HELM) {
            const T h = active ? ld_stream(h1 + eb + ij + k * P2) : T(0);
            wr *= h;
            ws *= h;
            wt *= h;
        }
        if (inblk) {
            sr[ij] = wr;
            ss[ij] = ws;
        }
        __syncthreads();
        T a = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) a += R.dti(l) * sr[j * P + l] + R.dtj(l) * ss[l * P + i];
        // D^T in t: plane k's flux reaches every output plane kk with D[k][kk]
#pragma unroll
        for (int kk = 0; kk < P; ++kk) acc[kk] += R.dk(D, k, kk) * wt + (kk == k ? a : T(0));
    }
    constexpr bool kSink = !std::is_same<Sink, NoSink>::value;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        T v = acc[k];
        if (HELM && active) v += ld_stream(h2b + eb + ij + k * P2) * uc[k];
        if constexpr (kSink) sink(k, v);
        else if (active) st_stream(v, out + eb + ij + k * P2);
        if (MODE != 0) dot += (double)uc[k] * (double)v;
    }
    if constexpr (!kSink) __syncthreads();  // the next tile rewrites the planes
}

}  // namespace sem
