// schwarz.hip -- the sum over overlapping local subdomains of Eq. 6 on the
// GPU:  z = sum_k R_k^T A_k^{-1} R_k r.
//
//  * Subdomain k is element k extended by one node layer into each
//    neighbour that exists (also across periodic faces); nodes on Dirichlet
//    faces are not unknowns.  Its extended index range per direction is
//    lo .. lo+count-1 within -1 .. N+1.
//  * A_k is separable (the fast-diagonalisation form): with the 1-D GLL
//    stiffness A_d and lumped mass B_d of the element's mean edge length in
//    direction d, assembled on the element and its existing neighbours (same
//    length) and restricted to the kept indices,
//        A_k = B_t x B_s x A_r + B_t x A_s x B_r + A_t x B_s x B_r.
//    With S_d^T B_d S_d = I and S_d^T A_d S_d = diag(lam_d),
//        A_k^{-1} = (S_t x S_s x S_r) diag(1/(lam_r + lam_s + lam_t)) (S_t x S_s x S_r)^T,
//    six 1-D contractions per element (fdm_kernel, one workgroup per
//    element, the element in LDS).  The 1-D factors are computed on the host
//    and shared by all elements with the same (length, side kinds).
//  * The local solutions are summed into every node they cover
//    (assemble_kernel): a node receives the contributions of all extended
//    elements that hold it, added in ascending (unwrapped) element order per
//    direction, so every copy of a shared node gets the same bits.
//  * <r, z> for CG is taken inside fdm_kernel as sum_k (R_k r) . y_k, i.e. the
//    sum over modes of yhat^2 / (lam_r + lam_s + lam_t), yhat = S^T R_k r.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "operator.hpp"
#include "schwarz.hpp"

namespace sem {

struct Lattice {
    int nel[3];
    int periodic[3];
    int dirichlet;  // bit 2d (2d+1): Dirichlet on the low (high) face of axis d
};

__host__ __device__ inline bool has_left(const Lattice &L, int d, int pos) { return pos > 0 || L.periodic[d]; }
__host__ __device__ inline bool has_right(const Lattice &L, int d, int pos)
{
    return pos < L.nel[d] - 1 || L.periodic[d];
}
// ---------------------------------------------------------------------------
// device kernels

// One workgroup per element (persistent walk); lane (l0, l1) < n^2 owns one
// line of the extended element in every contraction stage.  Each stage runs
// over the contracted index (inputs from LDS, one row of S per step) and
// keeps the line's n outputs in registers.  <R_k r, y_k> equals
// sum over modes of yhat^2 / (lam_r + lam_s + lam_t), yhat = S^T R_k r, and is
// taken where the scaling is applied.
template <int N>
__device__ inline void fdm_line(const double *__restrict__ Sd, const double *__restrict__ in, int in_stride,
                                double (&acc)[N + 3], bool transpose)
{
    constexpr int n = N + 3;
#pragma unroll
    for (int b = 0; b < n; ++b) acc[b] = 0.0;
#pragma unroll 2
    for (int a = 0; a < n; ++a) {
        const double x = in[a * in_stride];
        // transpose: acc[b] += S[a][b] x (S^T applied); else acc[b] += S[b][a] x
#pragma unroll
        for (int b = 0; b < n; ++b) acc[b] += (transpose ? Sd[a * n + b] : Sd[b * n + a]) * x;
    }
}

// workgroup of the local solves: the (N+3)^2 lines rounded up to wavefronts
template <int N>
constexpr int kFdmThreads = ((N + 3) * (N + 3) + 63) / 64 * 64;

template <int N>
__global__ __launch_bounds__(256) void fdm_kernel(int64_t E, Lattice L, const double *__restrict__ r,
                                                  const int32_t *__restrict__ tidx,
                                                  const double *__restrict__ table,
                                                  const int32_t *__restrict__ meta, double *__restrict__ zext,
                                                  double *__restrict__ partial, const PcgState *__restrict__ st)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    constexpr int n = N + 3, n2 = n * n, n3 = n2 * n, TE = n2 + n;
    if (st && st->done) return;
    __shared__ double U[n3], V[n3];
    const int tid = threadIdx.x;
    const bool line = tid < n2;
    const int l0 = tid % n, l1 = tid / n;
    double dot = 0.0;
    double acc[n];
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int ei = (int)e;
        const int pos[3] = {ei % L.nel[0], (ei / L.nel[0]) % L.nel[1], ei / (L.nel[0] * L.nel[1])};
        // the element's 1-D factors: workgroup-uniform addresses (scalar loads)
        const double *S[3];
        int lo[3], cnt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int t = tidx[e * 3 + d];
            S[d] = table + (int64_t)t * TE;
            lo[d] = meta[2 * t];
            cnt[d] = meta[2 * t + 1];
        }
        const double *Lm[3] = {S[0] + n2, S[1] + n2, S[2] + n2};
        // R_k r: extended node (a, b, c) from the element or a neighbour (r is
        // continuous: any copy of a node holds its value); 0 beyond the kept
        // range.  All of a lane's loads are issued together, out-of-range ones
        // from the element's first node.
        constexpr int kIt = (n3 + kFdmThreads<N> - 1) / kFdmThreads<N>;
        double gv[kIt];
        bool gk[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int q = tid + it * kFdmThreads<N>;
            const int a[3] = {q % n, (q / n) % n, q / n2};
            bool ok = q < n3 && a[0] < cnt[0] && a[1] < cnt[1] && a[2] < cnt[2];
            int ep[3], loc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int x = lo[d] + a[d];
                int p2 = pos[d], lc = x;
                if (x == -1) { p2 -= 1; lc = N - 1; }
                else if (x == N + 1) { p2 += 1; lc = 1; }
                if (p2 < 0) p2 += L.nel[d];
                if (p2 >= L.nel[d]) p2 -= L.nel[d];
                ok = ok && p2 >= 0 && p2 < L.nel[d] && lc >= 0 && lc <= N;
                ep[d] = p2;
                loc[d] = lc;
            }
            const int64_t e2 = ep[0] + (int64_t)L.nel[0] * (ep[1] + (int64_t)L.nel[1] * ep[2]);
            gv[it] = r[ok ? e2 * P3 + loc[0] + P * loc[1] + P2 * loc[2] : e * P3];
            gk[it] = ok;
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int q = tid + it * kFdmThreads<N>;
            if (q < n3) U[q] = gk[it] ? gv[it] : 0.0;
        }
        __syncthreads();
        // 1: along r, S_r^T (line s = l0, t = l1): U -> V
        if (line) {
            fdm_line<N>(S[0], U + l1 * n2 + l0 * n, 1, acc, true);
#pragma unroll
            for (int b = 0; b < n; ++b) V[l1 * n2 + l0 * n + b] = acc[b];
        }
        __syncthreads();
        // 2: along s, S_s^T (line r' = l0, t = l1): V -> U
        if (line) {
            fdm_line<N>(S[1], V + l1 * n2 + l0, n, acc, true);
#pragma unroll
            for (int b = 0; b < n; ++b) U[l1 * n2 + b * n + l0] = acc[b];
        }
        __syncthreads();
        // 3: along t, S_t^T, scaling, S_t (line r' = l0, s' = l1): U -> V -> V
        if (line) {
            fdm_line<N>(S[2], U + l1 * n + l0, n2, acc, true);
            const double lrs = Lm[0][l0] + Lm[1][l1];
#pragma unroll
            for (int b = 0; b < n; ++b) {
                const double den = lrs + Lm[2][b];
                const double y = den > 0.0 ? acc[b] / den : 0.0;
                dot += acc[b] * y;
                V[b * n2 + l1 * n + l0] = y;
            }
            fdm_line<N>(S[2], V + l1 * n + l0, n2, acc, false);
#pragma unroll
            for (int k = 0; k < n; ++k) V[k * n2 + l1 * n + l0] = acc[k];
        }
        __syncthreads();
        // 4: along s, S_s (line r = l0, t = l1): V -> U
        if (line) {
            fdm_line<N>(S[1], V + l1 * n2 + l0, n, acc, false);
#pragma unroll
            for (int j = 0; j < n; ++j) U[l1 * n2 + j * n + l0] = acc[j];
        }
        __syncthreads();
        // 5: along r, S_r (line s = l0, t = l1): U -> V
        if (line) {
            fdm_line<N>(S[0], U + l1 * n2 + l0 * n, 1, acc, false);
#pragma unroll
            for (int i = 0; i < n; ++i) V[l1 * n2 + l0 * n + i] = acc[i];
        }
        __syncthreads();
        for (int q = tid; q < n3; q += kFdmThreads<N>) st_stream(V[q], zext + e * n3 + q);
        __syncthreads();
    }
    if (partial) {
        double p[2] = {0.0, dot};
        block_reduce_store<2>(p, partial, 2);
    }
}

// z at every local node: the sum of the extended solutions that hold it,
// 0 at Dirichlet nodes (invdiag 0).  Per direction a node of index idx is
// held by its element (offset 0) and, when idx <= 1 or idx >= N-1, by the
// neighbour on that side (N >= 3: at most two holders per direction, in
// ascending offset).  The eight candidates are loaded together, invalid ones
// from a clamped address, and summed in ascending order with selects; N = 2
// (a node of index 1 is held by both neighbours) takes the general loop.
template <int N>
__global__ __launch_bounds__(256) void assemble_kernel(int64_t E, Lattice L, const double *__restrict__ zext,
                                                       const double *__restrict__ inv, double *__restrict__ z,
                                                       const PcgState *__restrict__ st)
{
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    constexpr int n = N + 3, n2 = n * n, n3 = n2 * n;
    static_assert(N >= 2, "the overlap of one node layer needs N >= 2");
    if (st && st->done) return;
    const int64_t nL = E * P3;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nL; q += (int64_t)gridDim.x * blockDim.x) {
        const int ei = (int)(q / P3);
        const int rem = (int)(q - (int64_t)ei * P3);
        const int idx[3] = {rem % P, (rem / P) % P, rem / P2};
        const int pos[3] = {ei % L.nel[0], (ei / L.nel[0]) % L.nel[1], ei / (L.nel[0] * L.nel[1])};
        double s = 0.0;
        if constexpr (N >= 3) {
            // per direction: candidate t = 0, 1 (ascending offset): validity,
            // lattice position and position in that element's kept range
            bool ok[3][2];
            int el[3][2], ps[3][2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int lo_side = idx[d] <= 1, hi_side = idx[d] >= N - 1;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    // offsets: (-1, 0) near the low face, (0, +1) near the high face, (0, -) inside
                    const int delta = lo_side ? t - 1 : (hi_side ? t : 0);
                    bool v = lo_side || hi_side || t == 0;
                    const int ext = idx[d] - delta * N;
                    int p2 = pos[d] + delta;
                    if (p2 < 0) { v = v && L.periodic[d]; p2 += L.nel[d]; }
                    if (p2 >= L.nel[d]) { v = v && L.periodic[d]; p2 -= L.nel[d]; }
                    const bool left = p2 > 0 || L.periodic[d], right = p2 < L.nel[d] - 1 || L.periodic[d];
                    const int lo2 = left ? -1 : ((L.dirichlet >> (2 * d)) & 1);
                    const int hi2 = right ? N + 1 : (((L.dirichlet >> (2 * d + 1)) & 1) ? N - 1 : N);
                    ok[d][t] = v && ext >= lo2 && ext <= hi2;
                    el[d][t] = p2;
                    ps[d][t] = ext - lo2;
                }
            }
            double val[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int tx = c & 1, ty = (c >> 1) & 1, tz = c >> 2;
                const bool good = ok[0][tx] && ok[1][ty] && ok[2][tz];
                const int e2 = el[0][tx] + L.nel[0] * (el[1][ty] + L.nel[1] * el[2][tz]);
                const int64_t a = good ? (int64_t)e2 * n3 + ps[0][tx] + n * ps[1][ty] + n2 * ps[2][tz]
                                       : (int64_t)ei * n3;
                val[c] = zext[a];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int tx = c & 1, ty = (c >> 1) & 1, tz = c >> 2;
                const bool good = ok[0][tx] && ok[1][ty] && ok[2][tz];
                s = good ? s + val[c] : s;
            }
        } else {
            bool ok[3][3];
            int el[3][3], ps[3][3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int delta = t - 1;
                    const int ext = idx[d] - delta * N;
                    int p2 = pos[d] + delta;
                    bool v = ext >= -1 && ext <= N + 1;
                    if (p2 < 0) { v = v && L.periodic[d]; p2 += L.nel[d]; }
                    if (p2 >= L.nel[d]) { v = v && L.periodic[d]; p2 -= L.nel[d]; }
                    const bool left = p2 > 0 || L.periodic[d], right = p2 < L.nel[d] - 1 || L.periodic[d];
                    const int lo2 = left ? -1 : ((L.dirichlet >> (2 * d)) & 1);
                    const int hi2 = right ? N + 1 : (((L.dirichlet >> (2 * d + 1)) & 1) ? N - 1 : N);
                    ok[d][t] = v && ext >= lo2 && ext <= hi2;
                    el[d][t] = p2;
                    ps[d][t] = ext - lo2;
                }
            }
#pragma unroll
            for (int tz = 0; tz < 3; ++tz)
#pragma unroll
                for (int ty = 0; ty < 3; ++ty)
#pragma unroll
                    for (int tx = 0; tx < 3; ++tx) {
                        if (!(ok[0][tx] && ok[1][ty] && ok[2][tz])) continue;
                        const int e2 = el[0][tx] + L.nel[0] * (el[1][ty] + L.nel[1] * el[2][tz]);
                        s += zext[(int64_t)e2 * n3 + ps[0][tx] + n * ps[1][ty] + n2 * ps[2][tz]];
                    }
        }
        z[q] = ld_stream(inv + q) > 0.0 ? s : 0.0;
    }
}

// ---------------------------------------------------------------------------
// host: 1-D factors

// Eigen-decomposition of a symmetric n x n matrix (row-major) by cyclic
// Jacobi rotations: a = v diag(d) v^T, eigenvectors in the columns of v.
static void symmetric_eigen(std::vector<double> a, int n, std::vector<double> &v, std::vector<double> &d)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                const double x = a[(size_t)p * n + q] * a[(size_t)p * n + q];
                tot += x;
                if (p != q) off += x;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    d.resize(n);
    for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
}

void fdm_1d(int N, const std::vector<double> &xi, const std::vector<double> &w, const std::vector<double> &D,
            double ell, int left, int right, std::vector<double> &S, std::vector<double> &lam, int &lo, int &count)
{
    (void)xi;
    const int P = N + 1, M = 3 * N + 1;
    std::vector<double> Ke((size_t)P * P), K((size_t)M * M, 0.0), B(M, 0.0);
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += D[(size_t)q * P + a] * w[q] * D[(size_t)q * P + b];
            Ke[(size_t)a * P + b] = (2.0 / ell) * s;
        }
    const int parts[3] = {left == kSideInterior ? 0 : -1, 1, right == kSideInterior ? 2 : -1};
    for (int p : parts) {
        if (p < 0) continue;
        for (int a = 0; a < P; ++a) {
            for (int b = 0; b < P; ++b) K[(size_t)(p * N + a) * M + p * N + b] += Ke[(size_t)a * P + b];
            B[p * N + a] += 0.5 * ell * w[a];
        }
    }
    lo = left == kSideInterior ? -1 : (left == kSideNeumann ? 0 : 1);
    const int hi = right == kSideInterior ? N + 1 : (right == kSideNeumann ? N : N - 1);
    count = hi - lo + 1;
    const int n = count;
    std::vector<double> C((size_t)n * n), sb(n);
    for (int a = 0; a < n; ++a) sb[a] = 1.0 / std::sqrt(B[N + lo + a]);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) C[(size_t)a * n + b] = K[(size_t)(N + lo + a) * M + N + lo + b] * sb[a] * sb[b];
    std::vector<double> Q;
    symmetric_eigen(C, n, Q, lam);
    S.assign((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) S[(size_t)a * n + b] = Q[(size_t)a * n + b] * sb[a];
}

// ---------------------------------------------------------------------------
// host: set-up and launches

template <typename X>
static X *smalloc(SchwarzSpace *Z, size_t count)
{
    void *p = nullptr;
    SEM_HIP(hipMalloc(&p, std::max<size_t>(count * sizeof(X), 16)));
    Z->allocations.push_back(p);
    return static_cast<X *>(p);
}

void schwarz_free(SchwarzSpace *Z)
{
    if (!Z) return;
    for (void *p : Z->allocations) (void)hipFree(p);
    delete Z;
}

static Lattice lattice_of(const sem_mesh *m, int dirichlet)
{
    Lattice L{};
    for (int d = 0; d < 3; ++d) {
        L.nel[d] = m->h.nel[d];
        L.periodic[d] = m->h.periodic[d];
    }
    L.dirichlet = dirichlet;
    return L;
}

SchwarzSpace *schwarz_build(sem_mesh *m, hipStream_t s)
{
    const HostMesh &h = m->h;
    const int N = h.N, P = N + 1, n = N + 3;
    const int64_t E = h.E, P3 = (int64_t)P * P * P;
    if (E >= INT32_MAX) fail(SEM_EUNSUPPORTED, "sem_set_schwarz: too many elements");
    SchwarzSpace *Z = new SchwarzSpace();
    try {
        Z->n = n;
        int faces = h.desc.dirichlet_faces;
        if (faces < 0) {
            faces = 0;
            for (int d = 0; d < 3; ++d)
                if (!h.periodic[d]) faces |= 3 << (2 * d);
        }
        for (int d = 0; d < 3; ++d)
            if (h.periodic[d]) faces &= ~(3 << (2 * d));
        Z->dirichlet = faces;
        const Lattice L = lattice_of(m, faces);
        // element corner coordinates -> mean edge lengths
        HostMesh ch;
        sem_mesh_desc d = h.desc;
        d.vertices = h.vertices.empty() ? nullptr : h.vertices.data();
        build_host_coords(d, ch);
        const int64_t nL = ch.nL;
        auto X = [&](int64_t e, int i, int j, int k, int c) {
            return ch.xyz[(size_t)c * nL + e * P3 + i + P * (j + (int64_t)P * k)];
        };
        auto dist = [&](int64_t e, int i0, int j0, int k0, int i1, int j1, int k1) {
            const double dx = X(e, i1, j1, k1, 0) - X(e, i0, j0, k0, 0);
            const double dy = X(e, i1, j1, k1, 1) - X(e, i0, j0, k0, 1);
            const double dz = X(e, i1, j1, k1, 2) - X(e, i0, j0, k0, 2);
            return std::sqrt(dx * dx + dy * dy + dz * dz);
        };
        const int TE = n * n + n;
        std::map<std::tuple<double, int, int>, int32_t> index;
        std::vector<double> table;
        std::vector<int32_t> meta, tidx((size_t)E * 3);
        std::vector<double> S1, lam;
        for (int64_t e = 0; e < E; ++e) {
            const int pos[3] = {(int)(e % h.nel[0]), (int)((e / h.nel[0]) % h.nel[1]),
                                (int)(e / ((int64_t)h.nel[0] * h.nel[1]))};
            const int c[2] = {0, N};
            double ell[3] = {0.0, 0.0, 0.0};
            for (int a : c)
                for (int b : c) {
                    ell[0] += dist(e, 0, a, b, N, a, b);  // r-edges at (j, k) = (a, b)
                    ell[1] += dist(e, a, 0, b, a, N, b);
                    ell[2] += dist(e, a, b, 0, a, b, N);
                }
            for (int dd = 0; dd < 3; ++dd) {
                const double len = ell[dd] / 4.0;
                const int left = has_left(L, dd, pos[dd]) ? kSideInterior
                                 : ((faces >> (2 * dd)) & 1) ? kSideDirichlet : kSideNeumann;
                const int right = has_right(L, dd, pos[dd]) ? kSideInterior
                                  : ((faces >> (2 * dd + 1)) & 1) ? kSideDirichlet : kSideNeumann;
                const auto key = std::make_tuple(len, left, right);
                auto it = index.find(key);
                if (it == index.end()) {
                    if (!(len > 0.0)) fail(SEM_EINVAL, "sem_set_schwarz: degenerate element edge");
                    int lo = 0, count = 0;
                    fdm_1d(N, h.xi, h.w, h.D, len, left, right, S1, lam, lo, count);
                    const size_t base = table.size();
                    table.resize(base + TE, 0.0);
                    for (int a = 0; a < count; ++a)
                        for (int b = 0; b < count; ++b) table[base + (size_t)a * n + b] = S1[(size_t)a * count + b];
                    for (int b = 0; b < n; ++b) table[base + (size_t)n * n + b] = b < count ? lam[b] : 1.0;
                    meta.push_back(lo);
                    meta.push_back(count);
                    it = index.emplace(key, (int32_t)(meta.size() / 2 - 1)).first;
                }
                tidx[(size_t)e * 3 + dd] = it->second;
            }
        }
        Z->n_table = (int64_t)meta.size() / 2;
        Z->tidx = smalloc<int32_t>(Z, tidx.size());
        Z->table = smalloc<double>(Z, table.size());
        Z->meta = smalloc<int32_t>(Z, meta.size());
        Z->zext = smalloc<double>(Z, (size_t)E * n * n * n);
        Z->zs = smalloc<double>(Z, (size_t)h.nL);
        SEM_HIP(hipMemcpyAsync(Z->tidx, tidx.data(), sizeof(int32_t) * tidx.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipMemcpyAsync(Z->table, table.data(), sizeof(double) * table.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipMemcpyAsync(Z->meta, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        schwarz_free(Z);
        throw;
    }
    return Z;
}

static int fdm_blocks(int64_t E) { return (int)std::max<int64_t>(1, std::min<int64_t>(E, kMaxSchwarzPairs)); }


int schwarz_apply(sem_mesh *m, const double *r, double *z, double *pairs, const PcgState *st, hipStream_t s)
{
    SchwarzSpace *Z = m->schwarz;
    const Lattice L = lattice_of(m, Z->dirichlet);
    const int64_t E = m->h.E, nL = m->h.nL;
    const int fb = fdm_blocks(E);
    const int ab = vec_blocks(nL);
    switch (m->h.N) {
#define SEM_SCHWARZ_CASE(n)                                                                                       \
    case n:                                                                                                       \
        hipLaunchKernelGGL(fdm_kernel<n>, dim3(fb), dim3(kFdmThreads<n>), 0, s, E, L, r, Z->tidx, Z->table,         \
                           Z->meta, Z->zext,                                                                      \
                           pairs, st);                                                                            \
        hipLaunchKernelGGL(assemble_kernel<n>, dim3(ab), dim3(256), 0, s, E, L, Z->zext, m->inv64, z, st);        \
        break;
        SEM_SCHWARZ_CASE(2) SEM_SCHWARZ_CASE(3) SEM_SCHWARZ_CASE(4) SEM_SCHWARZ_CASE(5)
        SEM_SCHWARZ_CASE(6) SEM_SCHWARZ_CASE(7) SEM_SCHWARZ_CASE(8) SEM_SCHWARZ_CASE(9) SEM_SCHWARZ_CASE(10)
        SEM_SCHWARZ_CASE(11) SEM_SCHWARZ_CASE(12)
#undef SEM_SCHWARZ_CASE
    default: fail(SEM_EUNSUPPORTED, "Schwarz: order out of range (2..12)");
    }
    SEM_HIP(hipGetLastError());
    return fb;
}

}  // namespace sem

extern "C" sem_status sem_host_fdm_1d(int N, double ell, int left, int right, double *S, double *lam, int *lo,
                                      int *count)
{
    using namespace sem;
    try {
        if (N < 1 || N > SEM_MAX_ORDER) fail(SEM_EINVAL, "sem_host_fdm_1d: N out of range");
        if (!(ell > 0.0)) fail(SEM_EINVAL, "sem_host_fdm_1d: ell must be positive");
        if (left < 0 || left > 2 || right < 0 || right > 2) fail(SEM_EINVAL, "sem_host_fdm_1d: unknown side kind");
        if (!S || !lam || !lo || !count) fail(SEM_EINVAL, "sem_host_fdm_1d: null argument");
        std::vector<double> xi, w, D, S1, l1;
        gll_rule(N, xi, w);
        lagrange_derivative(xi, D);
        int l = 0, c = 0;
        fdm_1d(N, xi, w, D, ell, left, right, S1, l1, l, c);
        std::memcpy(S, S1.data(), sizeof(double) * S1.size());
        std::memcpy(lam, l1.data(), sizeof(double) * l1.size());
        *lo = l;
        *count = c;
        return SEM_OK;
    } catch (const Failure &f) {
        return f.status;
    } catch (const std::bad_alloc &) {
        set_error("sem_host_fdm_1d: out of memory");
        return SEM_ENOMEM;
    }
}
