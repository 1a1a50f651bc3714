// setup.cpp -- host-side set-up of a structured hexahedral SEM mesh:
// GLL rule and derivative matrix, node coordinates, isoparametric geometric
// factors, lexicographic global numbering, the sorted gather-scatter plan and
// the assembled Jacobi diagonal.  Runs once per mesh; the products are
// uploaded by the C ABI layer.
//
// Paper (arXiv 2109.03592) section 2: the domain is split into hexahedral
// elements, each a tensor product of Lagrange interpolants on GLL points;
// global work (exchange of element face values) is separated from local
// matrix-free work.  Algorithm 1 reads the six geometric factors g1..g6.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "sem_internal.hpp"

namespace sem {

void host_parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &body)
{
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 32));
    nt = std::min<int64_t>(nt, std::max<int64_t>(1, n / 64));
    if (nt <= 1) {
        body(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&body, a, b] { body(a, b); });
    }
    for (auto &t : th) t.join();
}

// Legendre P_n(x) by the three-term recurrence.
static void legendre_pair(int n, double x, double &pn, double &pnm1, double &pnp1)
{
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) {
        pnm1 = 0.0; pn = 1.0; pnp1 = x;
        return;
    }
    for (int m = 1; m < n; ++m) {
        double c = ((2 * m + 1) * x * b - m * a) / (m + 1);
        a = b; b = c;
    }
    pnm1 = a; pn = b;
    pnp1 = ((2 * n + 1) * x * pn - n * pnm1) / (n + 1);
}

// GLL points are the zeros of (1 - x^2) P_N'(x), which is proportional to
// P_{N-1}(x) - P_{N+1}(x).  With f = P_{N+1} - P_{N-1}, f' = (2N+1) P_N, so the
// interior points follow from Newton's method on f started at the
// Chebyshev-Gauss-Lobatto points.  Weights 2 / (N (N+1) P_N(x_i)^2).
void gll_rule(int N, std::vector<double> &xi, std::vector<double> &w)
{
    xi.assign(N + 1, 0.0);
    w.assign(N + 1, 0.0);
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -std::cos(M_PI * i / N);
        for (int it = 0; it < 200; ++it) {
            double pn, pm, pp;
            legendre_pair(N, x, pn, pm, pp);
            double dx = (pp - pm) / ((2 * N + 1) * pn);
            x -= dx;
            if (std::fabs(dx) <= 1e-17) break;
        }
        xi[i] = x;
    }
    // symmetrise: the rule is exactly symmetric about 0
    for (int i = 0; i <= N / 2; ++i) {
        double a = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -a;
        xi[N - i] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double pn, pm, pp;
        legendre_pair(N, xi[i], pn, pm, pp);
        w[i] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
}

// Derivative of the Lagrange interpolants through the nodes, by barycentric
// weights lambda_j = 1 / prod_{m != j} (x_j - x_m):
//   D[i][j] = (lambda_j / lambda_i) / (x_i - x_j) (i != j),  D[i][i] = -sum_{j!=i} D[i][j].
void lagrange_derivative(const std::vector<double> &xi, std::vector<double> &D)
{
    const int P = (int)xi.size();
    std::vector<double> lam(P, 1.0);
    for (int j = 0; j < P; ++j)
        for (int m = 0; m < P; ++m)
            if (m != j) lam[j] /= (xi[j] - xi[m]);
    D.assign((size_t)P * P, 0.0);
    for (int i = 0; i < P; ++i) {
        double diag = 0.0;
        for (int j = 0; j < P; ++j) {
            if (j == i) continue;
            double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[(size_t)i * P + j] = v;
            diag -= v;
        }
        D[(size_t)i * P + i] = diag;
    }
}

namespace {

struct ElemIndex {
    int ex, ey, ez;
};

inline ElemIndex elem_index(const HostMesh &h, int64_t e)
{
    ElemIndex r;
    r.ex = (int)(e % h.nel[0]);
    r.ey = (int)((e / h.nel[0]) % h.nel[1]);
    r.ez = (int)(e / ((int64_t)h.nel[0] * h.nel[1]));
    return r;
}

void build_coords(const sem_mesh_desc &d, HostMesh &h)
{
    const int P = h.P;
    const int64_t P3 = (int64_t)P * P * P;
    h.xyz.assign((size_t)3 * h.nL, 0.0);
    double hx[3];
    for (int a = 0; a < 3; ++a) hx[a] = (d.hi[a] - d.lo[a]) / d.nel[a];
    const int nx = d.nel[0], ny = d.nel[1];
    double *X = h.xyz.data(), *Y = X + h.nL, *Z = Y + h.nL;
    host_parallel_for(h.E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            ElemIndex ix = elem_index(h, e);
            double V[8][3];
            for (int c = 0; c < 8; ++c) {
                int v[3] = {ix.ex + (c & 1), ix.ey + ((c >> 1) & 1), ix.ez + ((c >> 2) & 1)};
                if (d.vertices) {
                    int64_t vid = v[0] + (int64_t)(nx + 1) * (v[1] + (int64_t)(ny + 1) * v[2]);
                    for (int a = 0; a < 3; ++a) V[c][a] = d.vertices[vid * 3 + a];
                } else {
                    for (int a = 0; a < 3; ++a) V[c][a] = d.lo[a] + v[a] * hx[a];
                }
            }
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j)
                    for (int i = 0; i < P; ++i) {
                        const int64_t o = e * P3 + i + (int64_t)P * (j + (int64_t)P * k);
                        const double r = 0.5 * (h.xi[i] + 1.0), s = 0.5 * (h.xi[j] + 1.0),
                                     t = 0.5 * (h.xi[k] + 1.0);
                        if (d.mapping == SEM_MAP_PIPE_SQ2DISK) {
                            const double Xs = d.lo[0] + (ix.ex + r) * hx[0];
                            const double Ys = d.lo[1] + (ix.ey + s) * hx[1];
                            X[o] = Xs * std::sqrt(1.0 - 0.5 * Ys * Ys);
                            Y[o] = Ys * std::sqrt(1.0 - 0.5 * Xs * Xs);
                            Z[o] = d.lo[2] + (ix.ez + t) * hx[2];
                        } else {
                            // trilinear blend of the 8 vertices
                            const double fr[2] = {1.0 - r, r}, fs[2] = {1.0 - s, s}, ft[2] = {1.0 - t, t};
                            double acc[3] = {0, 0, 0};
                            for (int c = 0; c < 8; ++c) {
                                const double wgt = fr[c & 1] * fs[(c >> 1) & 1] * ft[(c >> 2) & 1];
                                for (int a = 0; a < 3; ++a) acc[a] += wgt * V[c][a];
                            }
                            X[o] = acc[0]; Y[o] = acc[1]; Z[o] = acc[2];
                        }
                    }
        }
    });
}

// Singular nodes of the square-to-disk map: square coordinates (+-1, +-1).
inline bool pipe_corner(const HostMesh &h, const ElemIndex &ix, int i, int j)
{
    const int N = h.N;
    const bool xe = (ix.ex == 0 && i == 0) || (ix.ex == h.nel[0] - 1 && i == N);
    const bool ye = (ix.ey == 0 && j == 0) || (ix.ey == h.nel[1] - 1 && j == N);
    return xe && ye;
}

void build_geometry(const sem_mesh_desc &d, HostMesh &h)
{
    const int P = h.P;
    const int64_t P3 = (int64_t)P * P * P;
    h.G.assign((size_t)6 * h.nL, 0.0);
    h.B.assign((size_t)h.nL, 0.0);
    const double *Xa[3] = {h.xyz.data(), h.xyz.data() + h.nL, h.xyz.data() + 2 * h.nL};
    const double *D = h.D.data();
    std::atomic<int> bad{0};
    host_parallel_for(h.E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            const ElemIndex ix = elem_index(h, e);
            double *Ge = h.G.data() + e * 6 * P3;
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j)
                    for (int i = 0; i < P; ++i) {
                        const int64_t p = i + (int64_t)P * (j + (int64_t)P * k);
                        // J[a][b] = d x_a / d r_b  (a: x,y,z; b: r,s,t)
                        double J[3][3];
                        for (int a = 0; a < 3; ++a) {
                            const double *xe = Xa[a] + e * P3;
                            double dr = 0, ds = 0, dt = 0;
                            for (int l = 0; l < P; ++l) {
                                dr += D[i * P + l] * xe[l + P * (j + P * k)];
                                ds += D[j * P + l] * xe[i + P * (l + P * k)];
                                dt += D[k * P + l] * xe[i + P * (j + P * l)];
                            }
                            J[a][0] = dr; J[a][1] = ds; J[a][2] = dt;
                        }
                        // cofactors C[a][b]; inverse Ji[b][a] = C[a][b] / det
                        double C[3][3];
                        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
                        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
                        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
                        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
                        const double Wq = h.w[i] * h.w[j] * h.w[k];
                        double g[6], bm;
                        const bool corner = d.mapping == SEM_MAP_PIPE_SQ2DISK && pipe_corner(h, ix, i, j);
                        if (corner) {
                            for (int c = 0; c < 6; ++c) g[c] = 0.0;
                            bm = 0.0;
                        } else {
                            if (!(det > 0.0) || !std::isfinite(det)) bad.store(1, std::memory_order_relaxed);
                            // grad r_b = row b of J^{-1} = C[.][b] / det;
                            // G_bc = W det (grad r_b . grad r_c) = W (C[:,b] . C[:,c]) / det
                            const int pb[6] = {0, 1, 2, 0, 0, 1}, pc[6] = {0, 1, 2, 1, 2, 2};
                            for (int c = 0; c < 6; ++c) {
                                double s = 0.0;
                                for (int a = 0; a < 3; ++a) s += C[a][pb[c]] * C[a][pc[c]];
                                g[c] = Wq * s / det;
                            }
                            bm = Wq * det;
                        }
                        for (int c = 0; c < 6; ++c) Ge[c * P3 + p] = g[c];
                        h.B[e * P3 + p] = bm;
                    }
        }
    });
    if (bad.load()) fail(SEM_EINVAL, "sem_setup: element with non-positive Jacobian determinant");
}

void build_numbering(const sem_mesh_desc &d, HostMesh &h)
{
    const int N = h.N, P = h.P;
    const int64_t P3 = (int64_t)P * P * P;
    for (int a = 0; a < 3; ++a) h.ext[a] = (int64_t)d.nel[a] * N + (d.periodic[a] ? 0 : 1);
    h.nG = h.ext[0] * h.ext[1] * h.ext[2];
    if (h.nG >= INT32_MAX || h.nL >= INT32_MAX)
        fail(SEM_EUNSUPPORTED, "sem_setup: more than 2^31-1 nodes");
    h.gid.assign((size_t)h.nL, 0);
    host_parallel_for(h.E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            const ElemIndex ix = elem_index(h, e);
            for (int k = 0; k < P; ++k) {
                int64_t c = (int64_t)ix.ez * N + k;
                if (d.periodic[2] && c == h.ext[2]) c = 0;
                for (int j = 0; j < P; ++j) {
                    int64_t b = (int64_t)ix.ey * N + j;
                    if (d.periodic[1] && b == h.ext[1]) b = 0;
                    for (int i = 0; i < P; ++i) {
                        int64_t a = (int64_t)ix.ex * N + i;
                        if (d.periodic[0] && a == h.ext[0]) a = 0;
                        h.gid[e * P3 + i + P * (j + (int64_t)P * k)] = (int32_t)(a + h.ext[0] * (b + h.ext[1] * c));
                    }
                }
            }
        }
    });
    // Dirichlet mask from the lattice position of each global node
    int faces = d.dirichlet_faces;
    if (faces < 0) {
        faces = 0;
        for (int a = 0; a < 3; ++a)
            if (!d.periodic[a]) faces |= 3 << (2 * a);
    }
    h.gmask.assign((size_t)h.nG, 0);
    host_parallel_for(h.nG, [&](int64_t g0, int64_t g1) {
        for (int64_t g = g0; g < g1; ++g) {
            const int64_t idx[3] = {g % h.ext[0], (g / h.ext[0]) % h.ext[1], g / (h.ext[0] * h.ext[1])};
            uint8_t m = 0;
            for (int a = 0; a < 3; ++a) {
                if (d.periodic[a]) continue;
                if (idx[a] == 0 && ((faces >> (2 * a)) & 1)) m = 1;
                if (idx[a] == h.ext[a] - 1 && ((faces >> (2 * a + 1)) & 1)) m = 1;
            }
            h.gmask[g] = m;
        }
    });
}

// Gather-scatter plan.  Global ids with two or more copies and no mask are
// "summed" ids; masked ids are "zeroed" ids.  Each id lists its local copies
// in ascending local index (a stable counting sort by global id), which fixes
// the summation order.  Summed ids come first, both groups ascending by id.
void build_gs_plan(HostMesh &h)
{
    std::vector<int64_t> start((size_t)h.nG + 1, 0);
    for (int64_t l = 0; l < h.nL; ++l) start[(size_t)h.gid[l] + 1]++;
    h.gmult.assign((size_t)h.nG, 0);
    for (int64_t g = 0; g < h.nG; ++g) h.gmult[g] = (uint8_t)start[g + 1];
    for (int64_t g = 0; g < h.nG; ++g) start[g + 1] += start[g];
    std::vector<int32_t> sorted((size_t)h.nL);
    {
        std::vector<int64_t> cur(start.begin(), start.end() - 1);
        for (int64_t l = 0; l < h.nL; ++l) sorted[cur[h.gid[l]]++] = (int32_t)l;
    }
    h.n_shared_local = h.n_shared_global = h.n_masked_global = 0;
    int64_t n_sum = 0, n_zero = 0, len_sum = 0, len_zero = 0;
    for (int64_t g = 0; g < h.nG; ++g) {
        const int64_t m = h.gmult[g];
        if (m >= 2) { h.n_shared_global++; h.n_shared_local += m; }
        if (h.gmask[g]) { n_zero++; len_zero += m; h.n_masked_global++; }
        else if (m >= 2) { n_sum++; len_sum += m; }
    }
    h.gs_n_sum = n_sum;
    h.gs_n_ids = n_sum + n_zero;
    h.gs_off.assign((size_t)h.gs_n_ids + 1, 0);
    h.gs_idx.assign((size_t)(len_sum + len_zero), 0);
    int64_t id = 0, pos = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t g = 0; g < h.nG; ++g) {
            const bool take = pass == 0 ? (!h.gmask[g] && h.gmult[g] >= 2) : (h.gmask[g] != 0);
            if (!take) continue;
            h.gs_off[id++] = (int32_t)pos;
            for (int64_t q = start[g]; q < start[g + 1]; ++q) h.gs_idx[pos++] = sorted[q];
        }
    }
    h.gs_off[id] = (int32_t)pos;
    h.gs_plan_len = pos;
}

}  // namespace

// Local diagonal of Algorithm 1's operator at (i,j,k), obtained by applying
// it to the unit vector of that node:
//   sum_l D[l][i]^2 g1(l,j,k) + sum_l D[l][j]^2 g2(i,l,k) + sum_l D[l][k]^2 g3(i,j,l)
//   + 2 D[i][i] D[j][j] g4 + 2 D[i][i] D[k][k] g5 + 2 D[j][j] D[k][k] g6,
// then summed over copies with the plan (same order as the device
// gather-scatter) and inverted; masked nodes get 0.
void build_jacobi(HostMesh &h)
{
    const int P = h.P;
    const int64_t P3 = (int64_t)P * P * P;
    const double *D = h.D.data();
    h.invdiag.assign((size_t)h.nL, 0.0);
    host_parallel_for(h.E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            const double *Ge = h.G.data() + e * 6 * P3;
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j)
                    for (int i = 0; i < P; ++i) {
                        const int64_t p = i + (int64_t)P * (j + (int64_t)P * k);
                        double acc = 0.0;
                        for (int l = 0; l < P; ++l) {
                            const double di = D[l * P + i], dj = D[l * P + j], dk = D[l * P + k];
                            acc += di * di * Ge[0 * P3 + l + P * (j + P * k)];
                            acc += dj * dj * Ge[1 * P3 + i + P * (l + P * k)];
                            acc += dk * dk * Ge[2 * P3 + i + P * (j + P * l)];
                        }
                        const double dii = D[i * P + i], djj = D[j * P + j], dkk = D[k * P + k];
                        acc += 2.0 * dii * djj * Ge[3 * P3 + p];
                        acc += 2.0 * dii * dkk * Ge[4 * P3 + p];
                        acc += 2.0 * djj * dkk * Ge[5 * P3 + p];
                        h.invdiag[e * P3 + p] = acc;
                    }
        }
    });
    // assemble over copies: summed ids in plan order, zeroed ids -> 0
    for (int64_t id = 0; id < h.gs_n_ids; ++id) {
        const int32_t a = h.gs_off[id], b = h.gs_off[id + 1];
        double s = 0.0;
        if (id < h.gs_n_sum)
            for (int32_t q = a; q < b; ++q) s += h.invdiag[h.gs_idx[q]];
        for (int32_t q = a; q < b; ++q) h.invdiag[h.gs_idx[q]] = s;
    }
    int bad = 0;
    for (int64_t l = 0; l < h.nL; ++l) {
        if (h.gmask[h.gid[l]]) {
            h.invdiag[l] = 0.0;
        } else {
            if (!(h.invdiag[l] > 0.0)) bad = 1;
            h.invdiag[l] = 1.0 / h.invdiag[l];
        }
    }
    if (bad) fail(SEM_EINVAL, "non-positive assembled diagonal (degenerate mesh)");
}

void build_host_coords(const sem_mesh_desc &d, HostMesh &h)
{
    h.N = d.N;
    h.P = d.N + 1;
    for (int a = 0; a < 3; ++a) h.nel[a] = d.nel[a];
    h.E = (int64_t)d.nel[0] * d.nel[1] * d.nel[2];
    h.nL = h.E * h.P * h.P * h.P;
    gll_rule(h.N, h.xi, h.w);
    build_coords(d, h);
}

void build_host_mesh(const sem_mesh_desc &d, HostMesh &h)
{
    if (d.N < 1 || d.N > SEM_MAX_ORDER) fail(SEM_EINVAL, "sem_setup: N must be in 1..SEM_MAX_ORDER");
    for (int a = 0; a < 3; ++a) {
        if (d.nel[a] < 1) fail(SEM_EINVAL, "sem_setup: element counts must be positive");
        if (!(d.hi[a] > d.lo[a])) fail(SEM_EINVAL, "sem_setup: need hi > lo on every axis");
    }
    if (d.mapping != SEM_MAP_BOX && d.mapping != SEM_MAP_PIPE_SQ2DISK)
        fail(SEM_EINVAL, "sem_setup: unknown mapping");
    h.N = d.N;
    h.P = d.N + 1;
    for (int a = 0; a < 3; ++a) {
        h.nel[a] = d.nel[a];
        h.periodic[a] = d.periodic[a] ? 1 : 0;
    }
    h.E = (int64_t)d.nel[0] * d.nel[1] * d.nel[2];
    h.nL = h.E * h.P * h.P * h.P;
    gll_rule(h.N, h.xi, h.w);
    lagrange_derivative(h.xi, h.D);
    build_coords(d, h);
    build_geometry(d, h);
    build_numbering(d, h);
    build_gs_plan(h);
    build_jacobi(h);
}

}  // namespace sem
