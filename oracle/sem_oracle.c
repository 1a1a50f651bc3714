/*
 * sem_oracle.c -- plain, slow, FP64 CPU reference of the spectral-element
 * Poisson path: GLL rule, derivative matrix, hexahedral meshes, isoparametric
 * geometric factors, global numbering, the matrix-free local operator, the
 * direct-stiffness gather-scatter, the Jacobi diagonal and Jacobi-PCG.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU library.
 *
 * Paper: "Strong Scaling of OpenACC enabled Nek5000 on several GPU based HPC
 * systems" (arXiv 2109.03592).  Citations are to its sections, equations and
 * Algorithm 1 (the axhelm kernel).
 *
 * Plain loops only; the single optimisation is an OpenMP "parallel for" over
 * elements (or points) where iterations are independent, which does not change
 * any result.  The gather-scatter is a sequential loop in ascending local
 * index, which fixes its summation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sem_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops: n > 0 sets the count; returns the count the
 * next parallel loop uses (1 without OpenMP).  The loops' results do not
 * depend on it (each iteration writes its own outputs).                     */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Legendre polynomial P_n and its first derivative, by the three-term
 * recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}.                        */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int m = 1; m < n; ++m) {
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        /* P'_{m+1} = P'_{m-1} + (2m+1) P_m */
        double d2 = d0 + (2.0 * m + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1; *dp = d1;
}

/* Gauss-Lobatto-Legendre rule of order N (N+1 points), section 2: the element
 * basis is the tensor product of Lagrange interpolants on these points.
 * Endpoints are -1 and 1; interior points are the roots of P'_N, found by
 * Newton's method from the Chebyshev-Lobatto guesses -cos(pi i / N); P''_N
 * comes from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P.
 * Weights: w_i = 2 / (N (N+1) P_N(xi_i)^2).                                  */
void orc_gll(int N, double *xi, double *w)
{
    const double pi = 3.14159265358979323846;
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(pi * i / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, &p, &dp);
            double ddp = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / ddp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double p, dp;
        legendre(N, xi[i], &p, &dp);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
}

/* Derivative matrix D[i][l] = l_l'(xi_i), the derivative of the l-th Lagrange
 * interpolant at node i (Algorithm 1 applies it as dxm1(i,l)*u(l,...) in the
 * first pass and its transpose in the second).  Closed form for GLL points:
 * D[i][l] = P_N(xi_i) / (P_N(xi_l) (xi_i - xi_l)) for i != l,
 * D[0][0] = -N(N+1)/4, D[N][N] = N(N+1)/4, other diagonal entries 0.         */
void orc_deriv(int N, const double *xi, double *D)
{
    int P = N + 1;
    double *pn = (double *)malloc(sizeof(double) * P);
    for (int i = 0; i < P; ++i) { double dp; legendre(N, xi[i], &pn[i], &dp); }
    for (int i = 0; i < P; ++i)
        for (int l = 0; l < P; ++l) {
            double v;
            if (i != l) v = pn[i] / (pn[l] * (xi[i] - xi[l]));
            else if (i == 0) v = -N * (N + 1.0) / 4.0;
            else if (i == N) v = N * (N + 1.0) / 4.0;
            else v = 0.0;
            D[i * P + l] = v;
        }
    free(pn);
}

/* ------------------------------------------------------------------------- */
/* Mesh: an nx*ny*nz lattice of hexahedra, element e = ex + nx (ey + ny ez),
 * local node (i,j,k) of element e at local index e P^3 + i + P j + P^2 k
 * (Fortran u(lx1,ly1,lz1,e) order of Algorithm 1).                          */

long orc_num_elements(const orc_mesh *m) { return (long)m->nel[0] * m->nel[1] * m->nel[2]; }
long orc_num_local(const orc_mesh *m)
{
    long P = m->N + 1;
    return orc_num_elements(m) * P * P * P;
}

static void elem_xyz(const orc_mesh *m, long e, int *ex, int *ey, int *ez)
{
    *ex = (int)(e % m->nel[0]);
    *ey = (int)((e / m->nel[0]) % m->nel[1]);
    *ez = (int)(e / ((long)m->nel[0] * m->nel[1]));
}

/* Global lattice extent along one axis: nel*N+1 points, or nel*N when periodic
 * (the last layer is identified with the first).                             */
static long lattice_extent(const orc_mesh *m, int d)
{
    return (long)m->nel[d] * m->N + (m->periodic[d] ? 0 : 1);
}

/* Node coordinates of the elements listed in elems[0..ne) (all elements when
 * elems is NULL), written to x,y,z at index (listpos) P^3 + local node.
 * Box: trilinear map of (xi_i, xi_j, xi_k) from the element's 8 vertices,
 * taken from m->vertices when given, else from the uniform lattice lo..hi.
 * Pipe: square coordinates X, Y (uniform lattice on lo..hi) mapped to the disk
 * by (X sqrt(1 - Y^2/2), Y sqrt(1 - X^2/2)); z stays uniform.                 */
void orc_coords(const orc_mesh *m, const double *xi, const long *elems, long ne,
                double *x, double *y, double *z)
{
    const int N = m->N, P = N + 1;
    const long P3 = (long)P * P * P;
    if (!elems) ne = orc_num_elements(m);
    const int nx = m->nel[0], ny = m->nel[1], nz = m->nel[2];
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = (m->hi[d] - m->lo[d]) / m->nel[d];

#pragma omp parallel for schedule(static)
    for (long q = 0; q < ne; ++q) {
        long e = elems ? elems[q] : q;
        int ex, ey, ez;
        elem_xyz(m, e, &ex, &ey, &ez);
        /* the 8 vertex positions of this element */
        double V[8][3];
        for (int c = 0; c < 8; ++c) {
            int vx = ex + (c & 1), vy = ey + ((c >> 1) & 1), vz = ez + ((c >> 2) & 1);
            if (m->vertices) {
                long vid = vx + (long)(nx + 1) * (vy + (long)(ny + 1) * vz);
                for (int d = 0; d < 3; ++d) V[c][d] = m->vertices[vid * 3 + d];
            } else {
                V[c][0] = m->lo[0] + vx * h[0];
                V[c][1] = m->lo[1] + vy * h[1];
                V[c][2] = m->lo[2] + vz * h[2];
            }
        }
        (void)nz;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long o = q * P3 + i + (long)P * j + (long)P * P * k;
                    double r = 0.5 * (xi[i] + 1.0), s = 0.5 * (xi[j] + 1.0), t = 0.5 * (xi[k] + 1.0);
                    if (m->mapping == ORC_MAP_PIPE) {
                        double X = m->lo[0] + (ex + r) * h[0];
                        double Y = m->lo[1] + (ey + s) * h[1];
                        double Z = m->lo[2] + (ez + t) * h[2];
                        x[o] = X * sqrt(1.0 - 0.5 * Y * Y);
                        y[o] = Y * sqrt(1.0 - 0.5 * X * X);
                        z[o] = Z;
                    } else {
                        double wgt[8];
                        for (int c = 0; c < 8; ++c)
                            wgt[c] = ((c & 1) ? r : 1.0 - r) * (((c >> 1) & 1) ? s : 1.0 - s) *
                                     (((c >> 2) & 1) ? t : 1.0 - t);
                        double px = 0, py = 0, pz = 0;
                        for (int c = 0; c < 8; ++c) {
                            px += wgt[c] * V[c][0];
                            py += wgt[c] * V[c][1];
                            pz += wgt[c] * V[c][2];
                        }
                        x[o] = px; y[o] = py; z[o] = pz;
                    }
                }
    }
}

/* True where the pipe map is singular: GLL nodes whose square coordinates are
 * exactly (+-1, +-1), i.e. lattice corners of the square cross-section.
 * Decided from integer indices only.                                         */
static int pipe_singular(const orc_mesh *m, int ex, int ey, int i, int j)
{
    int N = m->N;
    int xedge = (ex == 0 && i == 0) || (ex == m->nel[0] - 1 && i == N);
    int yedge = (ey == 0 && j == 0) || (ey == m->nel[1] - 1 && j == N);
    return m->mapping == ORC_MAP_PIPE && xedge && yedge;
}

/* Isoparametric geometric factors (Algorithm 1 reads them as g1xyz..g6xyz):
 * with x_r = sum_l D[i][l] x(l,j,k) (and s, t, and y, z alike), J the 3x3
 * Jacobian d(x,y,z)/d(r,s,t) and W = w_i w_j w_k the quadrature weight,
 *   G = W det(J) J^{-1} J^{-T},  g1=G_rr g2=G_ss g3=G_tt g4=G_rs g5=G_rt g6=G_st,
 *   B = W det(J)   (diagonal mass matrix).
 * The pairing g4<->(r,s), g5<->(r,t), g6<->(s,t) is the one Algorithm 1's
 * combine step uses.  Output G has 6 planes of length nloc = ne P^3
 * (component-major: G[c*nloc + point]).  Pipe nodes where the map is singular
 * get G = 0 and B = 0 (that quadrature point is dropped).                    */
void orc_geom(const orc_mesh *m, const double *w, const double *D, const long *elems, long ne,
              const double *x, const double *y, const double *z, double *G, double *B)
{
    const int N = m->N, P = N + 1;
    const long P3 = (long)P * P * P;
    if (!elems) ne = orc_num_elements(m);
    const long nloc = ne * P3;

#pragma omp parallel for schedule(static)
    for (long q = 0; q < ne; ++q) {
        long e = elems ? elems[q] : q;
        int ex, ey, ez;
        elem_xyz(m, e, &ex, &ey, &ez);
        const double *X[3] = {x + q * P3, y + q * P3, z + q * P3};
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long p = i + (long)P * j + (long)P * P * k;
                    double J[3][3];
                    for (int a = 0; a < 3; ++a) {
                        double dr = 0, ds = 0, dt = 0;
                        for (int l = 0; l < P; ++l) {
                            dr += D[i * P + l] * X[a][l + P * j + P * P * k];
                            ds += D[j * P + l] * X[a][i + P * l + P * P * k];
                            dt += D[k * P + l] * X[a][i + P * j + P * P * l];
                        }
                        J[a][0] = dr; J[a][1] = ds; J[a][2] = dt;
                    }
                    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    /* inverse via the adjugate: Ji[a][b] = d(r_a)/d(x_b) */
                    double Ji[3][3];
                    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    double W = w[i] * w[j] * w[k];
                    double g[6];
                    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
                    for (int c = 0; c < 6; ++c) {
                        double s = 0;
                        for (int b = 0; b < 3; ++b) s += Ji[pa[c]][b] * Ji[pb[c]][b];
                        g[c] = W * det * s;
                    }
                    double bm = W * det;
                    if (pipe_singular(m, ex, ey, i, j)) {
                        for (int c = 0; c < 6; ++c) g[c] = 0.0;
                        bm = 0.0;
                    }
                    for (int c = 0; c < 6; ++c) G[c * nloc + q * P3 + p] = g[c];
                    B[q * P3 + p] = bm;
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Global numbering (section 2: global operations exchange element face values;
 * the numbering itself is a canonical lexicographic choice): the lattice index
 * of node (i,j,k) of element (ex,ey,ez) is a = ex N + i, b = ey N + j,
 * c = ez N + k (reduced modulo the extent on a periodic axis), and
 * gid = a + gx (b + gy c).                                                    */
long orc_num_global(const orc_mesh *m)
{
    return lattice_extent(m, 0) * lattice_extent(m, 1) * lattice_extent(m, 2);
}

void orc_numbering(const orc_mesh *m, const long *elems, long ne, int64_t *gid)
{
    const int N = m->N, P = N + 1;
    const long P3 = (long)P * P * P;
    if (!elems) ne = orc_num_elements(m);
    long gx = lattice_extent(m, 0), gy = lattice_extent(m, 1), gz = lattice_extent(m, 2);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < ne; ++q) {
        long e = elems ? elems[q] : q;
        int ex, ey, ez;
        elem_xyz(m, e, &ex, &ey, &ez);
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long a = (long)ex * N + i, b = (long)ey * N + j, c = (long)ez * N + k;
                    if (m->periodic[0]) a %= gx;
                    if (m->periodic[1]) b %= gy;
                    if (m->periodic[2]) c %= gz;
                    gid[q * P3 + i + P * j + P * P * k] = a + gx * (b + gy * c);
                }
    }
}

/* Dirichlet mask per global id: 1 on a non-periodic boundary face selected by
 * m->dirichlet (bit 2d: low face of axis d, bit 2d+1: high face).            */
void orc_global_mask(const orc_mesh *m, uint8_t *gmask)
{
    long ext[3] = {lattice_extent(m, 0), lattice_extent(m, 1), lattice_extent(m, 2)};
    long nG = ext[0] * ext[1] * ext[2];
#pragma omp parallel for schedule(static)
    for (long g = 0; g < nG; ++g) {
        long idx[3] = {g % ext[0], (g / ext[0]) % ext[1], g / (ext[0] * ext[1])};
        uint8_t mk = 0;
        for (int d = 0; d < 3; ++d) {
            if (m->periodic[d]) continue;
            if (idx[d] == 0 && (m->dirichlet >> (2 * d) & 1)) mk = 1;
            if (idx[d] == ext[d] - 1 && (m->dirichlet >> (2 * d + 1) & 1)) mk = 1;
        }
        gmask[g] = mk;
    }
}

/* Multiplicity per global id: the number of local copies.                    */
void orc_multiplicity(long nloc, const int64_t *gid, long nglob, int32_t *gmult)
{
    memset(gmult, 0, sizeof(int32_t) * nglob);
    for (long l = 0; l < nloc; ++l) gmult[gid[l]] += 1;
}

/* ------------------------------------------------------------------------- */
/* Local operator of one element in tensor-product form (section 2: the GLL
 * stiffness of Eq. 5, or Eq. 4's Helmholtz form; Algorithm 1 evaluates the
 * same operator).  With D_a the 1-D derivative matrix acting along axis a of
 * the element's (i,j,k) grid (a = r: i, s: j, t: k), G the symmetric 3x3
 * matrix of geometric factors at each point (g1 = G_rr, g2 = G_ss,
 * g3 = G_tt, g4 = G_rs, g5 = G_rt, g6 = G_st; weights and det J folded in):
 *   A_e u = sum_a D_a^T (h1 sum_b G_ab (D_b u)) + h2 B u,
 * evaluated as three stages: the reference gradient (D_r u, D_s u, D_t u),
 * the pointwise metric product, and the transposed contractions, each
 * direction in its own pass and the three added per point (r, then s, then
 * t).  Every contraction sums over its index in ascending order.  h1 == NULL
 * means h1 = 1 (Poisson); h2 or B == NULL means no mass term.             */

/* y = (M along axis `axis`) x on a P^3 grid, or with M transposed:
 *   axis 0: y(i,j,k) = sum_l M(i,l) x(l,j,k)   (transposed: M(l,i))
 *   axis 1: y(i,j,k) = sum_l M(j,l) x(i,l,k)
 *   axis 2: y(i,j,k) = sum_l M(k,l) x(i,j,l)                             */
static void contract_axis(int P, const double *M, int transposed, int axis, const double *x, double *y)
{
    const long stride = axis == 0 ? 1 : (axis == 1 ? P : (long)P * P);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                const int row = axis == 0 ? i : (axis == 1 ? j : k);
                const long base = i + (long)P * j + (long)P * P * k - (long)row * stride;
                double sum = 0.0;
                for (int l = 0; l < P; ++l) {
                    const double m = transposed ? M[l * P + row] : M[row * P + l];
                    sum += m * x[base + l * stride];
                }
                y[i + (long)P * j + (long)P * P * k] = sum;
            }
}

void orc_ax(int N, long ne, const double *D, const double *G, const double *h1,
            const double *h2, const double *B, const double *u, double *w)
{
    const int P = N + 1;
    const long P3 = (long)P * P * P;
    const long nloc = ne * P3;
    /* position in G of the factor G_ab (component-major, g1..g6 as above) */
    static const int comp[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma omp parallel
    {
        double *grad = (double *)malloc(sizeof(double) * 3 * P3);  /* D_a u        */
        double *flux = (double *)malloc(sizeof(double) * 3 * P3);  /* h1 G grad    */
        double *part = (double *)malloc(sizeof(double) * 3 * P3);  /* D_a^T flux_a */
#pragma omp for schedule(static)
        for (long e = 0; e < ne; ++e) {
            const double *ue = u + e * P3;
            for (int ax = 0; ax < 3; ++ax) contract_axis(P, D, 0, ax, ue, grad + ax * P3);
            for (long p = 0; p < P3; ++p) {
                const long o = e * P3 + p;
                const double scale = h1 ? h1[o] : 1.0;
                for (int ax = 0; ax < 3; ++ax) {
                    double f = 0.0;
                    for (int bx = 0; bx < 3; ++bx) f += G[comp[ax][bx] * nloc + o] * grad[bx * P3 + p];
                    flux[ax * P3 + p] = f * scale;
                }
            }
            for (int ax = 0; ax < 3; ++ax) contract_axis(P, D, 1, ax, flux + ax * P3, part + ax * P3);
            for (long p = 0; p < P3; ++p) {
                const long o = e * P3 + p;
                double v = part[p] + part[P3 + p] + part[2 * P3 + p];
                if (h2 && B) v += h2[o] * B[o] * ue[p];
                w[o] = v;
            }
        }
        free(grad); free(flux); free(part);
    }
}

/* ------------------------------------------------------------------------- */
/* Direct-stiffness summation Q Q^T followed by the Dirichlet mask: every local
 * copy of global node g receives s_g = sum of all copies of g, the sum taken
 * in ascending local index starting from 0; masked g get 0.  Sequential on
 * purpose, which fixes the summation order.                                  */
void orc_gs(long nloc, const int64_t *gid, long nglob, const uint8_t *gmask, double *v)
{
    double *s = (double *)calloc((size_t)nglob, sizeof(double));
    for (long l = 0; l < nloc; ++l) s[gid[l]] += v[l];
    for (long l = 0; l < nloc; ++l) v[l] = (gmask && gmask[gid[l]]) ? 0.0 : s[gid[l]];
    free(s);
}

/* ------------------------------------------------------------------------- */
/* Assembled Jacobi diagonal.  The local diagonal of Algorithm 1's operator at
 * (i,j,k) follows from applying it to a unit vector:
 *   sum_l D[l][i]^2 g1(l,j,k) + sum_l D[l][j]^2 g2(i,l,k) + sum_l D[l][k]^2 g3(i,j,l)
 *   + 2 D[i][i] D[j][j] g4 + 2 D[i][i] D[k][k] g5 + 2 D[j][j] D[k][k] g6   (times h1)
 * plus h2 B for the Helmholtz mass term; it is then summed over copies (gs),
 * and invdiag = 1/diag on unmasked nodes, 0 on masked ones.                   */
void orc_jacobi(int N, long ne, const double *D, const double *G, const double *h1,
                const double *h2, const double *B, const int64_t *gid, long nglob,
                const uint8_t *gmask, double *invdiag)
{
    const int P = N + 1;
    const long P3 = (long)P * P * P;
    const long nloc = ne * P3;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < ne; ++e)
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    long o = e * P3 + i + (long)P * j + (long)P * P * k;
                    double d = 0;
                    for (int l = 0; l < P; ++l) {
                        long orr = e * P3 + l + (long)P * j + (long)P * P * k;
                        long oss = e * P3 + i + (long)P * l + (long)P * P * k;
                        long ott = e * P3 + i + (long)P * j + (long)P * P * l;
                        double hr = h1 ? h1[orr] : 1.0, hs = h1 ? h1[oss] : 1.0, ht = h1 ? h1[ott] : 1.0;
                        d += D[l * P + i] * D[l * P + i] * G[0 * nloc + orr] * hr;
                        d += D[l * P + j] * D[l * P + j] * G[1 * nloc + oss] * hs;
                        d += D[l * P + k] * D[l * P + k] * G[2 * nloc + ott] * ht;
                    }
                    double h = h1 ? h1[o] : 1.0;
                    d += 2.0 * D[i * P + i] * D[j * P + j] * G[3 * nloc + o] * h;
                    d += 2.0 * D[i * P + i] * D[k * P + k] * G[4 * nloc + o] * h;
                    d += 2.0 * D[j * P + j] * D[k * P + k] * G[5 * nloc + o] * h;
                    if (h2 && B) d += h2[o] * B[o];
                    invdiag[o] = d;
                }
    orc_gs(nloc, gid, nglob, gmask, invdiag);
    for (long l = 0; l < nloc; ++l)
        invdiag[l] = (gmask && gmask[gid[l]]) ? 0.0 : 1.0 / invdiag[l];
}

/* ------------------------------------------------------------------------- */
/* Unique-dof inner product: every global node counted once, i.e. the local
 * sum weighted by 1/multiplicity.                                            */
static double dot_unique(long nloc, const double *a, const double *b, const int64_t *gid,
                         const int32_t *gmult)
{
    double s = 0;
    for (long l = 0; l < nloc; ++l) s += a[l] * b[l] / gmult[gid[l]];
    return s;
}

/* w = mask(Q Q^T (A_L v)) on the whole mesh.                                 */
static void apply_A(const orc_problem *pb, const double *v, double *w)
{
    orc_ax(pb->N, pb->ne, pb->D, pb->G, pb->h1, pb->h2, pb->B, v, w);
    orc_gs(pb->nloc, pb->gid, pb->nglob, pb->gmask, w);
}

void orc_apply(const orc_problem *pb, const double *v, double *w) { apply_A(pb, v, w); }

/* Jacobi-preconditioned conjugate gradients on the masked, assembled system
 * A x = b (b continuous and masked).  x holds the initial guess on entry.
 *   r = b - A x, z = invdiag r, p = z, rho = <r,z>;
 *   loop: w = A p; sigma = <p,w>; alpha = rho/sigma; x += alpha p; r -= alpha w;
 *         stop when ||r|| <= tol ||b||; z = invdiag r; rho' = <r,z>;
 *         beta = rho'/rho; p = z + beta p.
 * On exit the true residual b - A x is recomputed; if it still exceeds tol the
 * iteration restarts from x (at most 3 restarts).  Returns 0 on convergence,
 * 1 when max_iter is reached, 2 on breakdown (sigma <= 0 or not finite).      */
int orc_pcg(const orc_problem *pb, const double *b, double *x, double tol, int max_iter,
            orc_pcg_stats *st)
{
    const long n = pb->nloc;
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    int32_t *gmult = (int32_t *)malloc(sizeof(int32_t) * pb->nglob);
    orc_multiplicity(n, pb->gid, pb->nglob, gmult);

    double bnorm = sqrt(dot_unique(n, b, b, pb->gid, gmult));
    int status = 1, iters = 0, restarts = 0;
    double rel = 0;
    for (;;) {
        apply_A(pb, x, w);
        for (long l = 0; l < n; ++l) r[l] = b[l] - w[l];
        double rn = sqrt(dot_unique(n, r, r, pb->gid, gmult));
        rel = bnorm > 0 ? rn / bnorm : rn;
        if (rel <= tol) { status = 0; break; }
        if (iters >= max_iter) { status = 1; break; }
        if (iters > 0) {
            if (restarts == 3) { status = 1; break; }
            restarts++;
        }
        for (long l = 0; l < n; ++l) { z[l] = pb->invdiag[l] * r[l]; p[l] = z[l]; }
        double rho = dot_unique(n, r, z, pb->gid, gmult);
        int inner_done = 0;
        while (iters < max_iter) {
            apply_A(pb, p, w);
            double sigma = dot_unique(n, p, w, pb->gid, gmult);
            if (!(sigma > 0) || !isfinite(sigma)) { status = 2; inner_done = 2; break; }
            double alpha = rho / sigma;
            for (long l = 0; l < n; ++l) { x[l] += alpha * p[l]; r[l] -= alpha * w[l]; }
            iters++;
            double rn2 = sqrt(dot_unique(n, r, r, pb->gid, gmult));
            if (rn2 <= tol * bnorm) { inner_done = 1; break; }
            for (long l = 0; l < n; ++l) z[l] = pb->invdiag[l] * r[l];
            double rho1 = dot_unique(n, r, z, pb->gid, gmult);
            double beta = rho1 / rho;
            rho = rho1;
            for (long l = 0; l < n; ++l) p[l] = z[l] + beta * p[l];
        }
        if (inner_done == 2) break;
    }
    if (st) {
        st->iterations = iters;
        st->restarts = restarts;
        st->rel_residual = rel;
        st->bnorm = bnorm;
    }
    free(r); free(z); free(p); free(w); free(gmult);
    return status;
}
