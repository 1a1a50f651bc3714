// lattice.hpp -- the plan-free gather-scatter's view of a mesh as a lattice
// of hexahedra: the enumeration of the face-lattice nodes and the local
// offsets of each node's copies.  Host and device share these functions, so
// the host can check the enumeration the kernels walk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

// Division by an invariant 32-bit divisor d >= 1 as a multiply-high, an add
// and two shifts (Granlund and Montgomery, "Division by invariant integers
// using multiplication", PLDI 1994, the unsigned round-up method): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, n),  n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0)
// for every unsigned 32-bit n.  The lanes of the lattice gather-scatter
// decode their positions with it instead of the compiler's generic division.
struct UDiv {
    uint32_t m;
    uint32_t s1, s2;
};

inline UDiv udiv_make(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;
    UDiv u;
    u.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    u.s1 = l < 1 ? l : 1;
    u.s2 = l > 1 ? l - 1 : 0;
    return u;
}

__host__ __device__ inline uint32_t udiv(const UDiv &u, uint32_t n)
{
    const uint32_t t = (uint32_t)(((uint64_t)u.m * n) >> 32);  // one v_mul_hi_u32 on the device
    return (t + ((n - t) >> u.s1)) >> u.s2;
}

// Gather-scatter on the element lattice.  Every mesh here is a lattice of
// nel[0] x nel[1] x nel[2] hexahedra, and the global node at lattice position
// (X, Y, Z) has its copies at the elements and GLL indices that the position
// fixes: along each axis one copy inside an element (X mod N != 0), or the
// two ends of neighbouring elements (X mod N == 0), or one end at a
// non-periodic boundary.  The kernel therefore reads no plan: one lane per
// node of the face lattice (some coordinate a multiple of N), met element
// layer by element layer in z.  Per layer zl: the z-plane Z = zl N (ext[0]
// ext[1] nodes, x fastest); then per element row yl in y: the N - 1 rows
// Y = yl N, Z = zl N + 1 .. zl N + N - 1 (ext[0] nodes each, x fastest),
// followed, while yl < nel[1], by the x-face nodes of the element row
// (zl, yl) that lie off both (X mod N == 0, Y and Z not) face by face: per
// x-face q its (N - 1)^2 nodes with y fastest, so that consecutive lanes
// read consecutive rows of the two elements that share the face and the next
// face's lanes the other end of the same rows, while the y-rows just before
// touch the neighbouring rows of the same elements.  Copies are summed in
// ascending local index (nested z, y, x over each axis's copies in
// ascending element), which is the plan's
// order whenever a node's copies lie in distinct elements, i.e. every
// periodic axis has at least two elements.  Masked (Dirichlet) nodes get 0
// at every copy; an unmasked node with one copy is left untouched, as the
// plan leaves it.
struct GsLattice {
    int N;
    int nel[3];
    int periodic[3];
    int faces;          // Dirichlet face bits: axis a low face 1 << 2a, high face 1 << (2a + 1)
    int ext[3];         // distinct lattice coordinates per axis
    int np0;            // x coordinates that are multiples of N
    int c_zplane;       // nodes of a z-plane: ext[0] ext[1]
    int c_yrows;        // the N - 1 y-rows of an element row: (N - 1) ext[0]
    int c_unit;         // c_yrows + np0 (N - 1)^2: y-rows and x-faces of an element row
    int c_layer;        // c_zplane + nel[1] c_unit (+ c_yrows when y is not periodic)
    int64_t n_nodes;    // face-lattice nodes in all
    // the divisions of the position decode, and the element strides of the
    // copies' offsets (elements of a z-layer, (N+1)^3 values per element)
    UDiv d_layer, d_ext0, d_unit, d_N, d_Nm1;
    int64_t stride_e[3];  // offset of one element step along x, y, z
};

// zplanes_only: enumerate the z-planes alone (the nodes with Z mod N == 0);
// the rest is left to the row-streaming kernel.
inline bool gs_lattice_make(int N, const int nel[3], const int periodic[3], int faces, GsLattice &L,
                            bool zplanes_only = false)
{
    if (N < 1) return false;
    L.N = N;
    L.faces = faces;
    int64_t ext[3], np[3];
    for (int a = 0; a < 3; ++a) {
        if (nel[a] < 1 || (periodic[a] && nel[a] < 2)) return false;
        L.nel[a] = nel[a];
        L.periodic[a] = periodic[a] ? 1 : 0;
        ext[a] = (int64_t)nel[a] * N + (periodic[a] ? 0 : 1);
        np[a] = periodic[a] ? nel[a] : (int64_t)nel[a] + 1;
        if (ext[a] >= INT32_MAX) return false;
        L.ext[a] = (int)ext[a];
    }
    const int64_t c_zplane = ext[0] * ext[1];
    const int64_t c_yrows = zplanes_only ? 0 : (int64_t)(N - 1) * ext[0];
    const int64_t c_unit = zplanes_only ? 0 : c_yrows + np[0] * (N - 1) * (N - 1);
    const int64_t c_layer = c_zplane + nel[1] * c_unit + (periodic[1] ? 0 : c_yrows);
    const int64_t n = (int64_t)nel[2] * c_layer + (periodic[2] ? 0 : c_zplane);
    // lanes decode positions with 32-bit arithmetic
    if (n >= INT32_MAX) return false;
    L.np0 = (int)np[0];
    L.c_zplane = (int)c_zplane;
    L.c_yrows = (int)c_yrows;
    L.c_unit = (int)c_unit;
    L.c_layer = (int)c_layer;
    L.n_nodes = n;
    L.d_layer = udiv_make((uint32_t)c_layer);
    L.d_ext0 = udiv_make((uint32_t)ext[0]);
    L.d_unit = udiv_make((uint32_t)(c_unit > 0 ? c_unit : 1));  // N = 1: z-planes only
    L.d_N = udiv_make((uint32_t)N);
    L.d_Nm1 = udiv_make((uint32_t)(N > 1 ? N - 1 : 1));
    const int64_t P3 = (int64_t)(N + 1) * (N + 1) * (N + 1);
    L.stride_e[0] = P3;
    L.stride_e[1] = P3 * nel[0];
    L.stride_e[2] = P3 * nel[0] * nel[1];
    return true;
}

// Copies along one axis of the lattice coordinate X (see GsLattice): count,
// element coordinate and GLL index of each, in ascending element coordinate;
// `masked` when X lies on a Dirichlet face.
struct AxisCopies {
    int c;
    int e[2], n[2];
    bool masked;
};

__host__ __device__ inline AxisCopies axis_copies(unsigned X, const UDiv &dN, int N, int nel, int periodic, int ext,
                                         int lo_bit, int hi_bit)
{
    AxisCopies a;
    a.masked = false;
    const int q = (int)udiv(dN, X), r = (int)X - q * N;
    if (r != 0) {
        a.c = 1; a.e[0] = q; a.n[0] = r; a.e[1] = q; a.n[1] = r;
    } else if (X == 0) {
        a.e[0] = 0; a.n[0] = 0;
        if (periodic) {
            a.c = 2; a.e[1] = nel - 1; a.n[1] = N;
        } else {
            a.c = 1; a.e[1] = 0; a.n[1] = 0; a.masked = lo_bit != 0;
        }
    } else if (!periodic && (int)X == ext - 1) {
        a.c = 1; a.e[0] = nel - 1; a.n[0] = N; a.e[1] = nel - 1; a.n[1] = N; a.masked = hi_bit != 0;
    } else {
        a.c = 2; a.e[0] = q - 1; a.n[0] = N; a.e[1] = q; a.n[1] = 0;
    }
    return a;
}

// Lattice position (X, Y, Z) of face-lattice node u < L.n_nodes, in the
// enumeration GsLattice describes.
__host__ __device__ inline void gs_lattice_pos(const GsLattice &L, unsigned u, unsigned &X, unsigned &Y, unsigned &Z)
{
    const unsigned N = (unsigned)L.N, ext0 = (unsigned)L.ext[0];
    const unsigned zl = udiv(L.d_layer, u), r = u - zl * (unsigned)L.c_layer;
    if (r < (unsigned)L.c_zplane) {
        Z = zl * N;
        Y = udiv(L.d_ext0, r);
        X = r - Y * ext0;
        return;
    }
    const unsigned r1 = r - (unsigned)L.c_zplane;
    const unsigned yl = udiv(L.d_unit, r1), r2 = r1 - yl * (unsigned)L.c_unit;
    if (r2 < (unsigned)L.c_yrows) {
        const unsigned zo = udiv(L.d_ext0, r2);
        Z = zl * N + 1 + zo;
        Y = yl * N;
        X = r2 - zo * ext0;
    } else {
        const unsigned b = r2 - (unsigned)L.c_yrows, Nm1 = N - 1;
        const unsigned v1 = udiv(L.d_Nm1, b), jj = b - v1 * Nm1;
        const unsigned q = udiv(L.d_Nm1, v1), kk = v1 - q * Nm1;
        X = q * N;
        Y = yl * N + 1 + jj;
        Z = zl * N + 1 + kk;
    }
}

// The copies of the node at (X, Y, Z): per axis its copies, and the local
// offset of copy q = (qz * 2 + qy) * 2 + qx, defined for qz < cz.c,
// qy < cy.c and qx < cx.c; these ascend with q.  `cnt` copies in all;
// `masked` when the node lies on a Dirichlet face.
struct LatticeCopies {
    AxisCopies cx, cy, cz;
    int64_t a[8];
    int cnt;
    bool masked;
};

__host__ __device__ inline LatticeCopies gs_lattice_copies(const GsLattice &L, unsigned X, unsigned Y, unsigned Z)
{
    const int N = L.N;
    LatticeCopies c;
    c.cx = axis_copies(X, L.d_N, N, L.nel[0], L.periodic[0], L.ext[0], L.faces & 1, L.faces & 2);
    c.cy = axis_copies(Y, L.d_N, N, L.nel[1], L.periodic[1], L.ext[1], L.faces & 4, L.faces & 8);
    c.cz = axis_copies(Z, L.d_N, N, L.nel[2], L.periodic[2], L.ext[2], L.faces & 16, L.faces & 32);
    const AxisCopies &cx = c.cx, &cy = c.cy, &cz = c.cz;
    c.masked = cx.masked || cy.masked || cz.masked;
    c.cnt = cx.c * cy.c * cz.c;
    const int P = N + 1;
    // offset of a copy = sum over the axes of (element coordinate x element
    // stride + GLL index x index stride)
    int64_t ox[2], oy[2], oz[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        ox[q] = (int64_t)cx.e[q] * L.stride_e[0] + cx.n[q];
        oy[q] = (int64_t)cy.e[q] * L.stride_e[1] + cy.n[q] * P;
        oz[q] = (int64_t)cz.e[q] * L.stride_e[2] + cz.n[q] * P * P;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) c.a[q] = oz[q >> 2] + oy[(q >> 1) & 1] + ox[q & 1];
    return c;
}

// The fused CG update's view of the same copies, element by element: the
// copies of a face node along one axis, for an element at coordinate c
// of nel: on its low face (GLL index 0) and on its high face (index N), as
// in GsLattice: count, and per copy the element offset from c and the GLL
// index, in ascending element coordinate; `masked` on a Dirichlet face.
// Off the faces a node has one copy, itself.
struct AxisSide {
    int c;
    int de[2], n[2];
    bool masked;
};
struct ElemAxis {
    AxisSide lo, hi;
};
template <int N>
__host__ __device__ inline ElemAxis elem_axis(int c, int nel, int periodic, int lo_bit, int hi_bit)
{
    ElemAxis a;
    a.lo.masked = a.hi.masked = false;
    if (c > 0) {
        a.lo.c = 2; a.lo.de[0] = -1; a.lo.n[0] = N; a.lo.de[1] = 0; a.lo.n[1] = 0;
    } else if (periodic) {
        a.lo.c = 2; a.lo.de[0] = 0; a.lo.n[0] = 0; a.lo.de[1] = nel - 1; a.lo.n[1] = N;
    } else {
        a.lo.c = 1; a.lo.de[0] = a.lo.de[1] = 0; a.lo.n[0] = a.lo.n[1] = 0; a.lo.masked = lo_bit != 0;
    }
    if (c < nel - 1) {
        a.hi.c = 2; a.hi.de[0] = 0; a.hi.n[0] = N; a.hi.de[1] = 1; a.hi.n[1] = 0;
    } else if (periodic) {
        a.hi.c = 2; a.hi.de[0] = -(nel - 1); a.hi.n[0] = 0; a.hi.de[1] = 0; a.hi.n[1] = N;
    } else {
        a.hi.c = 1; a.hi.de[0] = a.hi.de[1] = 0; a.hi.n[0] = a.hi.n[1] = N; a.hi.masked = hi_bit != 0;
    }
    return a;
}

// This lane's copies along one axis (GLL index n): count, and per copy the
// offset from the lane's own value (element offset x element stride + GLL
// index change x index stride), in 32 bits (the caller keeps the E-vector
// below 2^31 values).
struct LaneAxis {
    int c;
    int d[2];
    bool masked;
};
template <int N>
__host__ __device__ inline LaneAxis lane_axis(const ElemAxis &a, int n, int estride, int nstride)
{
    LaneAxis l;
    const AxisSide &sd = n == 0 ? a.lo : a.hi;
    const bool face = n == 0 || n == N;
    l.c = face ? sd.c : 1;
    l.masked = face && sd.masked;
#pragma unroll
    for (int q = 0; q < 2; ++q) l.d[q] = face ? sd.de[q] * estride + (sd.n[q] - n) * nstride : 0;
    return l;
}

}  // namespace sem
