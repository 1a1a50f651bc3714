// Host check of the plan-free gather-scatter's enumeration (lattice.hpp):
// on lattices of every periodicity, order, Dirichlet face set and a few
// sizes, every lane index t < n_nodes decodes to a distinct node of the face
// lattice, all of them are met, and the
// copies of each node are exactly the local indices at its position, in
// ascending order, with every element-face local index met once, and the
// element layers in z come one after another; and that the fused CG
// update's per-element copy rule agrees with the lattice rule node by node.  Prints
// "OK <cases>" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2109_03592_amd/csrc/lattice.hpp"

using namespace sem;

static int fail_case(const char *what, int N, const int *nel, const int *per, long t)
{
    std::printf("FAIL %s N=%d nel=%dx%dx%d periodic=%d%d%d t=%ld\n", what, N, nel[0], nel[1], nel[2], per[0], per[1],
                per[2], t);
    return 1;
}

static int check(int N, const int nel[3], const int per[3], int faces)
{
    GsLattice L{};
    const bool ok = gs_lattice_make(N, nel, per, faces, L);
    const bool expect = !(per[0] && nel[0] < 2) && !(per[1] && nel[1] < 2) && !(per[2] && nel[2] < 2);
    if (ok != expect) return fail_case("make", N, nel, per, -1);
    if (!ok) return 0;
    const int P = N + 1;
    long ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = (long)nel[a] * N + (per[a] ? 0 : 1);
    long nface = 0;
    for (long Z = 0; Z < ext[2]; ++Z)
        for (long Y = 0; Y < ext[1]; ++Y)
            for (long X = 0; X < ext[0]; ++X)
                if (X % N == 0 || Y % N == 0 || Z % N == 0) ++nface;
    if (nface != L.n_nodes) return fail_case("count", N, nel, per, -1);
    const long E = (long)nel[0] * nel[1] * nel[2], nloc = E * P * P * P;
    std::vector<unsigned char> seen((size_t)(ext[0] * ext[1] * ext[2]), 0), cover((size_t)nloc, 0);
    long prev_layer = 0;
    for (long t = 0; t < L.n_nodes; ++t) {
        unsigned X, Y, Z;
        gs_lattice_pos(L, (unsigned)t, X, Y, Z);
        if (X >= ext[0] || Y >= ext[1] || Z >= ext[2]) return fail_case("range", N, nel, per, t);
        if (!(X % N == 0 || Y % N == 0 || Z % N == 0)) return fail_case("not a face node", N, nel, per, t);
        const long gid = X + ext[0] * (Y + ext[1] * (long)Z);
        if (seen[gid]++) return fail_case("met twice", N, nel, per, t);
        // element layers in z one after another
        const long layer = Z / N;
        if (layer < prev_layer) return fail_case("layer order", N, nel, per, t);
        prev_layer = layer;
        const LatticeCopies c = gs_lattice_copies(L, X, Y, Z);
        const unsigned pos[3] = {X, Y, Z};
        const AxisCopies *ax[3] = {&c.cx, &c.cy, &c.cz};
        bool masked = false;
        int cnt = 1;
        for (int a = 0; a < 3; ++a) {
            const bool lo = !per[a] && pos[a] == 0, hi = !per[a] && (long)pos[a] == ext[a] - 1;
            masked = masked || (lo && (faces >> (2 * a) & 1)) || (hi && (faces >> (2 * a + 1) & 1));
            cnt *= (pos[a] % N == 0 && !lo && !hi) ? 2 : 1;
        }
        if (c.masked != masked || c.cnt != cnt) return fail_case("count or mask", N, nel, per, t);
        long last = -1;
        for (int q = 0; q < 8; ++q) {
            const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
            if (!(qz < c.cz.c && qy < c.cy.c && qx < c.cx.c)) continue;
            const long o = c.a[q];
            if (o < 0 || o >= nloc || o <= last) return fail_case("copy offset", N, nel, per, t);
            last = o;
            const long e = o / (P * P * P), l = o % (P * P * P);
            const long ijk[3] = {l % P, (l / P) % P, l / (P * P)};
            const long ec[3] = {e % nel[0], (e / nel[0]) % nel[1], e / ((long)nel[0] * nel[1])};
            for (int a = 0; a < 3; ++a) {
                long p = ec[a] * N + ijk[a];
                if (per[a]) p %= (long)nel[a] * N;
                if (p != (long)pos[a]) return fail_case("copy position", N, nel, per, t);
            }
            if (cover[o]++) return fail_case("copy met twice", N, nel, per, t);
        }
        (void)ax;
    }
    for (long o = 0; o < nloc; ++o) {
        const long l = o % (P * P * P);
        const long i = l % P, j = (l / P) % P, k = l / (P * P);
        const bool face = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
        if (cover[o] != (face ? 1 : 0)) return fail_case("cover", N, nel, per, o);
    }
    return 0;
}

// The fused CG update's per-element copy rule (elem_axis, lane_axis) against
// the lattice rule: for every element-face node, the same mask, the same
// number of copies and the same offsets in the same order.
template <int N>
static int check_update_rule(const int nel[3], const int per[3], int faces)
{
    GsLattice L{};
    if (!gs_lattice_make(N, nel, per, faces, L)) return 0;
    constexpr int P = N + 1, P2 = P * P, P3 = P2 * P;
    const int sy = nel[0] * P3, sz = nel[0] * nel[1] * P3;
    long ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = (long)nel[a] * N + (per[a] ? 0 : 1);
    for (int ez = 0; ez < nel[2]; ++ez)
        for (int ey = 0; ey < nel[1]; ++ey)
            for (int ex = 0; ex < nel[0]; ++ex) {
                const ElemAxis ax = elem_axis<N>(ex, nel[0], per[0], faces & 1, faces & 2);
                const ElemAxis ay = elem_axis<N>(ey, nel[1], per[1], faces & 4, faces & 8);
                const ElemAxis az = elem_axis<N>(ez, nel[2], per[2], faces & 16, faces & 32);
                const long e = ex + (long)nel[0] * (ey + (long)nel[1] * ez);
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j)
                        for (int i = 0; i < P; ++i) {
                            if (!(i == 0 || i == N || j == 0 || j == N || k == 0 || k == N)) continue;
                            const long o = e * P3 + i + (long)P * j + (long)P2 * k;
                            const LaneAxis cx = lane_axis<N>(ax, i, P3, 1);
                            const LaneAxis cy = lane_axis<N>(ay, j, sy, P);
                            const LaneAxis cz = lane_axis<N>(az, k, sz, P2);
                            unsigned pos[3] = {(unsigned)(ex * N + i), (unsigned)(ey * N + j), (unsigned)(ez * N + k)};
                            for (int a = 0; a < 3; ++a)
                                if (per[a]) pos[a] %= (unsigned)ext[a];
                            const LatticeCopies c = gs_lattice_copies(L, pos[0], pos[1], pos[2]);
                            const bool masked = cx.masked || cy.masked || cz.masked;
                            const int cnt = cx.c * cy.c * cz.c;
                            if (masked != c.masked || cnt != c.cnt)
                                return fail_case("update rule: mask or count", N, nel, per, o);
                            for (int q = 0; q < 8; ++q) {
                                const int qz = q >> 2, qy = (q >> 1) & 1, qx = q & 1;
                                if (!(qz < cz.c && qy < cy.c && qx < cx.c)) continue;
                                const long a = o + (cz.d[qz] + cy.d[qy] + cx.d[qx]);
                                if (a != c.a[q]) return fail_case("update rule: copy offset", N, nel, per, o);
                            }
                        }
            }
    return 0;
}

template <int N>
static int check_update_rules(int &cases)
{
    const int sizes[][3] = {{1, 1, 1}, {2, 1, 3}, {3, 2, 2}, {2, 3, 4}};
    for (const auto &nel : sizes)
        for (int pm = 0; pm < 8; ++pm) {
            const int per[3] = {pm & 1, (pm >> 1) & 1, (pm >> 2) & 1};
            for (int faces : {0, 63, 0b010110, 0b101001}) {
                if (check_update_rule<N>(nel, per, faces)) return 1;
                ++cases;
            }
        }
    return 0;
}

int main()
{
    int cases = 0;
    const int sizes[][3] = {{1, 1, 1}, {2, 1, 3}, {1, 3, 2}, {3, 2, 2}, {2, 3, 4}, {4, 2, 1}};
    for (int N = 1; N <= 12; ++N)
        for (const auto &nel : sizes)
            for (int pm = 0; pm < 8; ++pm) {
                const int per[3] = {pm & 1, (pm >> 1) & 1, (pm >> 2) & 1};
                for (int faces : {0, 63, 0b010110, 0b101001}) {
                    if (check(N, nel, per, faces)) return 1;
                    ++cases;
                }
            }
    const int big[3] = {24, 24, 6}, pipe_per[3] = {0, 0, 1};
    if (check(7, big, pipe_per, 0b001111)) return 1;
    const int big9[3] = {12, 12, 8};
    if (check(9, big9, pipe_per, 0b001111)) return 1;
    cases += 2;
    if (check_update_rules<3>(cases) || check_update_rules<4>(cases) || check_update_rules<5>(cases) ||
        check_update_rules<7>(cases) || check_update_rules<9>(cases) || check_update_rules<12>(cases))
        return 1;
    std::printf("OK %d\n", cases);
    return 0;
}
