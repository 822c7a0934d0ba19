// Per-vertex contribution tables and per-cell delta tables (host code).
//
// A lattice vertex sees the 2^n cells around it (2x2 quadrant in 2D, 2x2x2
// octant block in 3D).  Its contribution to each descriptor is the share of
// the cubical cells of that neighbourhood it owns: all of the vertex, half of
// each of its edges, a quarter of each face, an eighth of each cube (Table 1 and
// Table 2 of the paper, columns V, E, F, Vox).  The tables below are built by
// counting exactly those shares for every one of the 16 (2D) or 256 (3D) masks,
// scaled to integers:
//   2D: {4*EC, 2*perimeter, 4*area}, EC = V - E/2 + F/4 (8-C); for 4-C the
//       vertex count V is the number of 4-connected pieces in the quadrant
//       (Table 1, "V (4-C)" column).
//   3D: {8*EC, 2*crease, 4*surface, 8*volume}, EC = V - E/2 + F/4 - C/8 (26-C);
//       6-C uses the share of the face-adjacency complex (active cells,
//       face-adjacent pairs, full axis-plane 2x2 squares, full 2x2x2 cube).
//
// Per-cell delta tables: when cell p enters the filtration (cells ordered by
// level, ties by position), every vertex at a corner of p changes from its
// mask without p to its mask with p; the change of p is the sum of those
// differences over p's 2^n corners, i.e. the paper's "born"/"dies" increments
// of Algorithm 1 telescoped per cell.  For 2D the 8 neighbours of p decide all
// four corner masks, so the whole delta is one table lookup.
#include "ecc_internal.h"

#include <algorithm>
#include <array>
#include <cstring>
#include <vector>

namespace ecc {

// ---------------------------------------------------------------------------
// 2D
// ---------------------------------------------------------------------------
// quadrant mask bits: 0 = (i-1,j-1), 1 = (i-1,j), 2 = (i,j-1), 3 = (i,j)
// the four lattice edges at the vertex, as the two pixels beside each half-edge
static const int kEdges2[4][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}};

static int pieces4(int m) {
    // 4-connected pieces of the active pixels of a quadrant: only the two
    // diagonal pairs {0,3} and {1,2} without their connectors split
    int n = __builtin_popcount(m);
    if (n == 2 && (m == 0x9 || m == 0x6)) return 2;
    return n > 0 ? 1 : 0;
}

void vertex_table_2d(int connectivity, int32_t out[16][4]) {
    for (int m = 0; m < 16; ++m) {
        int v = m ? 1 : 0;
        if (connectivity == 4) v = pieces4(m);
        int e = 0, per = 0;
        for (auto &ed : kEdges2) {
            int a = m >> ed[0] & 1, b = m >> ed[1] & 1;
            e += (a | b);
            per += (a ^ b);
        }
        int f = __builtin_popcount(m);
        out[m][0] = 4 * v - 2 * e + f;  // 4 * (V - E/2 + F/4)
        out[m][1] = per;                // 2 * (per/2)
        out[m][2] = f;                  // 4 * (F/4)
        out[m][3] = 0;
    }
}

// neighbour order of the 8-bit per-cell pattern (row offset, column offset)
const int kNbr2[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};

// kappa of a 2x2 block of cells around a lattice edge (the crease measure of
// Table 2's perimeter column): 1 for one or three cells in, 2 for two cells on
// a diagonal, else 0.  Mask bits as for the 2D quadrant (a*2 + b).
static int kappa_of_mask(int m) {
    const int n = __builtin_popcount(m);
    if (n == 1 || n == 3) return 1;
    if (n == 2 && (m == 6 || m == 9)) return 2;
    return 0;
}

void crease_delta_table_2d(int32_t delta[256]) {
    // the four blocks at the corners (cr, cc) of pixel p = (0,0), as in
    // cell_delta_table_2d
    for (int pat = 0; pat < 256; ++pat) {
        auto precedes = [&](int dr, int dc) -> int {
            for (int k = 0; k < 8; ++k)
                if (kNbr2[k][0] == dr && kNbr2[k][1] == dc) return pat >> k & 1;
            return 0;
        };
        int32_t s = 0;
        for (int cr = 0; cr < 2; ++cr)
            for (int cc = 0; cc < 2; ++cc) {
                int m0 = 0, pbit = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const int dr = cr - 1 + a, dc = cc - 1 + b, bit = a * 2 + b;
                        if (dr == 0 && dc == 0)
                            pbit = bit;
                        else if (precedes(dr, dc))
                            m0 |= 1 << bit;
                    }
                s += kappa_of_mask(m0 | 1 << pbit) - kappa_of_mask(m0);
            }
        delta[pat] = s;
    }
}

int vertex_class_2d(int m) {
    switch (__builtin_popcount(m)) {
    case 0: return -1;
    case 1: return 0;
    case 2: return (m == 6 || m == 9) ? 2 : 1;  // pixels on a diagonal: b0 b3 or b1 b2
    case 3: return 3;
    default: return 4;
    }
}

// 3D octant classes: the orbits of the 256 masks (bit dx + 2dy + 4dz) under the
// 48 symmetries of the cube (axis permutations and reflections), the rows of
// Table 2.  The 21 non-empty orbits are numbered by (number of voxels, smallest
// mask in the orbit); the empty mask is -1.
int octant_class_3d(int mask) {
    static const std::array<int8_t, 256> table = [] {
        std::array<int, 256> rep{};
        const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        for (int m = 0; m < 256; ++m) {
            int best = 256;
            for (const auto &pm : perms)
                for (int f = 0; f < 8; ++f) {
                    int img = 0;
                    for (int b = 0; b < 8; ++b) {
                        if (!(m >> b & 1)) continue;
                        const int c[3] = {b & 1, b >> 1 & 1, b >> 2 & 1};
                        int nb = 0;
                        for (int a = 0; a < 3; ++a) nb |= (c[pm[a]] ^ (f >> a & 1)) << a;
                        img |= 1 << nb;
                    }
                    best = std::min(best, img);
                }
            rep[m] = best;
        }
        std::vector<int> reps;
        for (int m = 1; m < 256; ++m)
            if (rep[m] == m) reps.push_back(m);
        std::sort(reps.begin(), reps.end(), [](int a, int b) {
            const int pa = __builtin_popcount(a), pb = __builtin_popcount(b);
            return pa != pb ? pa < pb : a < b;
        });
        std::array<int8_t, 256> t{};
        t[0] = -1;
        for (int m = 1; m < 256; ++m)
            t[m] = (int8_t)(std::find(reps.begin(), reps.end(), rep[m]) - reps.begin());
        return t;
    }();
    return table[mask & 255];
}

// For each corner c = cx + 2 cy + 4 cz of a voxel and each octant mask m of
// the 2x2x2 block at that corner (the voxel is bit 7 - c of it): the class of
// m and of m without the voxel (0xFF when that block is empty).
void class_transitions_3d(uint16_t out[8][256]) {
    for (int c = 0; c < 8; ++c)
        for (int m = 0; m < 256; ++m) {
            const int cn = octant_class_3d(m), co = octant_class_3d(m & ~(1 << (7 - c)));
            out[c][m] = (uint16_t)((cn < 0 ? 0 : cn) | (co < 0 ? 0xFF : co) << 8);
        }
}

void class_delta_table_2d(int32_t delta[256][5]) {
    // the four vertices at the corners (cr, cc) of pixel p = (0,0), as in
    // cell_delta_table_2d: one class leaves (unless the quadrant was empty)
    // and one arrives
    for (int pat = 0; pat < 256; ++pat) {
        auto precedes = [&](int dr, int dc) -> int {
            for (int k = 0; k < 8; ++k)
                if (kNbr2[k][0] == dr && kNbr2[k][1] == dc) return pat >> k & 1;
            return 0;
        };
        int32_t s[5] = {0, 0, 0, 0, 0};
        for (int cr = 0; cr < 2; ++cr)
            for (int cc = 0; cc < 2; ++cc) {
                int m0 = 0, pbit = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const int dr = cr - 1 + a, dc = cc - 1 + b, bit = a * 2 + b;
                        if (dr == 0 && dc == 0)
                            pbit = bit;
                        else if (precedes(dr, dc))
                            m0 |= 1 << bit;
                    }
                const int c0 = vertex_class_2d(m0), c1 = vertex_class_2d(m0 | 1 << pbit);
                if (c0 >= 0) --s[c0];
                ++s[c1];
            }
        for (int c = 0; c < 5; ++c) delta[pat][c] = s[c];
    }
}

int pattern_of_index(int n) {
    int p = 0;
    for (int i = 0; i < 4; ++i) {
        p |= ((n >> i) & 1) << (2 * i);            // index bit i: neighbour 2i
        p |= ((n >> (4 + i)) & 1) << (2 * i + 1);  // index bit 4+i: neighbour 2i+1
    }
    return p;
}

void cell_delta_table_2d(int connectivity, int32_t delta[256][3]) {
    int32_t T[16][4];
    vertex_table_2d(connectivity, T);
    // for the vertex at corner (cr, cc) in {0,1}^2 of pixel p = (0,0) the
    // quadrant holds pixels (cr-1+a, cc-1+b), a,b in {0,1}, at bit a*2+b
    for (int pat = 0; pat < 256; ++pat) {
        auto precedes = [&](int dr, int dc) -> int {
            for (int k = 0; k < 8; ++k)
                if (kNbr2[k][0] == dr && kNbr2[k][1] == dc) return pat >> k & 1;
            return 0;
        };
        int32_t s[3] = {0, 0, 0};
        for (int cr = 0; cr < 2; ++cr)
            for (int cc = 0; cc < 2; ++cc) {
                int m0 = 0, pbit = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        int dr = cr - 1 + a, dc = cc - 1 + b;
                        int bit = a * 2 + b;
                        if (dr == 0 && dc == 0)
                            pbit = bit;
                        else if (precedes(dr, dc))
                            m0 |= 1 << bit;
                    }
                int m1 = m0 | 1 << pbit;
                for (int c = 0; c < 3; ++c) s[c] += T[m1][c] - T[m0][c];
            }
        // shares were scaled by 4 (EC, area) and 2 (perimeter); per-cell sums are exact
        delta[pat][0] = s[0] / 4;
        delta[pat][1] = s[1] / 2;
        delta[pat][2] = s[2] / 4;
    }
}

// ---------------------------------------------------------------------------
// 3D
// ---------------------------------------------------------------------------
// octant bit (dx + 2dy + 4dz), offsets in {0,1}^3 from the lower corner
void vertex_table_3d(int connectivity, int32_t out[256][4]) {
    for (int m = 0; m < 256; ++m) {
        auto act = [&](int b) { return m >> b & 1; };
        int c = __builtin_popcount(m);
        // 12 faces at the vertex: octant pairs that differ along one axis
        int f_touch = 0, f_bound = 0;
        for (int b = 0; b < 8; ++b)
            for (int a = 0; a < 3; ++a)
                if (!(b >> a & 1)) {
                    int u = act(b), w = act(b | 1 << a);
                    f_touch += (u | w);
                    f_bound += (u ^ w);
                }
        // 6 edges at the vertex: the 4 octants sharing one coordinate value
        int e_touch = 0, crease2 = 0;
        for (int a = 0; a < 3; ++a) {
            int o1 = (a + 1) % 3, o2 = (a + 2) % 3;
            for (int s = 0; s < 2; ++s) {
                int q0 = s << a, q1 = q0 | 1 << o1, q2 = q1 | 1 << o2, q3 = q0 | 1 << o2;
                int k0 = act(q0), k1 = act(q1), k2 = act(q2), k3 = act(q3);
                int n = k0 + k1 + k2 + k3;
                e_touch += n > 0;
                int kappa = (n == 1 || n == 3) ? 1 : ((n == 2 && k0 == k2) ? 2 : 0);
                crease2 += kappa;  // 2 * (kappa / 2)
            }
        }
        int v = m ? 1 : 0;
        int ec8;
        if (connectivity == 6) {
            // share of the face-adjacency complex: each active cell is a vertex
            // seen by 8 lattice vertices, each active face-adjacent pair by 4,
            // each full axis-plane square by 2, the full cube by 1
            int pairs = 0, squares = 0;
            for (int b = 0; b < 8; ++b)
                for (int a = 0; a < 3; ++a)
                    if (!(b >> a & 1)) pairs += act(b) & act(b | 1 << a);
            for (int a = 0; a < 3; ++a)  // squares normal to axis a
                for (int s = 0; s < 2; ++s) {
                    int o1 = (a + 1) % 3, o2 = (a + 2) % 3;
                    int q0 = s << a;
                    squares += act(q0) & act(q0 | 1 << o1) & act(q0 | 1 << o2) &
                               act(q0 | 1 << o1 | 1 << o2);
                }
            int cube = (m == 255);
            ec8 = c - 2 * pairs + 4 * squares - 8 * cube;
        } else {
            ec8 = 8 * v - 4 * e_touch + 2 * f_touch - c;  // 8 * (V - E/2 + F/4 - C/8)
        }
        out[m][0] = ec8;
        out[m][1] = crease2;
        out[m][2] = f_bound;  // 4 * (faces/4)
        out[m][3] = c;        // 8 * (C/8)
    }
}

}  // namespace ecc

extern "C" ecc_status ecc_vertex_table(int32_t ndim, int32_t connectivity, int32_t *out) {
    if (!out) return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_table: out is NULL");
    if (ndim == 2) {
        if (connectivity == 0) connectivity = 8;
        if (connectivity != 8 && connectivity != 4)
            return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_table: 2D connectivity must be 8 or 4");
        int32_t t[16][4];
        ecc::vertex_table_2d(connectivity, t);
        std::memcpy(out, t, sizeof(t));
        return ECC_OK;
    }
    if (ndim == 3) {
        if (connectivity == 0) connectivity = 26;
        if (connectivity != 26 && connectivity != 6)
            return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_table: 3D connectivity must be 26 or 6");
        int32_t t[256][4];
        ecc::vertex_table_3d(connectivity, t);
        std::memcpy(out, t, sizeof(t));
        return ECC_OK;
    }
    return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_table: ndim must be 2 or 3");
}

extern "C" ecc_status ecc_vertex_class_table(int32_t ndim, int32_t *out) {
    if (!out) return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_class_table: out is NULL");
    if (ndim == 2) {
        for (int m = 0; m < 16; ++m) out[m] = ecc::vertex_class_2d(m);
        return ECC_OK;
    }
    if (ndim == 3) {
        for (int m = 0; m < 256; ++m) out[m] = ecc::octant_class_3d(m);
        return ECC_OK;
    }
    return ecc::fail(ECC_ERR_INVALID_ARG, "ecc_vertex_class_table: ndim must be 2 or 3");
}
