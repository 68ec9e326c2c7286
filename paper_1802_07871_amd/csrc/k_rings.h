// k_rings.h -- ring statistics of the carbon bond graph: shortest-path rings
// (Franzblau 1991) of at most RING_MAX members, the bonds on no ring (chain
// bonds) and the in-plane orientation of every 6-membered ring, the analysis
// the paper draws for its growth and anneal runs (rings by size, chains, a
// 6-ring hue that repeats every 60 degrees).
//
// Bonds: two C atoms with an image of one within r_bond of the other, taken
// from the covalent list (complete up to S_CC at the current positions), one
// edge per atom pair.  Rings: one thread per C atom enumerates, by depth-first
// search, the simple cycles whose smallest user index is its own atom, each
// once (second vertex below the last), and keeps those with no shortcut: for
// every two ring vertices at ring distance d (at most 4), no path of fewer
// than d bonds joins them in the whole graph.  The cell must be at least
// max_size * r_bond wide in every periodic direction, so neither a cycle nor
// a shortcut can wind around it.
#pragma once
#include "ctbop_dev.h"
#include "k_tersoff.h"

namespace ctbop {

constexpr int RING_DEG = 12;       // C neighbours per atom at most
constexpr int RING_MAX = 8;        // largest ring
constexpr int RING_C = 1;          // type index of carbon
constexpr int CLOSE_ONLY = 0x80;   // search-cursor flag: this path atom may only close the ring

// counter slots
enum : int {
    RC_BONDS = 9,                  // 0..8: rings by size
    RC_CHAIN = 10,
    RC_LISTED = 11,                // rings found (listed up to the caller's capacity)
    RC_HIST = 12,                  // 6-rings that entered the histogram
    RC_OVERFLOW = 13,              // atoms with more than RING_DEG C neighbours
    RC_N = 16
};

struct RingWs {
    uint32_t *adj;                 // [npad * RING_DEG] covalent-list entries (row | image code) of the C neighbours
    int *deg;                      // [npad]
    uint32_t *mark;                // [npad * RING_DEG] 1: that bond lies on a ring
    unsigned long long *cnt;       // [RC_N]
    unsigned long long *hist;      // [nbins]
    int32_t *list;                 // [cap * 9] (size, user indices in ring order, -1 padding) or null
    double *orient;                // [cap] (6-rings: orientation in degrees; others: -1) or null
    long long cap;
};

struct RingCfg {
    double rb2;                    // r_bond^2
    int max_size;
    int nbins;
    double n[3], u[3], w[3];       // plane normal, reference direction in the plane, n x u
    double cos_tilt_min;           // rings whose normal is within the tilt limit; < -1: no limit
};

// C neighbours of every C atom and the cleared bond marks
__global__ void __launch_bounds__(TILE) k_ring_adj(const Tile *tiles, Seg *segs, RingWs W, RingCfg c)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double4 dtab[NCODE];
    load_dtab2<double>(S, dtab);
    const int s = T.row0 + threadIdx.x;
    if (s >= S.npad) return;
    uint32_t *row = W.adj + (size_t)s * RING_DEG;
    int nd = 0;
    if (s < S.n) {
        const double4 li = S.xs64[s];
        if ((int)li.w == RING_C) {
            const size_t rl = (size_t)s * S.Ws;
            const int ns = S.scnt[s];
            for (int e = 0; e < ns; e++) {
                const uint32_t ent = S.sidx[rl + e];
                const int j = (int)(ent & J_MASK);
                if (j == s) continue;
                const double4 lj = S.xs64[j];
                if ((int)lj.w != RING_C) continue;
                const R3<double> d = pair_vec<double>(li, lj, dtab[ent >> CODE_SHIFT]);
                if (d.x * d.x + d.y * d.y + d.z * d.z >= c.rb2) continue;
                bool dup = false;
                for (int k = 0; k < nd && k < RING_DEG; k++) dup |= (row[k] & J_MASK) == (uint32_t)j;
                if (dup) continue;
                if (nd < RING_DEG) row[nd] = ent;
                nd++;
            }
            if (nd > RING_DEG) {
                atomicAdd(&W.cnt[RC_OVERFLOW], 1ull);
                nd = RING_DEG;
            }
        }
    }
    W.deg[s] = nd;
    for (int k = 0; k < RING_DEG; k++) W.mark[(size_t)s * RING_DEG + k] = 0u;
}

__device__ __forceinline__ int ring_nb(const RingWs &W, int v, int k)
{
    return (int)(W.adj[(size_t)v * RING_DEG + k] & J_MASK);
}

__device__ bool ring_adjacent(const RingWs &W, int a, int b)
{
    const int da = W.deg[a];
    for (int k = 0; k < da; k++)
        if (ring_nb(W, a, k) == b) return true;
    return false;
}

// a path of fewer than d bonds (2 <= d <= 4) from a to b?
__device__ bool ring_shortcut(const RingWs &W, int a, int b, int d)
{
    if (ring_adjacent(W, a, b)) return true;
    if (d <= 2) return false;
    const int da = W.deg[a], db = W.deg[b];
    for (int k = 0; k < da; k++) {
        const int cv = ring_nb(W, a, k);
        if (ring_adjacent(W, cv, b)) return true;                 // a - cv - b
        if (d <= 3) continue;
        for (int m = 0; m < db; m++) {
            const int e = ring_nb(W, b, m);
            if (e != a && e != cv && ring_adjacent(W, cv, e)) return true;   // a - cv - e - b
        }
    }
    return false;
}

__device__ __forceinline__ R3<double> ring_bond(const Seg &S, const RingWs &W, const double4 *dtab, int v, int k)
{
    const uint32_t ent = W.adj[(size_t)v * RING_DEG + k];
    return pair_vec<double>(S.xs64[v], S.xs64[ent & J_MASK], dtab[ent >> CODE_SHIFT]);
}

// Orientation (degrees in [0, 60)) and |cos| of the tilt of the 6-ring whose
// vertices, unwrapped along its bonds, are p[0..5].
__device__ double ring_orientation(const R3<double> *p, const RingCfg &c, double &cos_tilt)
{
    double cx = 0, cy = 0, cz = 0;
    for (int k = 0; k < 6; k++) {
        cx += p[k].x;
        cy += p[k].y;
        cz += p[k].z;
    }
    cx /= 6.0;
    cy /= 6.0;
    cz /= 6.0;
    double nx = 0, ny = 0, nz = 0;
    for (int k = 0; k < 6; k++) {
        const int l = (k + 1) % 6;
        const double ax = p[k].x - cx, ay = p[k].y - cy, az = p[k].z - cz;
        const double bx = p[l].x - cx, by = p[l].y - cy, bz = p[l].z - cz;
        nx += ay * bz - az * by;
        ny += az * bx - ax * bz;
        nz += ax * by - ay * bx;
    }
    cos_tilt = ::fabs(nx * c.n[0] + ny * c.n[1] + nz * c.n[2]) / ::sqrt(nx * nx + ny * ny + nz * nz);
    double zr = 0.0, zi = 0.0;
    for (int k = 0; k < 3; k++) {
        const double dx = p[k + 3].x - p[k].x, dy = p[k + 3].y - p[k].y, dz = p[k + 3].z - p[k].z;
        const double th = ::atan2(dx * c.w[0] + dy * c.w[1] + dz * c.w[2], dx * c.u[0] + dy * c.u[1] + dz * c.u[2]);
        double sn, cs;
        ::sincos(6.0 * th, &sn, &cs);
        zr += cs;
        zi += sn;
    }
    double ang = ::atan2(zi, zr) * (180.0 / M_PI) / 6.0;
    if (ang < 0.0) ang += 60.0;
    return ang;
}

// One thread per C atom: the rings whose smallest user index is this atom.
// The search path and its neighbour cursors live in LDS, one column per thread.
__global__ void __launch_bounds__(TILE) k_rings(const Tile *tiles, Seg *segs, RingWs W, RingCfg c)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double4 dtab[NCODE];
    __shared__ int lpath[RING_MAX][TILE];
    __shared__ uint8_t lit[RING_MAX][TILE];
    load_dtab2<double>(S, dtab);
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n || W.deg[s] < 2) return;
    const int tx = threadIdx.x;
    const int u0 = S.perm[s];
    int depth = 0;
    lpath[0][tx] = s;
    lit[0][tx] = 0;
    while (depth >= 0) {
        const int v = lpath[depth][tx];
        const int cur = lit[depth][tx];
        const int it = cur & ~CLOSE_ONLY;
        if (it >= W.deg[v]) {
            depth--;
            continue;
        }
        lit[depth][tx] = (uint8_t)(cur + 1);
        const int wv = ring_nb(W, v, it);
        if ((cur & CLOSE_ONLY) && wv != s) continue;
        if (wv == s) {
            // a cycle of depth + 1 atoms, listed once: second vertex below the last
            if (depth < 2 || S.perm[lpath[1][tx]] > S.perm[v]) continue;
            const int L = depth + 1;
            bool sp = true;
            for (int a = 0; a < L && sp; a++)
                for (int b = a + 2; b < L && sp; b++) {
                    const int d = min(b - a, L - (b - a));
                    if (d >= 2 && ring_shortcut(W, lpath[a][tx], lpath[b][tx], d)) sp = false;
                }
            if (!sp) continue;
            atomicAdd(&W.cnt[L], 1ull);
            for (int m = 0; m < L; m++)
                atomicOr(&W.mark[(size_t)lpath[m][tx] * RING_DEG + ((lit[m][tx] & ~CLOSE_ONLY) - 1)], 1u);
            double ang = -1.0;
            if (L == 6) {
                R3<double> p[6];
                p[0] = {0.0, 0.0, 0.0};
                for (int m = 0; m < 5; m++) {
                    const R3<double> bnd = ring_bond(S, W, dtab, lpath[m][tx], (lit[m][tx] & ~CLOSE_ONLY) - 1);
                    p[m + 1] = {p[m].x + bnd.x, p[m].y + bnd.y, p[m].z + bnd.z};
                }
                double ct;
                ang = ring_orientation(p, c, ct);
                if (c.cos_tilt_min < -1.0 || ct >= c.cos_tilt_min) {
                    int bin = (int)(ang / 60.0 * c.nbins);
                    bin = bin < 0 ? 0 : (bin >= c.nbins ? c.nbins - 1 : bin);
                    atomicAdd(&W.hist[bin], 1ull);
                    atomicAdd(&W.cnt[RC_HIST], 1ull);
                }
            }
            const unsigned long long slot = atomicAdd(&W.cnt[RC_LISTED], 1ull);
            if (W.list && (long long)slot < W.cap) {
                int32_t *o = W.list + (size_t)slot * 9;
                o[0] = L;
                for (int m = 0; m < RING_MAX; m++) o[1 + m] = m < L ? S.perm[lpath[m][tx]] : -1;
                if (W.orient) W.orient[slot] = ang;
            }
            continue;
        }
        if (depth + 1 >= c.max_size || S.perm[wv] < u0) continue;
        bool on = false;
        for (int k = 1; k <= depth; k++) on |= lpath[k][tx] == wv;
        if (on) continue;
        // A shortest-path ring has no chord: wv may not be bonded to a path
        // atom other than its predecessor, and once bonded to the start it
        // can only close the ring.
        bool chord = false, closes = false;
        const int dw = W.deg[wv];
        for (int k = 0; k < dw && !chord; k++) {
            const int y = ring_nb(W, wv, k);
            closes |= y == s;
            for (int m = 1; m < depth; m++) chord |= lpath[m][tx] == y;
        }
        if (chord) continue;
        depth++;
        lpath[depth][tx] = wv;
        lit[depth][tx] = (closes && depth >= 2) ? (uint8_t)CLOSE_ONLY : (uint8_t)0;
    }
}

// bonds (each once) and the bonds on no ring
__global__ void __launch_bounds__(TILE) k_ring_chain(const Tile *tiles, Seg *segs, RingWs W)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n) return;
    const int ds = W.deg[s];
    unsigned long long nb = 0, nc = 0;
    for (int k = 0; k < ds; k++) {
        const int t = ring_nb(W, s, k);
        if (S.perm[t] < S.perm[s]) continue;
        nb++;
        bool on = W.mark[(size_t)s * RING_DEG + k] != 0u;
        const int dt = W.deg[t];
        for (int m = 0; m < dt && !on; m++)
            if (ring_nb(W, t, m) == s) on = W.mark[(size_t)t * RING_DEG + m] != 0u;
        if (!on) nc++;
    }
    if (nb) atomicAdd(&W.cnt[RC_BONDS], nb);
    if (nc) atomicAdd(&W.cnt[RC_CHAIN], nc);
}

} // namespace ctbop
