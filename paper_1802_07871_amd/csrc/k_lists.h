// k_lists.hip -- cell binning, deterministic counting sort into cell order,
// and the two Verlet neighbour lists built from a cell stencil.
//
// Atoms are binned on a grid of at least (rc + skin)/2 wide cells laid along
// the (possibly tilted) cell vectors.  Rows of every later kernel are atoms in
// cell order ("sorted rows").  Each sorted atom keeps FP32 coordinates local
// to its cell's origin; the vector to a neighbour in a cell offset by
// d = (d0, d1, d2) grid steps (periodic images included) is
//     r = (l_j - l_i) + D(d),   D(d) = d0 h0/nb0 + d1 h1/nb1 + d2 h2/nb2,
// which keeps every pair vector exact to FP32 rounding of a few Angstrom,
// independent of the box size.  A list entry packs the neighbour row (23 bits)
// and the code of d (9 bits, |d_k| <= 3).
#pragma once
#include "ctbop_dev.h"

namespace ctbop {

__global__ void k_set_seg(Seg *dst, Seg src) { *dst = src; }

__global__ void k_set_warm(SegState *st, int warm) { st->warm = warm; }

__global__ void k_call_init(const int *seg_ids, Seg *segs, int nseg, int force_rebuild)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    SegState *st = segs[seg_ids[k]].sst;
    st->rebuild = (force_rebuild || !st->built) ? 1 : 0;
    st->ticket = 0;
    st->done = 0;
    st->iters = 0;
    st->status = 0;
    st->forces_done = 0;
}

// A neighbour list rebuild is needed once any atom moved more than skin/2
// since the last build (then no pair can have crossed into the cutoff), or
// once any atom changed species: the covalent list's radius is per species
// pair.  Sorted row i still holds the species of the last gather in xs64.w.
__global__ void k_check_disp(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->rebuild) return;
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    double dx = S.x[i] - S.ref_x[i];
    double dy = S.x[S.n + i] - S.ref_x[S.n + i];
    double dz = S.x[2 * S.n + i] - S.ref_x[2 * S.n + i];
    double lim = 0.5 * S.skin;
    bool moved = dx * dx + dy * dy + dz * dz > lim * lim;
    bool retyped = (int)S.xs64[i].w != S.type[S.perm[i]];
    if (moved || retyped) S.sst->rebuild = 1;
}

// fractional coordinates, folded along periodic vectors; the integer fold is
// returned in w
__device__ __forceinline__ void frac_wrap(const Seg &S, double x, double y, double z, double s[3], double w[3])
{
#pragma unroll
    for (int b = 0; b < 3; b++) {
        s[b] = x * S.hi[0][b] + y * S.hi[1][b] + z * S.hi[2][b];
        w[b] = S.pbc[b] ? -floor(s[b]) : 0.0;
        s[b] += w[b];
    }
}

__device__ __forceinline__ int cell_index(const Seg &S, const double s[3], int c[3])
{
#pragma unroll
    for (int b = 0; b < 3; b++) {
        int v = (int)floor(s[b] * S.nb[b]);
        c[b] = v < 0 ? 0 : (v >= S.nb[b] ? S.nb[b] - 1 : v);
    }
    return (c[0] * S.nb[1] + c[1]) * S.nb[2] + c[2];
}

// clear cell counters; mark padding rows
__global__ void k_bin_clear(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    const int tl = T.row0 / TILE;
    for (int c = tl * TILE + threadIdx.x; c < S.ncell; c += S.ntile * TILE) S.cell_cnt[c] = 0;
    int row = T.row0 + threadIdx.x;
    if (row >= S.n && row < S.npad) {
        S.perm[row] = -1;
        S.csort[row] = 0;
        S.lcnt[row] = 0;
        S.scnt[row] = 0;
    }
    if (tl == 0 && threadIdx.x == 0) {
        S.sst->maxl = 0;
        S.sst->maxs = 0;
        S.sst->nnz_long = 0;
        S.sst->nnz_short = 0;
    }
}

__global__ void k_bin(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    double s[3], w[3];
    int c[3];
    frac_wrap(S, S.x[i], S.x[S.n + i], S.x[2 * S.n + i], s, w);
    int ci = cell_index(S, s, c);
    S.cell_of[i] = ci;
    atomicAdd(&S.cell_cnt[ci], 1);
}

// Exclusive scan of the cell counts into cell_start, in three passes over
// the segment's tiles (each tile takes a contiguous chunk of the cells), with
// the counts zeroed for use as fill counters: the chunks' sums (the tiles'
// partials), their exclusive scan (one block per segment), then each chunk's
// starts from its tile's offset.  Integer counts, so any order is exact.
__device__ __forceinline__ void scan_chunk(const Seg &S, int tl, int &c0, int &c1)
{
    const int ch = (S.ncell + S.ntile - 1) / S.ntile;
    c0 = min(S.ncell, tl * ch);
    c1 = min(S.ncell, c0 + ch);
}

__global__ void __launch_bounds__(TILE) k_scan_part(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    __shared__ double lds[4];
    int c0, c1;
    scan_chunk(S, T.row0 / TILE, c0, c1);
    double v[1] = {0.0};
    for (int c = c0 + threadIdx.x; c < c1; c += TILE) v[0] += (double)S.cell_cnt[c];
    tile_partials<1>(S, T.row0 / TILE, v, lds);
}

__global__ void __launch_bounds__(TILE) k_scan_mid(const int *seg_ids, Seg *segs)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (!S.sst->rebuild) return;
    __shared__ int lds[4];
    // each thread a contiguous run of tiles: its run's total, the block's
    // exclusive scan of the totals, then the run's offsets (in place)
    const int per = (S.ntile + TILE - 1) / TILE;
    const int t0 = min(S.ntile, (int)threadIdx.x * per), t1 = min(S.ntile, t0 + per);
    int sum = 0;
    for (int t = t0; t < t1; t++) sum += (int)S.part[t];
    int run = block_excl_scan(sum, lds);
    for (int t = t0; t < t1; t++) {
        const int v = (int)S.part[t];
        S.part[t] = (double)run;
        run += v;
    }
    if (threadIdx.x == TILE - 1) S.cell_start[S.ncell] = run;
}

__global__ void __launch_bounds__(TILE) k_scan_fin(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    __shared__ int lds[4];
    __shared__ int tot;
    int c0, c1;
    scan_chunk(S, T.row0 / TILE, c0, c1);
    int base = (int)S.part[T.row0 / TILE];
    for (int cb = c0; cb < c1; cb += TILE) {
        const int c = cb + threadIdx.x;
        const int v = c < c1 ? S.cell_cnt[c] : 0;
        const int ex = block_excl_scan(v, lds);
        if (threadIdx.x == TILE - 1) tot = ex + v;
        if (c < c1) {
            S.cell_start[c] = base + ex;
            S.cell_cnt[c] = 0;
        }
        __syncthreads();
        base += tot;
        __syncthreads();
    }
}

__global__ void k_scatter(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    int c = S.cell_of[i];
    int slot = S.cell_start[c] + atomicAdd(&S.cell_cnt[c], 1);
    S.perm_tmp[slot] = i;
}

// Order each cell's atoms by user index (the scatter's order is arbitrary),
// so the sorted frame -- and every sum over it -- is deterministic: the atom
// the scatter put at row k goes to its cell's first row plus the number of
// the cell's atoms with a smaller user index.  Then record, per sorted row,
// its cell, its offset (fold minus cell origin) and the reference positions
// for the displacement test.
__global__ void k_cell_sort(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    const int k = T.row0 + threadIdx.x;
    if (k >= S.n) return;
    const int i = S.perm_tmp[k];
    const int c = S.cell_of[i];
    const int a = S.cell_start[c], b = S.cell_start[c + 1];
    int row = a;
    for (int m = a; m < b; m++) row += (S.perm_tmp[m] < i) ? 1 : 0;
    S.perm[row] = i;
    const int c0 = c / (S.nb[1] * S.nb[2]), c1 = (c / S.nb[2]) % S.nb[1], c2 = c % S.nb[2];
    const double x = S.x[i], y = S.x[S.n + i], z = S.x[2 * S.n + i];
    double s[3], w[3];
    frac_wrap(S, x, y, z, s, w);
    S.csort[row] = c;
#pragma unroll
    for (int a2 = 0; a2 < 3; a2++) {
        double o = w[0] * S.h[0][a2] + w[1] * S.h[1][a2] + w[2] * S.h[2][a2]
                 - (c0 * S.cw[0][a2] + c1 * S.cw[1][a2] + c2 * S.cw[2][a2]);
        S.off[a2 * S.npad + row] = o;
    }
    S.ref_x[i] = x;
    S.ref_x[S.n + i] = y;
    S.ref_x[2 * S.n + i] = z;
}

// Local coordinates of every sorted atom for this call's positions, and the
// starting charges in the sorted frame (with their sum, for the projection).
// warm: 0 = zeros, 1 = the last solution, 2 = extrapolate the last solutions
// by the polynomial through the last m of them (m = min(kept, PRED_ORDER)),
// for consecutive MD steps: the value at the next step of the polynomial of
// degree m-1 through q_0, q_-1, ..., q_-(m-1) is sum_k (-1)^k C(m, k+1) q_-k.
__device__ __forceinline__ double pred_coef(int m, int k)
{
    // (-1)^k C(m, k+1) for m <= 4
    constexpr double C[5][4] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {2, 1, 0, 0}, {3, 3, 1, 0}, {4, 6, 4, 1}};
    return (k & 1) ? -C[m][k] : C[m][k];
}
template <typename R>
__global__ void k_gather(const Tile *tiles, Seg *segs, int warm)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    double q0 = 0.0;
    if (s < S.n) {
        const int i = S.perm[s];
        double4 w;
        w.x = S.x[i] + S.off[s];
        w.y = S.x[S.n + i] + S.off[S.npad + s];
        w.z = S.x[2 * S.n + i] + S.off[2 * S.npad + s];
        w.w = (double)S.type[i];
        V4 v;
        v.x = (R)w.x;
        v.y = (R)w.y;
        v.z = (R)w.z;
        v.w = (R)w.w;
        reinterpret_cast<V4 *>(S.xs)[s] = v;
        if ((void *)S.xs64 != S.xs) S.xs64[s] = w;
        const int wm = warm < 0 ? S.sst->warm : warm;
        if (wm) {
            int m = 1;
            if (wm == 2) m = min(S.sst->nhist, (S.q_ring ? NHIST : 0) + 1);
            m = min(m, PRED_ORDER);
            if (m >= 1) {
                q0 = pred_coef(m, 0) * S.q_state[i];
                const int head = S.sst->qhead;
                for (int k = 1; k < m; k++) {
                    const int slot = (head - (k - 1) + NHIST) % NHIST;
                    q0 += pred_coef(m, k) * S.q_ring[(size_t)slot * S.n + i];
                }
            }
        }
        S.q[s] = q0;
    } else if (s < S.npad) {
        S.q[s] = 0.0;
    }
    __shared__ double lds[4];
    double v1[1] = {q0};
    tile_partials<1>(S, T.row0 / TILE, v1, lds);
}

// apply the projection of the starting charges onto sum q = Q
__global__ void k_qfix(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    if (s < S.n) S.q[s] += S.sst->qshift;
}

__global__ void k_fin_qshift(const int *seg_ids, Seg *segs)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[4];
    double tot[1];
    seg_total<1>(S, lds, tot);
    if (threadIdx.x == 0) S.sst->qshift = (S.Q - tot[0]) / S.n;
}

// table of D(code) for the block's segment, in LDS
template <typename R>
__device__ __forceinline__ void load_dtab(const Seg &S, typename Vec4<R>::type *tab)
{
    for (int c = threadIdx.x; c < NCODE; c += blockDim.x) {
        int d0 = c / 49 - 3, d1 = (c / 7) % 7 - 3, d2 = c % 7 - 3;
        typename Vec4<R>::type v;
        v.x = (R)(d0 * S.cw[0][0] + d1 * S.cw[1][0] + d2 * S.cw[2][0]);
        v.y = (R)(d0 * S.cw[0][1] + d1 * S.cw[1][1] + d2 * S.cw[2][1]);
        v.z = (R)(d0 * S.cw[0][2] + d1 * S.cw[1][2] + d2 * S.cw[2][2]);
        v.w = 0;
        tab[c] = v;
    }
    __syncthreads();
}

// The tile's halo from its bitmap (in LDS, HALO_WORDS words, complete): the
// distinct rows of its list entries within HALO_WIN / 2 rows of its first
// row.  hpre holds the set bits before each word, halo the marked rows in
// order (when at most HALO_MAX), nhalo their number.  Every thread of the
// block calls it.
__device__ __forceinline__ void write_halo(const Seg &S, const Tile &T, const unsigned long long *bm, int *wsum)
{
    constexpr int WPT = HALO_WORDS / TILE;   // words per thread
    static_assert(HALO_WORDS % TILE == 0, "whole words per thread");
    const int tl = T.row0 / TILE;
    const int w0 = threadIdx.x * WPT;
    int c = 0;
#pragma unroll
    for (int k = 0; k < WPT; k++) c += __popcll(bm[w0 + k]);
    // exclusive scan of c over the block: within the wave, then the waves
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int before = inc - c, total = 0;
    for (int w = 0; w < TILE / 64; w++) {
        if (w < wv) before += wsum[w];
        total += wsum[w];
    }
    const auto hb = gblw(S.hbits + (size_t)tl * HALO_WORDS);
    const auto hp = gblw(S.hpre + (size_t)tl * HALO_WORDS);
    const auto hl = gblw(S.halo + (size_t)tl * HALO_MAX);
    const int org = T.row0 - HALO_WIN / 2;
    int at = before;
#pragma unroll
    for (int k = 0; k < WPT; k++) {
        unsigned long long b = bm[w0 + k];
        hb[w0 + k] = b;
        hp[w0 + k] = (uint16_t)at;
        if (total <= HALO_MAX) {
            while (b) {
                const int bit = __ffsll((long long)b) - 1;
                hl[at++] = (uint32_t)(org + 64 * (w0 + k) + bit);
                b &= b - 1;
            }
        } else {
            at += __popcll(b);
        }
    }
    if (threadIdx.x == 0) S.nhalo[tl] = total;
}

// Both lists for every sorted atom: the cell stencil visited in a fixed order,
// each cell's atoms in sorted order, so rows are deterministic.  L lanes per
// atom take L consecutive atoms of a cell at a time (one coalesced read of
// their coordinates); group ballots place the accepted ones in list order.
// Per-row statistics are reduced over the block before one atomic each.
template <typename R, int L>
__global__ void __launch_bounds__(TILE) k_build(const Tile *tiles, Seg *segs, Params<R> P)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    __shared__ V4 dtab[NCODE];
    __shared__ int red[4][5];
    __shared__ unsigned long long hbm[HALO_WORDS];
    __shared__ int wsum[TILE / 64];
    for (int w = threadIdx.x; w < HALO_WORDS; w += TILE) hbm[w] = 0ull;
    load_dtab<R>(S, dtab);
    __syncthreads();
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    // the segment's fields in registers: the list stores below cannot change them
    const int Wl = S.Wl, Ws = S.Ws, n = S.n;
    const int nb0 = S.nb[0], nb1 = S.nb[1], nb2 = S.nb[2];
    const int st0 = S.st[0], st1 = S.st[1], st2 = S.st[2];
    const bool pbc0 = S.pbc[0], pbc1 = S.pbc[1], pbc2 = S.pbc[2];
    const auto csort = gbl(S.csort);
    const auto cstart = gbl(S.cell_start);
    constexpr int G = TILE / L;
    const int lane = threadIdx.x % L;
    const unsigned below = (1u << lane) - 1u;
    int st_or = 0, mx_l = 0, mx_s = 0, sum_l = 0, sum_s = 0;
    for (int k = threadIdx.x / L; k < TILE; k += G) {
        const int s = T.row0 + k;
        if (s >= n) continue;                  // the whole group skips together
        const V4 li = ld4<R>(xs, s);
        const int ti = (int)li.w;
        const float sc2_0 = P.s_cut2[ti * 2], sc2_1 = P.s_cut2[ti * 2 + 1];
        const int c = csort[s];
        const int c0 = c / (nb1 * nb2), c1 = (c / nb2) % nb1, c2 = c % nb2;
        const auto lrow = gblw(S.lidx + (size_t)s * Wl);
        const auto srow = gblw(S.sidx + (size_t)s * Ws);
        // the atom's fractional place in its cell: a stencil cell at offset d
        // spans fractional offsets [d - f, d - f + 1] from it per axis, at
        // least g = max(0, d - f, f - d - 1) cells; cells whose g^2 sum
        // exceeds cull2 hold no list entry and are not scanned (rows of the
        // stencil whose first two g already do are skipped, and each row's
        // run of cells along the last axis is trimmed to the sphere)
        const float lx = (float)li.x, ly = (float)li.y, lz = (float)li.z;
        const float f0 = lx * S.cwi[0][0] + ly * S.cwi[1][0] + lz * S.cwi[2][0];
        const float f1 = lx * S.cwi[0][1] + ly * S.cwi[1][1] + lz * S.cwi[2][1];
        const float f2 = lx * S.cwi[0][2] + ly * S.cwi[1][2] + lz * S.cwi[2][2];
        const float cull2 = S.cull2;
        int nl = 0, ns = 0;
        bool close = false;
        for (int d0 = -st0; d0 <= st0; d0++) {
            const float g0 = fmaxf(0.0f, fmaxf((float)d0 - f0, f0 - (float)d0 - 1.0f));
            const float rem0 = cull2 - g0 * g0;
            if (rem0 < 0.0f) continue;
            int e0 = c0 + d0;
            if (pbc0) { e0 %= nb0; if (e0 < 0) e0 += nb0; }
            else if (e0 < 0 || e0 >= nb0) continue;
            for (int d1 = -st1; d1 <= st1; d1++) {
                const float g1 = fmaxf(0.0f, fmaxf((float)d1 - f1, f1 - (float)d1 - 1.0f));
                const float rem1 = rem0 - g1 * g1;
                if (rem1 < 0.0f) continue;
                int e1 = c1 + d1;
                if (pbc1) { e1 %= nb1; if (e1 < 0) e1 += nb1; }
                else if (e1 < 0 || e1 >= nb1) continue;
                // The cells of one stencil row along the last axis are
                // consecutive, and so are their atoms: the lanes walk each
                // run of cells that does not cross the periodic seam as one
                // range (in the same order as cell by cell), and each lane
                // takes its atom's offset from the atom's cell.
                const int rowc = (e0 * nb1 + e1) * nb2;
                const float g2max = sqrtf(rem1);
                int dlo = max(-st2, (int)ceilf(f2 - 1.0f - g2max)), dhi = min(st2, (int)floorf(f2 + g2max));
                if (!pbc2) {
                    dlo = max(dlo, -c2);
                    dhi = min(dhi, nb2 - 1 - c2);
                }
                for (int dr = dlo; dr <= dhi;) {
                    int er = c2 + dr;
                    if (pbc2) { er %= nb2; if (er < 0) er += nb2; }
                    const int len = min(dhi - dr + 1, nb2 - er);
                    const int m0 = cstart[rowc + er], m1 = cstart[rowc + er + len];
                    for (int mb = m0; mb < m1; mb += L) {
                        const int m = mb + lane;
                        bool inl = false, ins = false;
                        uint32_t ent = 0;
                        // the candidate's cell and position, both loaded before
                        // either is used (lanes past the run load its last atom)
                        const int mc = min(m, m1 - 1);
                        const int cm = csort[mc];
                        const V4 lj = ld4<R>(xs, mc);
                        const int d2 = m < m1 ? dr + (cm - rowc - er) : 0;
                        const int code = code_of(d0, d1, d2);
                        const V4 D = dtab[code];
                        R rx = (lj.x - li.x) + D.x, ry = (lj.y - li.y) + D.y, rz = (lj.z - li.z) + D.z;
                        float r2 = (float)(rx * rx + ry * ry + rz * rz);
                        if (m < m1 && !(m == s && code == CODE_CENTER)) {
                            if (r2 < P.l_cut2) {
                                inl = true;
                                if (r2 < P.close2) close = true;
                                ins = r2 < ((int)lj.w ? sc2_1 : sc2_0);
                                ent = (uint32_t)m | ((uint32_t)code << CODE_SHIFT);
                            }
                        }
                        const unsigned gl = group_ballot<L>(inl), gs = group_ballot<L>(ins);
                        if (inl) {
                            const int at = nl + __popc(gl & below);
                            if (at < Wl) lrow[at] = ent;
                            const int hw = m - T.row0 + HALO_WIN / 2;
                            if ((unsigned)hw < (unsigned)HALO_WIN) atomicOr(&hbm[hw >> 6], 1ull << (hw & 63));
                        }
                        if (ins) {
                            const int at = ns + __popc(gs & below);
                            if (at < Ws) srow[at] = ent;
                        }
                        nl += __popc(gl);
                        ns += __popc(gs);
                    }
                    dr += len;
                }
            }
        }
        const bool any_close = group_ballot<L>(close) != 0u;
        if (lane == 0) {
            if (any_close) st_or |= ST_TOO_CLOSE;
            if (nl > Wl || ns > Ws) st_or |= ST_OVERFLOW;
            const int cl = nl < Wl ? nl : Wl, cs = ns < Ws ? ns : Ws;
            S.lcnt[s] = cl;
            S.scnt[s] = cs;
            mx_l = max(mx_l, nl);
            mx_s = max(mx_s, ns);
            sum_l += cl;
            sum_s += cs;
        }
    }
    // block totals, then one atomic per statistic
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        st_or |= __shfl_xor(st_or, o, 64);
        mx_l = max(mx_l, __shfl_xor(mx_l, o, 64));
        mx_s = max(mx_s, __shfl_xor(mx_s, o, 64));
        sum_l += __shfl_xor(sum_l, o, 64);
        sum_s += __shfl_xor(sum_s, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = st_or;
        red[wv][1] = mx_l;
        red[wv][2] = mx_s;
        red[wv][3] = sum_l;
        red[wv][4] = sum_s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            red[0][0] |= red[w][0];
            red[0][1] = max(red[0][1], red[w][1]);
            red[0][2] = max(red[0][2], red[w][2]);
            red[0][3] += red[w][3];
            red[0][4] += red[w][4];
        }
        if (red[0][0]) atomicOr(&S.sst->status, red[0][0]);
        atomicMax(&S.sst->maxl, red[0][1]);
        atomicMax(&S.sst->maxs, red[0][2]);
        atomicAdd(&S.sst->nnz_long, (unsigned long long)red[0][3]);
        atomicAdd(&S.sst->nnz_short, (unsigned long long)red[0][4]);
    }
    write_halo(S, T, hbm, wsum);
}

// For every covalent entry (i -> j, d) the slot of (j -> i, -d) in row j:
// 16 lanes per row, one entry each, every lane searching its partner's row.
__global__ void __launch_bounds__(TILE) k_rev(const Tile *tiles, Seg *segs)
{
    constexpr int LR = 16;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (!S.sst->rebuild) return;
    const int lane = threadIdx.x % LR;
    const int Ws = S.Ws;
    const auto sidx = gbl(S.sidx);
    const auto scnt = gbl(S.scnt);
    bool bad = false;
    for (int k = threadIdx.x / LR; k < TILE; k += TILE / LR) {
        const int s = T.row0 + k;
        if (s >= S.n) break;                     // rows past n come last: the group is done
        const int ns = scnt[s];
        for (int e = lane; e < ns; e += LR) {
            const uint32_t ent = sidx[(size_t)s * Ws + e];
            const int j = (int)(ent & J_MASK), want = code_neg((int)(ent >> CODE_SHIFT));
            const uint32_t target = (uint32_t)s | ((uint32_t)want << CODE_SHIFT);
            const int nj = scnt[j];
            int f = -1;
            for (int m = 0; m < nj; m++)
                if (sidx[(size_t)j * Ws + m] == target) { f = m; break; }
            if (f < 0) { bad = true; f = 0; }
            S.srev[(size_t)s * Ws + e] = (uint8_t)f;
        }
    }
    if (bad) atomicOr(&S.sst->status, ST_REV);
}

__global__ void k_mark_built(const int *seg_ids, Seg *segs, int nseg)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    SegState *st = segs[seg_ids[k]].sst;
    if (st->rebuild) {
        st->built = 1;
        st->nrebuild += 1;
    }
}

} // namespace ctbop
