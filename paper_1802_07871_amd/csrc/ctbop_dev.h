// ctbop_dev.h -- device-side data structures shared by the HIP kernels.
//
// Work decomposition: every kernel runs on a table of tiles.  A tile is 256
// consecutive rows (atoms, in the sorted frame) of one segment (one atomic
// system), processed by one 256-thread block.  Segments are padded to whole
// tiles, so each block touches one segment only; per-tile partial sums are
// combined per segment in a fixed order by the segment's last block, which
// makes every reduction deterministic and independent of what else runs in
// the same launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctbop {

constexpr int TILE = 256;
constexpr int NPART = 16;              // doubles of partial sums per tile
constexpr int CODE_BITS = 9;           // stencil offset code in the list entry
constexpr int CODE_SHIFT = 23;         // low 23 bits: neighbour row
constexpr uint32_t J_MASK = (1u << CODE_SHIFT) - 1u;
constexpr int NCODE = 343;             // offsets (-3..3)^3
constexpr int CODE_CENTER = 171;       // offset (0,0,0)
constexpr int MAX_ATOMS = (1 << CODE_SHIFT) - 1;
constexpr int SLICE = 64;              // rows per slice of the sliced list layout (one wave)
constexpr int BK = 16;                 // rows per block of the block-Jacobi preconditioner
constexpr int WB = 32;                 // bond-row capacity (bonds inside S_ij per atom)
constexpr int NHIST = 3;               // charge solutions kept before the latest (predictor history)
constexpr int PRED_ORDER = 4;          // points of the starting-charge extrapolation (1..NHIST+1)
constexpr int HALO_WIN = 65536;        // rows around a tile's first row whose charges a tile may stage
constexpr int HALO_WORDS = HALO_WIN / 64;
#ifndef CTBOP_HALO_MAX
#define CTBOP_HALO_MAX 3072
#endif
constexpr int HALO_MAX = CTBOP_HALO_MAX; // staged rows per tile in the charge-solve product (LDS doubles)
// forms of a slice of the solver's sliced copy (swide)
constexpr uint8_t SL_HALO = 0, SL_FULL = 1, SL_OFF16 = 2;

// status bits (mapped to CTBOP_E_* codes on the host)
constexpr int ST_TOO_CLOSE = 1, ST_NOCONV = 2, ST_NOT_PD = 4, ST_OVERFLOW = 8, ST_REV = 16;

// ---------------------------------------------------------------------------
// potential parameters, precomputed on the host per context
// ---------------------------------------------------------------------------
template <typename R>
struct Params {
    // pair (ti*2 + tj): repulsion/attraction, cutoff radii, pi/(S-R)
    R A[4], B[4], lam1[4], lam2[4], Rc[4], Sc[4], piSR[4];
    // centre species: normalisation G, 1/(2 sigma), channel constants
    R G[2], inv2sig[2];
    R gam[2][2], c2[2][2], d2[2][2], h[2][2], nn[2][2], g[2][2], alpha[2][2];
    R c2d2[2][2];                      // c^2 / d^2 of the angular function
    R p;
    int p_is_2;
    int alpha_zero[2];                 // both channels of species t have alpha == 0
    // Coulomb
    R ke, rc, inv_rc, g3[4];           // g3 = (gamma_i gamma_j)^(-3/2)
    double chi[2], J[2], E0[2], mass[2];
    // list radii (squared), including the skin
    float l_cut2, s_cut2[4];
    float close2;                      // too-close threshold squared
};

// ---------------------------------------------------------------------------
// per-segment scalars (device), reset per call where noted
// ---------------------------------------------------------------------------
struct SegState {
    int rebuild;       // lists rebuilt in this call
    int ticket;        // last-block detection counter (returns to 0)
    int done;          // charge solve finished
    int iters;
    int status;        // ST_* bits, sticky until the next rebuild/call reset
    int maxl, maxs;    // largest list rows at the last build
    int built;         // lists exist
    int nhist;         // charge solutions kept for the starting-charge predictor (0..NHIST+1)
    int qhead;         // ring slot of the solution before the latest
    int warm;          // per-segment start mode when a launch passes warm < 0 (serving)
    int forces_done;   // serving: forces and energy of the current request are written
    int nrebuild;      // rebuilds since the system buffer was set up
    int cg_first;      // single-reduction solve: the next finalize is the solve's first
    int cg_last;       // single-reduction solve: the update now launched is the last
    double w;          // current residual shift
    double rho, alpha, beta, res;
    double sdinv;      // 1^T M 1 (sum of the preconditioner's row sums)
    double mu_prev;    // chemical potential of the previous solve
    double mshift;     // accumulated shift: r_stored = -(Hq+chi) + mshift
    double qshift;     // final re-projection of q onto sum q = Q
    double energy;
    unsigned long long nnz_long, nnz_short;   // list entries at the last build
    unsigned long long iters_total;           // charge-solve iterations since set-up
    double res0;                              // starting residual of the last solve
    double nnz_coul;                          // Coulomb entries inside rc at the last assembly
    double nnz_wide;                          // of which in slices that keep full entries
    double nnz_halo;                          // of which in slices of halo positions
    double nnz_slots;                         // entry slots the sliced product reads: 64 x longest row, per slice
    double nbond, ntrip;                      // bonds and ordered bond pairs (i; j, k) at the last evaluation
    // charge coupling (f_q) solve: p^T r, p^T H p and the coupling part of
    // phi'(0) along the current direction (line search)
    double pr, ps, A0;
    double m1s;        // single-reduction solve: m1^T s of the current direction
};

// ---------------------------------------------------------------------------
// segment descriptor: geometry, sizes and array addresses
// ---------------------------------------------------------------------------
struct Seg {
    double h[3][3];    // cell vectors as rows
    double hi[3][3];   // inverse: frac = x . hi
    double cw[3][3];   // cell-grid vectors: h[d] / nb[d]
    // the list build's cell culling: an atom's fractional place in its cell
    // is f = l . cwi (l its local coordinates); a point at fractional offset
    // s from it lies at least sqrt(lam |s|^2) away, lam the smallest
    // eigenvalue of the cell metric cw cw^T, so cells with |s|^2 > cull2 =
    // (rc + skin)^2 / lam (a margin added) hold no list entry of the atom
    float cwi[3][3];
    float cull2;
    int pbc[3];
    int nb[3];         // cell grid
    int st[3];         // stencil half-width per direction (<= 3)
    int ncell;
    int n, npad;       // atoms, padded to TILE
    int tile0, ntile;  // this segment's range in the tile table
    int Wl, Ws, Wb;    // row strides: Coulomb list, covalent list, bonds
    double Q;          // total charge
    double skin;
    // caller arrays (set per call)
    const double *x;   // SoA positions, 3n
    const int *type;   // n
    double *F;         // SoA forces out, 3n
    double *q_out;     // n
    double *E_out;     // 1
    // persistent arrays
    int *perm;         // sorted row -> user index        [npad]
    int *perm_tmp;     // the scatter's order of each cell's atoms (list build only) [npad]
    int *cell_of;      // user index -> cell              [n]
    int *csort;        // sorted row -> cell              [npad]
    int *cell_start;   // [ncell + 1]
    int *cell_cnt;     // [ncell]
    double *off;       // sorted: wrap*h - cell origin, SoA [3 npad]
    double *ref_x;     // user order positions at build, SoA [3n]
    void *xs;          // sorted local coordinates + type  [npad] float4 / double4
    double4 *xs64;     // the same in FP64 (bond lengths of the energy)  [npad]
    // Coulomb list: r < rc + skin at the last build, row-major, stride Wl.
    int *lcnt;         // [npad]
    uint32_t *lidx;    // [npad * Wl]
    // Coulomb rows of the current step (rewritten by every assembly): the
    // list entries inside rc in list order, row-major (hidx, with the
    // matrix entries Hr), and the same rows sliced column-major for the
    // charge-solve product (hsidx, H): slices of SLICE consecutive rows, entry
    // e of row s at (s / SLICE) * SLICE * Wl + e * SLICE + s % SLICE, so that
    // a wave, one row per lane, reads entry e of its 64 rows as one
    // contiguous segment.
    int *hcnt;         // [npad]
    uint32_t *hidx;    // [npad * Wl]
    void *Hr;          // [npad * Wl] float / double
    // The halo of a tile is the sorted set of distinct rows of its rows'
    // list entries (r < rc + skin at the last build) that lie within
    // HALO_WIN / 2 rows of the tile's first row: the list build marks them
    // in a bitmap over that window (hbits), with the running count of set
    // bits before each 64-bit word (hpre); halo lists them, nhalo counts
    // them.  The charge-solve product stages p of the halo in LDS once per
    // tile, so that each entry gathers from LDS.  In the sliced copy the
    // neighbours of a slice's entries are stored in one of three forms
    // (swide): their 16-bit positions in the tile's halo (hs16, SL_HALO)
    // when the halo holds at most HALO_MAX rows, else 16-bit offsets from
    // the slice's first slot (hs16, offset + 32768, SL_OFF16), and the full
    // entries (hsidx, SL_FULL) when a row of the slice has an entry beyond a
    // 16-bit offset from some slice of its tile (hwide flags those rows;
    // the entries of the other rows lie in the halo window).  Within each
    // tile the rows take the slice slots in order of decreasing length (ties
    // by row), so that the rows of a slice have similar lengths and a wave
    // reads few padding slots; slot t of a tile holds row hperm[t] of that
    // tile.
    uint32_t *hsidx;   // [npad * Wl]
    uint16_t *hs16;    // [npad * Wl]
    uint8_t *hwide;    // [npad]
    uint8_t *swide;    // [npad / SLICE], per slice of slots
    uint8_t *hperm;    // [npad]
    uint32_t *halo;    // [ntile * HALO_MAX]
    int *nhalo;        // [ntile]
    unsigned long long *hbits;  // [ntile * HALO_WORDS]
    uint16_t *hpre;    // [ntile * HALO_WORDS]
    void *H;           // [npad * Wl] float / double
    // covalent list: r < S_ij + skin at the last build, row-major, stride Ws
    int *scnt;         // [npad]
    uint32_t *sidx;    // [npad * Ws]
    uint8_t *srev;     // [npad * Ws]: slot of the reverse entry in the partner's row
    // Bonds of the current step: the covalent-list entries inside S_ij (FP64
    // distance), compacted in list order into rows of width Wb; cmap maps
    // each list slot to its bond index (255: outside) and bsrev holds each
    // bond's reverse list slot, so the reverse bond of (m, e) in the partner
    // i's row is cmap[i][bsrev[m][e]].  These arrays are sliced like the
    // solver's copy (entry e of row s at sliced(s, e, W)): a wave reading
    // entry e of its 64 rows reads one contiguous segment, and rows of nearby
    // atoms share cache lines.
    int *bcnt;         // [npad]
    uint32_t *bidx;    // [npad * Wb]
    uint8_t *bsrev;    // [npad * Wb]
    uint8_t *cmap;     // [npad * Ws]
    void *slot;        // [npad * Wb] per bond, float4 / double4: b, P1, P2, -
    double *ecov;      // [npad]
    double *Fcov;      // SoA [3 npad]
    double *q, *r, *p, *s, *jd;          // [npad]
    // block-Jacobi preconditioner: the inverse of each diagonal BK x BK block
    // of H (blocks of BK consecutive sorted rows), computed in FP32,
    // symmetrised and stored in FP16 (so the operator is exactly symmetric);
    // its row sums m1 = M 1 (of the stored entries, FP64) and y = M r
    _Float16 *binv;    // [npad * BK]: row s of its block's inverse at s * BK
    double *m1, *y;    // [npad]
    double *hz;        // [npad]: H y, the single-reduction solve's product
    double *q_state;   // user order charges of the last solve, for the warm start [n]
    double *q_ring;    // the NHIST solves before it, a ring of [NHIST][n] (predictor history; null: none)
    double *part;      // [NPART * ntile + 16 * FIN_SPLIT]: partial k of tile t at k * ntile + t, then group sums
    SegState *sst;
    // Charge-dependent coupling of the covalent part (fqk > 0; null arrays
    // otherwise): the bond attraction is scaled by f_q = exp(-fqk (q_i - q_j)^2).
    // rl holds the quadratic part of the residual, -(H q + chi) + shift, kept
    // by recursion; rold the last full residual (for the Polak-Ribiere
    // coefficient); wq per bond (sliced like the bond rows) the symmetrised
    // charge-free attraction (c_ij + c_ji)/2, c = fc b fA.
    double fqk;
    double *rl, *rold;  // [npad]
    double *wq;         // [npad * Wb]
};

struct Tile {
    int seg, row0;
};

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2.  Tiles are in spatial (cell) order, so the
// tile of block b is chosen to give each XCD one contiguous run of tiles:
// neighbouring tiles then share an L2 and their neighbour gathers hit it.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ Tile my_tile(const Tile *tiles)
{
    return tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Offset of entry 0 of row s in a sliced list of width W (entry e adds e * SLICE)
__device__ __forceinline__ size_t slice_base(int s, int W)
{
    return (size_t)(s & ~(SLICE - 1)) * (size_t)W + (size_t)(s & (SLICE - 1));
}

// Entry e of row s in a sliced array of row width W
__device__ __forceinline__ size_t sliced(int s, int e, int W) { return slice_base(s, W) + (size_t)e * SLICE; }

// A row of a sliced array, indexed by entry
template <typename T> struct SRow {
    T *p;
    __device__ __forceinline__ T &operator[](int e) const { return p[(size_t)e * SLICE]; }
};
template <typename T> __device__ __forceinline__ SRow<T> srow(T *a, int s, int W) { return SRow<T>{a + slice_base(s, W)}; }

// The same pointer in the global address space.  Pointers read from a Seg
// are generic, so their loads compile to flat instructions, which count on
// both the vector-memory and the LDS counters: every wait for one then waits
// for the other, and loads issued ahead cannot stay in flight across LDS
// traffic.  Global loads count on the vector-memory counter only.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gbl(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T *gblw(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// element i of an array of float4/double4, loaded as one global vector load
template <typename R> struct NVec4;
template <> struct NVec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NVec4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename R>
__device__ __forceinline__ typename Vec4<R>::type ld4(const typename Vec4<R>::type *p, size_t i)
{
    const typename NVec4<R>::type v = ((const __attribute__((address_space(1))) typename NVec4<R>::type *)p)[i];
    typename Vec4<R>::type o;
    o.x = v.x;
    o.y = v.y;
    o.z = v.z;
    o.w = v.w;
    return o;
}
template <typename R>
__device__ __forceinline__ void st4(typename Vec4<R>::type *p, size_t i, const typename Vec4<R>::type &o)
{
    typename NVec4<R>::type v;
    v.x = o.x;
    v.y = o.y;
    v.z = o.z;
    v.w = o.w;
    ((__attribute__((address_space(1))) typename NVec4<R>::type *)p)[i] = v;
}

__device__ __forceinline__ int code_of(int d0, int d1, int d2) { return ((d0 + 3) * 7 + (d1 + 3)) * 7 + (d2 + 3); }

// reverse offset code: (-d0, -d1, -d2)
__device__ __forceinline__ int code_neg(int c) { return (NCODE - 1) - c; }

// wave64 sum of a double (fixed butterfly order: deterministic)
// v plus lane-moved copy of v (a DPP move of both 32-bit halves; lanes of
// rows outside ROWS add 0)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_add(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (every lane active), returned in every
// lane.  The moves run in the vector ALU (data-parallel-primitive lane
// moves) instead of LDS permutes: pairs, quads, half rows and rows of 16 by
// mirrors, then row 0 into row 1 and row 2 into row 3 (broadcast of lane 15
// of each row), then rows 0-1 into rows 2-3 (lane 31); lane 63 ends with the
// total.  The order of the additions is fixed.
__device__ __forceinline__ double wave_sum(double v)
{
    v = dpp_add<0xb1>(v);          // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4e>(v);          // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141>(v);         // row_half_mirror
    v = dpp_add<0x140>(v);         // row_mirror
    v = dpp_add<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// sum across a group of `width` consecutive lanes (power of two <= 64)
template <int W>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

template <int W>
__device__ __forceinline__ int group_sumi(int v)
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// The W-bit slice of a wave ballot that belongs to this lane's group of W
// consecutive lanes (W a power of two <= 32).
template <int W>
__device__ __forceinline__ unsigned group_ballot(bool pred)
{
    const unsigned long long m = __ballot(pred);
    const int base = (int)(threadIdx.x & 63) & ~(W - 1);
    const unsigned all = (W == 32) ? 0xffffffffu : ((1u << W) - 1u);
    return (unsigned)(m >> base) & all;
}

// Exclusive prefix sum of one int per thread over the 256-thread block, in a
// fixed order; every thread of the block must call it.
__device__ __forceinline__ int block_excl_scan(int v, int *lds /* 4 */)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wv; w++) off += lds[w];
    __syncthreads();
    return off + x - v;
}

template <int W>
__device__ __forceinline__ float group_sumf(float v)
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// Block (256 threads) sum of K doubles per thread into out[0..K) (valid in
// thread 0).  Wave butterflies, then the 4 wave results in a fixed order.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds /* 4*K */, double (&out)[K])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; k++) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[wv * K + k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) out[k] = ((lds[k] + lds[K + k]) + lds[2 * K + k]) + lds[3 * K + k];
    }
    __syncthreads();
}

// Block sum of K values, written as this tile's partial sums.  Every kernel
// that reduces writes partials this way; a finalize kernel (one block per
// segment, launched next on the same stream) adds them up.  The kernel
// boundary makes the partials visible, so no block needs a device-scope fence.
template <int K>
__device__ __forceinline__ void tile_partials(const Seg &S, int tile_local, double (&v)[K], double *lds)
{
    double tot[K];
    block_sum<K>(v, lds, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) S.part[(size_t)k * S.ntile + tile_local] = tot[k];
    }
}

// The same, written as partials k0 .. k0+K-1 (so that two kernels can leave
// their sums for one finalize).
template <int K>
__device__ __forceinline__ void tile_partials_at(const Seg &S, int tile_local, double (&v)[K], double *lds, int k0)
{
    double tot[K];
    block_sum<K>(v, lds, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) S.part[(size_t)(k0 + k) * S.ntile + tile_local] = tot[k];
    }
}

// Sum partial k over the segment's tiles in a fixed order (all 256 threads of
// the finalize block; result valid in thread 0).
template <int K>
__device__ __forceinline__ void seg_total(const Seg &S, double *lds, double (&out)[K])
{
    double v[K];
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = 0.0;
    // unrolled so that the loads of several rounds are in flight together
    // (the sums still take the tiles in order)
    const auto part = gbl(S.part);
    const int nt = S.ntile;
#pragma unroll 8
    for (int t = threadIdx.x; t < nt; t += TILE) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += part[(size_t)k * nt + t];
    }
    block_sum<K>(v, lds, out);
}

// Two-stage sum of partials 0 .. K-1 over a segment's tiles (the
// single-reduction solve's finalize, 15 partials per tile): one block alone
// reads them at ~50 GB/s, the rate of one CU's outstanding misses, so FIN_SPLIT
// blocks first sum consecutive ranges of tiles (each thread about one tile),
// and the finalize adds the FIN_SPLIT group sums in order.  The group sums
// sit after the tiles' partials, 16 doubles per group.
constexpr int FIN_SPLIT = 16;
template <int K>
__device__ __forceinline__ void seg_group_sum(const Seg &S, int grp, double *lds /* 4 * K */)
{
    static_assert(K <= 16, "a group keeps 16 sums");
    const auto part = gbl(S.part);
    const int nt = S.ntile;
    const int per = (nt + FIN_SPLIT - 1) / FIN_SPLIT;
    const int t0 = grp * per, t1 = min(nt, t0 + per);
    double v[K];
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += TILE) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += part[(size_t)k * nt + t];
    }
    double tot[K];
    block_sum<K>(v, lds, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) S.part[(size_t)NPART * nt + grp * 16 + k] = tot[k];
    }
}

// The group sums added in group order (result valid in thread 0).
template <int K>
__device__ __forceinline__ void seg_total_groups(const Seg &S, double *lds /* FIN_SPLIT * K */, double (&out)[K])
{
    const double *g = S.part + (size_t)NPART * S.ntile;
    for (int i = threadIdx.x; i < FIN_SPLIT * K; i += blockDim.x) lds[i] = g[(i / K) * 16 + i % K];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            double a = lds[k];
            for (int b = 1; b < FIN_SPLIT; b++) a += lds[b * K + k];
            out[k] = a;
        }
    }
    __syncthreads();
}

} // namespace ctbop
