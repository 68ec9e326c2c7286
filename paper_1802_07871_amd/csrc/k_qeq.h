// k_qeq.h -- charge equilibration and the Coulomb terms.
//
// The charges minimise the energy at every call (Methods).  With the
// self energy chi q + J q^2/2 and the Coulomb kernel C_ij, the energy is
// quadratic in q, so the minimiser solves  H q + chi = mu 1,  sum q = Q,
// H = diag(J) + [C_ij summed over images].  It is found by projected
// block-Jacobi-preconditioned conjugate gradients:
//   z = M (r - w 1),  w = (1^T M r) / (1^T M 1),
// which keeps every direction on sum z = 0; M is the inverse of the diagonal
// blocks of H over BK consecutive sorted rows (atoms of one or two cells,
// which carry the strongest couplings).  The residual r is stored shifted
// by the running w (r = -(Hq + chi) + const), so it never carries the large
// multiplier mu, whose rounding would otherwise swamp r^T z.  Vectors,
// dot products and the projection are FP64; the matrix entries are stored in
// the pair precision (FP32 in the mixed build).
//
// Assembly and the force gather give each row LPR consecutive lanes, which
// read consecutive entries (neighbours in one cell, so their coordinates are
// gathered together) and combine by a fixed butterfly.  The charge-solve
// product runs one row per lane over a sliced copy of the rows, made once per
// step, where entry e of 64 consecutive rows is one contiguous segment.
#pragma once
#include "ctbop_dev.h"
#include "k_tersoff.h"

namespace ctbop {

// Shielded, tapered Coulomb kernel C(r) = ke T(r/rc) (r^3 + g3)^(-1/3) and
// (dC/dr)/r, evaluated in FP64 for a given distance: an FP32 seed of the
// reciprocal cube root and one Newton step, y <- y (4 - u y^3) / 3, leave a
// relative error of ~1e-13, so the only error left in the matrix entries is
// the (unbiased) rounding of r itself and of the stored FP32 value.
// The radial derivative comes divided by r, without a division: with
// T'(x) = -140 x^3 (1-x)^3 and x = r/rc,
//   (dC/dr)/r = ke [ -140 x^2 (1-x)^3 y / rc^2 - T r y^4 ].
__device__ __forceinline__ double rcbrt64(double u)
{
    // u^(-1/3) for u = r^3 + g3 > 0 (pairs are never closer than 0.5 A): the
    // hardware FP32 log2/exp2 seed (~1e-7) and one FP64 Newton step
    const double y = (double)__builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf((float)u));
    return y * (4.0 - u * y * y * y) * (1.0 / 3.0);
}

// g3 = gamma_ij^-3 of the pair
__device__ __forceinline__ double coul64_g(const Params<double> &P, double g3, double r, double &dCr)
{
    const double x = r * P.inv_rc, x2 = x * x, x3 = x2 * x;
    const double om = 1.0 - x, om2 = om * om;
    const double T = om2 * om2 * (1.0 + 4.0 * x + 10.0 * x2 + 20.0 * x3);
    const double u = r * r * r + g3;
    const double y = rcbrt64(u);
    const double y2 = y * y;
    dCr = P.ke * (-140.0 * P.inv_rc * P.inv_rc * x2 * om2 * om * y - T * r * y2 * y2);
    return P.ke * T * y;
}

__device__ __forceinline__ double coul64(const Params<double> &P, int pp, double r, double &dCr)
{
    return coul64_g(P, P.g3[pp], r, dCr);
}

// The same in FP32 (the mixed build's force gather): the hardware log2/exp2
// seed and one FP32 Newton step leave ~1 ulp in y; the pair's energy and
// force terms are then summed in FP64.  Per pair ~1e-7 relative, against the
// 1e-6 eV/atom and 1e-5 relative-force budget.
__device__ __forceinline__ float coul32_g(float ke, float inv_rc, float g3, float r, float &dCr)
{
    const float x = r * inv_rc, x2 = x * x, x3 = x2 * x;
    const float om = 1.0f - x, om2 = om * om;
    const float T = om2 * om2 * (1.0f + 4.0f * x + 10.0f * x2 + 20.0f * x3);
    const float u = r * r * r + g3;
    float y = __builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf(u));
    y = y * (4.0f - u * y * y * y) * 0.333333343f;
    const float y2 = y * y;
    dCr = ke * (-140.0f * inv_rc * inv_rc * x2 * om2 * om * y - T * r * y2 * y2);
    return ke * T * y;
}

__device__ __forceinline__ double coul64_val_g(const Params<double> &P, double g3, double r)
{
    const double x = r * P.inv_rc, x2 = x * x, x3 = x2 * x;
    const double om = 1.0 - x, om2 = om * om;
    const double T = om2 * om2 * (1.0 + 4.0 * x + 10.0 * x2 + 20.0 * x3);
    const double u = r * r * r + g3;
    const double y = rcbrt64(u);
    return P.ke * T * y;
}

__device__ __forceinline__ double coul64_val(const Params<double> &P, int pp, double r)
{
    return coul64_val_g(P, P.g3[pp], r);
}

struct CgCtl {
    double tol;
    int maxit;
};

// Distance of a list entry, in the pair precision R and then widened: every
// kernel that tests it against rc computes it this one way, so all of them
// agree on which entries lie inside.
template <typename R>
__device__ __forceinline__ double entry_r(const typename Vec4<R>::type &li, const typename Vec4<R>::type &lj,
                                          const typename Vec4<R>::type &D, R3<R> &d)
{
    d = pair_vec<R>(li, lj, D);
    return (double)dev_sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
}

// Assemble the Coulomb rows of the step: the list entries inside rc, in list
// order, into hidx/Hr (group ballots give each lane its place), and the
// starting residual r = -(H q0 + chi) + mu_prev.  A row is flagged (hwide)
// when one of its entries lies further from the tile than a 16-bit offset
// from any slice of the tile reaches (which keeps it in the halo window too).
template <typename R, int LPR>
__global__ void __launch_bounds__(TILE) k_assemble(const Tile *tiles, Seg *segs, Params<double> PD)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ V4 dtab[NCODE];
    load_dtab2<R>(S, dtab);
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    const auto qv = gbl(S.q);
    R *Hr = reinterpret_cast<R *>(S.Hr);
    const double mprev = S.sst->mu_prev;
    constexpr int G = TILE / LPR;
    const int lane = threadIdx.x % LPR;
    const unsigned below = (1u << lane) - 1u;
    // Each group stages its kept entries in LDS and writes them out FL at a
    // time: whole 128-byte lines of hidx (rows start on 2 KB boundaries), so
    // no line of the output is written in pieces.
    constexpr int FL = 32;
    __shared__ uint32_t bidx_lds[G][FL + LPR];
    __shared__ R bval_lds[G][FL + LPR];
    uint32_t *bi = bidx_lds[threadIdx.x / LPR];
    R *bv = bval_lds[threadIdx.x / LPR];
    for (int k = threadIdx.x / LPR; k < TILE; k += G) {
        const int s = T.row0 + k;
        if (s >= S.n) {
            if (s < S.npad && lane == 0) {
                S.hcnt[s] = 0;
                S.hwide[s] = 0;
            }
            continue;                          // the whole group skips together
        }
        const V4 li = xs[s];
        const int ti = (int)li.w;
        const double g3_0 = PD.g3[ti * 2], g3_1 = PD.g3[ti * 2 + 1];
        const int cnt = S.lcnt[s];
        const auto row = gbl(S.lidx + (size_t)s * S.Wl);
        const auto hrow = gblw(S.hidx + (size_t)s * S.Wl);
        const auto vrow = gblw(Hr + (size_t)s * S.Wl);
        double acc = 0.0;
        int nbuf = 0, done = 0;
        bool wide = false;
        const int tbase = s & ~(TILE - 1);      // the row may take any slice of its tile
        for (int e0 = 0; e0 < cnt; e0 += LPR) {
            const int e = e0 + lane;
            bool in = false;
            uint32_t ent = 0;
            int j = 0, tj = 0;
            double r = 0.0, qj = 0.0;
            if (e < cnt) {
                ent = row[e];
                j = (int)(ent & J_MASK);
                const V4 lj = ld4<R>(xs, j);
                qj = qv[j];                      // loaded beside the position (most entries are kept)
                tj = (int)lj.w;
                R3<R> d;
                r = entry_r<R>(li, lj, dtab[ent >> CODE_SHIFT], d);
                in = r < PD.rc;
            }
            const unsigned gm = group_ballot<LPR>(in);
            double cv = 0.0;
            if (in) {
                const int at = nbuf + __popc(gm & below);
                const R c = (R)coul64_val_g(PD, tj ? g3_1 : g3_0, r);
                bi[at] = ent;
                bv[at] = c;
                cv = (double)c;
                const int off = j - tbase;
                wide = wide || off - (TILE - SLICE) < -32768 || off > 32767;
            }
            acc += cv * qj;
            nbuf += __popc(gm);
            __builtin_amdgcn_wave_barrier();
            if (nbuf >= FL) {
                for (int t = lane; t < FL; t += LPR) {
                    hrow[done + t] = bi[t];
                    vrow[done + t] = bv[t];
                }
                const int rest = nbuf - FL;      // < LPR
                uint32_t ri = 0;
                R rv = (R)0;
                if (lane < rest) {
                    ri = bi[FL + lane];
                    rv = bv[FL + lane];
                }
                __builtin_amdgcn_wave_barrier();
                if (lane < rest) {
                    bi[lane] = ri;
                    bv[lane] = rv;
                }
                __builtin_amdgcn_wave_barrier();
                done += FL;
                nbuf = rest;
            }
        }
        for (int t = lane; t < nbuf; t += LPR) {
            hrow[done + t] = bi[t];
            vrow[done + t] = bv[t];
        }
        __builtin_amdgcn_wave_barrier();
        acc = group_sum<LPR>(acc);
        wide = group_ballot<LPR>(wide) != 0u;
        if (lane == 0) {
            const double qs = S.q[s];
            S.hcnt[s] = done + nbuf;
            S.hwide[s] = wide ? 1 : 0;
            S.jd[s] = PD.J[ti];
            S.r[s] = -(PD.J[ti] * qs + acc + PD.chi[ti]) + mprev;
            S.p[s] = 0.0;
        }
    }
}

// Sliced copy (hsidx, H) of the step's rows (hidx, Hr) for the charge-solve
// product, and the block-Jacobi preconditioner.  Each block first orders its
// tile's rows by decreasing length (the slot order, hperm), then transposes
// the tile one slice (SLICE slots) at a time through LDS, in chunks of HS_CH
// entries per row: four lanes read one row's chunk, 16 bytes each, of hidx
// and Hr (chunks of 16 rather than 32 entries keep the block's LDS under
// 40 KB, four blocks per CU: 736 -> 693 us), and add the entries whose
// neighbour lies in the row's own BK-row block into that block row in LDS,
// the four lanes in turn (so the additions keep list order); then every lane
// writes entries of its slot as slice columns (64 lanes store contiguous
// memory).  The tile's blocks (J on the diagonal) are then inverted in LDS by
// Gauss-Jordan elimination in FP32 (H is SPD and its blocks well conditioned,
// so no pivoting; the preconditioner only has to be symmetric positive
// definite, its accuracy sets the iteration count, not the solution),
// symmetrised and written with their row sums; the tile's partial sums of
// r m1 and m1 start the projection.
constexpr int HS_CH = 16;                // entries per row and chunk (4 lanes x 4)
constexpr int HS_E = HS_CH / 4;
constexpr int HS_LPR = 4;                // lanes reading one row's chunk

// entries e0 .. e0+N-1 of a row-major row (fewer when the row ends first)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int N, typename T>
__device__ __forceinline__ void loadN(const __attribute__((address_space(1))) T *row, int e0, int cnt, bool vec,
                                      T (&out)[N])
{
    if (vec && e0 + N <= cnt) {
        const __attribute__((address_space(1))) u32x4 *src = (const __attribute__((address_space(1))) u32x4 *)(row + e0);
        u32x4 w[N * sizeof(T) / 16];
#pragma unroll
        for (int k = 0; k < (int)(N * sizeof(T) / 16); k++) w[k] = src[k];
        memcpy(out, w, sizeof out);
    } else {
#pragma unroll
        for (int k = 0; k < N; k++) out[k] = e0 + k < cnt ? row[e0 + k] : (T)0;
    }
}

template <typename R>
__global__ void __launch_bounds__(TILE) k_hslice(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ uint32_t ci[SLICE][HS_CH + 1];
    __shared__ R cv[SLICE][HS_CH + 1];
    __shared__ float A[TILE / BK][BK][BK + 1];
    __shared__ int cnt_lds[TILE];
    __shared__ int slot_row[TILE];
    __shared__ int slot_cnt[TILE];
    __shared__ uint8_t wide_row[TILE];
    __shared__ uint8_t sw[TILE / SLICE];
    __shared__ double lds[4 * 6];
    __shared__ unsigned long long hbm[HALO_WORDS];
    __shared__ uint16_t hpre[HALO_WORDS];
    const int tid = threadIdx.x;
    const int own = T.row0 + tid;
    const bool live = own < S.n;
    const int own_cnt = live ? S.hcnt[own] : 0;
    cnt_lds[tid] = own_cnt;
    float *Af = &A[0][0][0];
    for (int w = tid; w < TILE / BK * BK * (BK + 1); w += TILE) Af[w] = 0.0f;
    wide_row[tid] = (live && S.hwide[own] != 0) ? 1 : 0;
    // the tile's halo bitmap: an entry's place in the halo is the set bits before its own
    const int tl = T.row0 / TILE;
    const bool hfit = S.nhalo[tl] <= HALO_MAX;
    if (hfit) {
        for (int w = tid; w < HALO_WORDS; w += TILE) {
            hbm[w] = S.hbits[(size_t)tl * HALO_WORDS + w];
            hpre[w] = S.hpre[(size_t)tl * HALO_WORDS + w];
        }
    }
    __syncthreads();
    // slot of each row: longer rows first, ties by row
    int rank = 0;
    for (int k = 0; k < TILE; k++) {
        const int c = cnt_lds[k];
        rank += (c > own_cnt || (c == own_cnt && k < tid)) ? 1 : 0;
    }
    slot_row[rank] = tid;
    slot_cnt[rank] = own_cnt;
    __syncthreads();
    // thread tid's slot is tid (row rk); a wave is a slice: the full form
    // when one of its rows needs it, else halo positions when the halo fits,
    // else 16-bit offsets from the slice's first slot
    const int rk = slot_row[tid];
    const int rrow = T.row0 + rk;
    S.hperm[own] = (uint8_t)rk;
    const uint8_t smode = __ballot(wide_row[rk] != 0) != 0ull ? SL_FULL : (hfit ? SL_HALO : SL_OFF16);
    if ((tid & (SLICE - 1)) == 0) {
        S.swide[own / SLICE] = smode;
        sw[tid / SLICE] = smode;
    }
    // slots padded to the slice's longest row (its first slot)
    const double slots = (tid & (SLICE - 1)) == 0 ? (double)SLICE * (double)slot_cnt[tid] : 0.0;
    __syncthreads();                         // every slice's form (sw) is set
    const R *Hr = reinterpret_cast<const R *>(S.Hr);
    const auto H = gblw(reinterpret_cast<R *>(S.H));
    const auto hsidx = gblw(S.hsidx);
    const auto hs16 = gblw(S.hs16);
    const bool vec = (S.Wl & 3) == 0;        // rows start on 16-byte boundaries
    for (int sl = 0; sl < TILE / SLICE; sl++) {
        const int slot0 = sl * SLICE;
        const int sbase = T.row0 + slot0;
        const int mlen = slot_cnt[slot0];
        const int mode = sw[sl];
        // reading: lanes 4l .. 4l+3 take slot l's row
        const int rl = tid / HS_LPR, rq = tid % HS_LPR;
        const int rrk = slot_row[slot0 + rl];
        const int rcnt = slot_cnt[slot0 + rl];
        const int rbb = (T.row0 + rrk) & ~(BK - 1);
        const auto irow = gbl(S.hidx + (size_t)(T.row0 + rrk) * S.Wl);
        const auto vrow = gbl(Hr + (size_t)(T.row0 + rrk) * S.Wl);
        // writing: lane l of wave w takes entries w, w+4, ... of slot l's chunk
        const int wl = tid % SLICE, wq = tid / SLICE;
        const int wcnt = slot_cnt[slot0 + wl];
        const size_t b0 = slice_base(sbase + wl, S.Wl);
        float *arow = &A[rrk / BK][rrk % BK][0];
        for (int E0 = 0; E0 < mlen; E0 += HS_CH) {
            const int e0 = E0 + rq * HS_E;
            if (e0 < rcnt) {
                uint32_t ie[HS_E];
                R ve[HS_E];
                loadN<HS_E>(irow, e0, rcnt, vec, ie);
                loadN<HS_E>(vrow, e0, rcnt, vec, ve);
#pragma unroll
                for (int k = 0; k < HS_E; k++) {
                    ci[rl][rq * HS_E + k] = ie[k];
                    cv[rl][rq * HS_E + k] = ve[k];
                }
                // entries whose neighbour lies in the row's own block, added
                // into its block row by the row's four lanes in turn (the
                // lanes of one wave: their LDS accesses stay in order), so
                // the additions keep list order
                for (int q4 = 0; q4 < HS_LPR; q4++) {
                    if (rq == q4) {
#pragma unroll
                        for (int k = 0; k < HS_E; k++) {
                            const unsigned col = (unsigned)((int)(ie[k] & J_MASK) - rbb);
                            if (e0 + k < rcnt && col < (unsigned)BK) arow[col] += (float)ve[k];
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < HS_CH / 4; k++) {
                const int c = wq + 4 * k;
                const int e = E0 + c;
                if (e < wcnt) {
                    const uint32_t ent = ci[wl][c];
                    if (mode == SL_HALO) {
                        const int hw = (int)(ent & J_MASK) - T.row0 + HALO_WIN / 2;
                        const unsigned long long below = (1ull << (hw & 63)) - 1ull;
                        hs16[b0 + (size_t)e * SLICE] = (uint16_t)(hpre[hw >> 6] + __popcll(hbm[hw >> 6] & below));
                    } else if (mode == SL_OFF16) {
                        hs16[b0 + (size_t)e * SLICE] = (uint16_t)((int)(ent & J_MASK) - sbase + 32768);
                    } else {
                        hsidx[b0 + (size_t)e * SLICE] = ent;
                    }
                    H[b0 + (size_t)e * SLICE] = cv[wl][c];
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // the tile's BK x BK blocks ([block][row][col]) hold the block rows; add
    // J on the diagonal (identity rows past n), then one row per thread in row order
    {
        const bool rlive = rrow < S.n;
        const int rb = rk / BK, ri = rk % BK;
        if (rlive) {
            A[rb][ri][ri] += (float)S.jd[rrow];
        } else {
#pragma unroll
            for (int t = 0; t < BK; t++) A[rb][ri][t] = (t == ri ? 1.0f : 0.0f);
        }
    }
    __syncthreads();
    const int blk = tid / BK, i = tid % BK;
    // in-place Gauss-Jordan inversion, thread i updates row i
    for (int k = 0; k < BK; k++) {
        const float piv = 1.0f / A[blk][k][k];
        const float aik = A[blk][i][k];
        float rowk[BK];
#pragma unroll
        for (int t = 0; t < BK; t++) rowk[t] = A[blk][k][t];
        __syncthreads();
        if (i == k) {
#pragma unroll
            for (int t = 0; t < BK; t++) A[blk][k][t] = (t == k) ? piv : rowk[t] * piv;
        } else {
            const float f = aik * piv;
#pragma unroll
            for (int t = 0; t < BK; t++) A[blk][i][t] = (t == k) ? -f : A[blk][i][t] - f * rowk[t];
        }
        __syncthreads();
    }
    // row i of the block (symmetrised), rounded to FP16 and stored as the
    // row's 16 entries; the row sum m1 is taken from the rounded entries, so
    // that the projection uses exactly the preconditioner that is applied
    double m1 = 0.0;
    _Float16 *bo = S.binv + (size_t)(T.row0 + blk * BK + i) * BK;
#pragma unroll
    for (int t = 0; t < BK; t++) {
        const _Float16 b = (_Float16)(0.5f * (A[blk][i][t] + A[blk][t][i]));
        bo[t] = b;
        m1 += (double)(float)b;
    }
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (live) {
        S.m1[own] = m1;
        v[0] = S.r[own] * m1;
        v[1] = (double)own_cnt;
        v[2] = sw[rank / SLICE] == SL_FULL ? (double)own_cnt : 0.0;
        v[4] = m1;
        v[5] = sw[rank / SLICE] == SL_HALO ? (double)own_cnt : 0.0;
    } else if (own < S.npad) {
        S.m1[own] = 0.0;
    }
    v[3] = slots;
    tile_partials<6>(S, T.row0 / TILE, v, lds);
}

// y = M r for row s: the row of s's block inverse (16 FP16 entries, two
// 16-byte loads) against the block's r, exchanged by shuffles within the BK
// lanes of the block (every lane of the block must call it; rows past n pass
// r = 0).  The inverse only sets the iteration count: symmetric and positive
// definite after rounding (its entries move by ~5e-4 relative, its smallest
// eigenvalues are ~1e-2 of its largest), so the solution is unchanged.
__device__ __forceinline__ double block_apply(const _Float16 *binv, int s, double r)
{
    static_assert(BK == 16, "a row of the block is two 16-byte words");
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    const auto B = gbl(reinterpret_cast<const h8 *>(binv + (size_t)s * BK));
    const h8 b0 = B[0], b1 = B[1];
    double y = 0.0;
#pragma unroll
    for (int t = 0; t < 8; t++) y += (double)(float)b0[t] * __shfl(r, t, BK);
#pragma unroll
    for (int t = 0; t < 8; t++) y += (double)(float)b1[t] * __shfl(r, 8 + t, BK);
    return y;
}

// First pass over the starting residual: its M-weighted mean w0 = 1^T M r /
// 1^T M 1, and the start of the single-reduction solve, whose first update
// shifts r by w0 (the shift left by rounding is measured by its first
// finalize and removed with the next update's shift; the charge coupling's
// solve and the adjoint take a second pass instead, k_shift_stats and
// k_fin_assemble, which set the state again).
__global__ void k_fin_w0(const int *seg_ids, Seg *segs)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[4 * 6];
    double tot[6];
    seg_total<6>(S, lds, tot);
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        st->sdinv = tot[4];
        st->w = tot[0] / tot[4];
        st->nnz_coul = tot[1];
        st->nnz_wide = tot[2];
        st->nnz_slots = tot[3];
        st->nnz_halo = tot[5];
        st->mshift = st->mu_prev - st->w;
        st->iters = 0;
        st->qshift = 0.0;
        st->cg_first = 1;
        st->cg_last = 0;
    }
}

// Second pass: r <- r - w0 and the sums of the shifted residual.  Forming
// r^T z and the projected norm from one-pass sums of the unshifted residual
// cancels catastrophically when r is nearly constant (for instance a
// single-species input, whose exact residual is constant).
__global__ void __launch_bounds__(TILE) k_shift_stats(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[4 * 4];
    const int s = T.row0 + threadIdx.x;
    const bool live = s < S.n;
    // the segment's pointers in registers before the first store
    const auto rv = gblw(S.r);
    const auto yv = gblw(S.y);
    const auto m1 = gbl(S.m1);
    const _Float16 *binv = S.binv;
    double r = 0.0;
    if (live) {
        const double w = S.sst->w;
        r = rv[s] - w;
        rv[s] = r;
        if (S.rl) S.rl[s] -= w;              // f_q coupling: the quadratic part too
    }
    const double y = block_apply(binv, s, r);
    double v[4] = {0, 0, 0, 0};
    if (live) {
        yv[s] = y;
        v[0] = r * m1[s];
        v[1] = r * y;
        v[2] = r;
        v[3] = r * r;
    }
    tile_partials<4>(S, T.row0 / TILE, v, lds);
}

__global__ void k_fin_assemble(const int *seg_ids, Seg *segs, CgCtl ctl)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[4 * 4];
    double tot[4];
    seg_total<4>(S, lds, tot);
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        const double w0 = st->w;
        const double w = tot[0] / st->sdinv;          // residual shift left after the first pass
        const double res2 = (tot[3] - tot[2] * tot[2] / S.n) / S.n;
        st->w = w;
        st->rho = tot[1] - w * tot[0];
        st->beta = 0.0;
        st->res = sqrt(fmax(res2, 0.0));
        st->res0 = st->res;
        st->mshift = st->mu_prev - w0 - w;
        st->iters = 0;
        st->qshift = 0.0;
        st->cg_first = 1;
        st->cg_last = 0;
        st->done = (st->res < ctl.tol) ? 1 : 0;
    }
}

// r <- r - w,  p <- M (r - w 1) + beta p = (y - w m1) + beta p (the charge
// coupling's nonlinear solve; the linear solves use the single-reduction form)
__global__ void __launch_bounds__(TILE) k_cg_dir(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done) return;
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n) return;
    const double w = S.sst->w, beta = S.sst->beta;
    const auto rv = gblw(S.r);
    const auto pv = gblw(S.p);
    const double y = gbl(S.y)[s], m1 = gbl(S.m1)[s], p = pv[s];
    const double r = rv[s] - w;
    rv[s] = r;
    pv[s] = (y - w * m1) + beta * p;
    if (S.rl) S.rl[s] -= w;                  // f_q coupling: the quadratic part too
}

// s = H p and the tile's share of p^T s, one row per lane; U entries of the
// row are loaded before their products are summed, so U gathers of p are in
// flight per lane (U accumulators, combined in a fixed order at the end).
template <typename R, int U, typename IDX>
__device__ __forceinline__ double spmv_row(const double *p_, const IDX *row_, const R *hrow_, int cnt, int jbase)
{
    const auto p = gbl(p_);
    const auto row = gbl(row_);
    const auto hrow = gbl(hrow_);
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; u++) acc[u] = 0.0;
    int e = 0;
    for (; e + U <= cnt; e += U) {
        IDX jj[U];
        R hh[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            jj[u] = __builtin_nontemporal_load(row + (size_t)(e + u) * SLICE);
            hh[u] = __builtin_nontemporal_load(hrow + (size_t)(e + u) * SLICE);
        }
#pragma unroll
        for (int u = 0; u < U; u++) acc[u] += (double)hh[u] * p[jbase + (int)(jj[u] & J_MASK)];
    }
    for (; e < cnt; e++)
        acc[0] += (double)__builtin_nontemporal_load(hrow + (size_t)e * SLICE) *
                  p[jbase + (int)(__builtin_nontemporal_load(row + (size_t)e * SLICE) & J_MASK)];
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) a += acc[u];
    return a;
}

// The same with p of the tile's halo staged in LDS (hp) and the row's
// entries as 16-bit halo positions; products and sums in the same order.
template <typename R, int U>
__device__ __forceinline__ double spmv_row_halo(const double *hp, const uint16_t *row_, const R *hrow_, int cnt)
{
    const auto row = gbl(row_);
    const auto hrow = gbl(hrow_);
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; u++) acc[u] = 0.0;
    int e = 0;
    for (; e + U <= cnt; e += U) {
        uint16_t jj[U];
        R hh[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            jj[u] = __builtin_nontemporal_load(row + (size_t)(e + u) * SLICE);
            hh[u] = __builtin_nontemporal_load(hrow + (size_t)(e + u) * SLICE);
        }
#pragma unroll
        for (int u = 0; u < U; u++) acc[u] += (double)hh[u] * hp[jj[u]];
    }
    for (; e < cnt; e++)
        acc[0] += (double)__builtin_nontemporal_load(hrow + (size_t)e * SLICE) *
                  hp[__builtin_nontemporal_load(row + (size_t)e * SLICE)];
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) a += acc[u];
    return a;
}

// What the product kernel computes: for the f_q coupling's nonlinear solve
// s = H p with p^T s and p^T r (the line search); for the single-reduction
// solve H y of y = M r, into hz, with the six sums its finalize needs.
enum SpmvMode { SP_FQ = 1, SP_CG1 = 2 };
constexpr int P_UPD = 0;    // single-reduction solve: partials 0..7 from the update,
constexpr int P_PRD = 8;    // 8..13 from the product
constexpr int P_CG1 = 14;   // partials the finalize adds up

// s = H p and the tile's share of p^T s, one slot (row) per lane over the
// sliced copy; U entries of the row are loaded before their products are
// summed (U accumulators, combined in a fixed order at the end).  The block
// first stages p of its tile's halo in LDS; a slice of halo positions then
// reads 6 bytes per entry from memory and p from LDS.  Slices of 16-bit
// offsets (the halo did not fit) or full entries gather p from memory.
template <typename R, int U, int MODE>
__global__ void __launch_bounds__(TILE) k_spmv(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done || (MODE == SP_CG1 && S.sst->cg_last)) return;
    __shared__ double lds[4 * 6];
    __shared__ double hp[HALO_MAX];
    const double *x = MODE == SP_CG1 ? S.y : S.p;
    // rows in order (the epilogue's loads and stores coalesce), loaded
    // first so that their latency hides behind the staging and the rows
    // (also in the FP64 kernel, where they cost a wave per SIMD: loading
    // them after the rows was slower)
    const int row = T.row0 + threadIdx.x;
    const bool live = row < S.n;
    double xs = 0.0, jd = 0.0, m1s = 0.0, rs = 0.0, ss = 0.0;
    if (live) {
        xs = x[row];
        jd = S.jd[row];
        if (MODE == SP_CG1) {
            m1s = S.m1[row];
            rs = S.r[row];
            ss = S.s[row];
        }
        if (MODE == SP_FQ) rs = S.r[row];
    }
    const int tl = T.row0 / TILE;
    const int nh = S.nhalo[tl];
    if (nh <= HALO_MAX) {
        const auto hl = gbl(S.halo + (size_t)tl * HALO_MAX);
        const auto pg = gbl(x);
        for (int k = threadIdx.x; k < nh; k += TILE) hp[k] = pg[hl[k]];
    }
    __syncthreads();
    // lane = slot: its row's off-diagonal sum, handed to the row's lane in LDS
    const int slot = T.row0 + threadIdx.x;
    const int rl = S.hperm[slot];
    const int s = T.row0 + rl;
    double a = 0.0;
    if (s < S.n) {
        const size_t b0 = slice_base(slot, S.Wl);
        const R *hrow = reinterpret_cast<const R *>(S.H) + b0;
        const int cnt = S.hcnt[s];
        const int mode = S.swide[slot / SLICE];
        a = mode == SL_HALO   ? spmv_row_halo<R, U>(hp, S.hs16 + b0, hrow, cnt)
            : mode == SL_FULL ? spmv_row<R, U, uint32_t>(x, S.hsidx + b0, hrow, cnt, 0)
                              : spmv_row<R, U, uint16_t>(x, S.hs16 + b0, hrow, cnt, (slot & ~(SLICE - 1)) - 32768);
    }
    __syncthreads();
    hp[rl] = a;
    __syncthreads();
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (live) {
        const double y = jd * xs + hp[threadIdx.x];
        if (MODE == SP_CG1) {
            S.hz[row] = y;
            v[0] = xs * y;                   // y^T H y
            v[1] = m1s * y;                  // m1^T H y
            v[2] = rs * y;                   // r^T H y
            v[3] = y * y;
            v[4] = ss * y;                   // s_old^T H y
            v[5] = y;
        } else {
            S.s[row] = y;
            v[0] = xs * y;
            v[1] = xs * rs;
        }
    }
    if (MODE == SP_CG1) {
        tile_partials_at<6>(S, tl, v, lds, P_PRD);
    } else {
        double w[2] = {v[0], v[1]};
        tile_partials<2>(S, tl, w, lds);
    }
}

// ---------------------------------------------------------------------------
// The same projected PCG with one reduction per iteration (Chronopoulos and
// Gear's rearrangement of conjugate gradients): the product is taken of
// y = M r, the unprojected preconditioned residual, and the direction's
// product follows by recurrence, s = H y + beta s.  The projection enters as
// the shift c of the residual, r <- r - c 1 with c = m1^T r / 1^T M 1, so that
// y = M r is the projected preconditioned residual; c of the next residual is
// known one step ahead from m1^T r and m1^T s.  The finalize also takes the
// projected norm of the next residual, |r|^2 - 2 alpha r^T s + alpha^2 |s|^2
// (each minus its mean part), from sums of the two kernels, so the solve
// stops after the update that meets the tolerance without a further product.
// An iteration is four launches: product (k_spmv, SP_CG1), the finalize's two
// stages (k_cg1_sum, k_cg1_fin), update.
// ---------------------------------------------------------------------------

// p <- y + beta p, s <- H y + beta s, q <- q + alpha p, r <- r - alpha s - c,
// y <- M r, and the tile's sums for the finalize.  FIRST: the solve's start,
// which only shifts r (by the shift left after the second pass) and clears
// p and s.
template <bool FIRST>
__global__ void __launch_bounds__(TILE) k_cg1_update(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done) return;
    __shared__ double lds[4 * 8];
    const int s = T.row0 + threadIdx.x;
    const bool live = s < S.n;
    const double alpha = S.sst->alpha, beta = S.sst->beta, c = S.sst->w;
    // the segment's pointers in registers before the first store
    const auto qv = gblw(S.q);
    const auto rv = gblw(S.r);
    const auto yv = gblw(S.y);
    const auto pv = gblw(S.p);
    const auto sv = gblw(S.s);
    const auto hz = gbl(S.hz);
    const _Float16 *binv = S.binv;
    double q = 0.0, r = 0.0, sn = 0.0;
    if (live) {
        if (FIRST) {
            q = qv[s];
            r = rv[s] - c;
            pv[s] = 0.0;
            sv[s] = 0.0;
        } else {
            const double p = yv[s] + beta * pv[s];
            sn = hz[s] + beta * sv[s];
            q = qv[s] + alpha * p;
            r = (rv[s] - alpha * sn) - c;
            pv[s] = p;
            sv[s] = sn;
            qv[s] = q;
        }
        rv[s] = r;
    }
    const double y = block_apply(binv, s, r);
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
        yv[s] = y;
        v[0] = y;                // 1^T M r = m1^T r (M symmetric)
        v[1] = r * y;
        v[2] = r;
        v[3] = r * r;
        v[4] = q;
        v[5] = r * sn;
        v[6] = sn * sn;
        v[7] = sn;
    }
    tile_partials_at<8>(S, T.row0 / TILE, v, lds, P_UPD);
}

// The residual after the last update and the stop test; then gamma = r^T y,
// delta = y^T H y, beta = gamma / gamma_old, alpha = gamma / (delta -
// beta gamma / alpha_old) (= gamma / p^T H p), the next shift c and the
// projected norm of the next residual, which marks the coming update as the
// last when it meets the tolerance.
// First stage of the finalize: FIN_SPLIT blocks per segment, each summing
// the 15 partials over its range of tiles.
__global__ void __launch_bounds__(TILE) k_cg1_sum(const int *seg_ids, Seg *segs)
{
    const Seg &S = segs[seg_ids[blockIdx.x / FIN_SPLIT]];
    if (S.sst->done) return;
    __shared__ double lds[4 * P_CG1];
    seg_group_sum<P_CG1>(S, blockIdx.x % FIN_SPLIT, lds);
}

__global__ void __launch_bounds__(TILE) k_cg1_fin(const int *seg_ids, Seg *segs, CgCtl ctl)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (S.sst->done) return;
    __shared__ double lds[FIN_SPLIT * P_CG1];
    double t[P_CG1];
    seg_total_groups<P_CG1>(S, lds, t);
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        const double n = S.n;
        const double rr = t[P_UPD + 3] - t[P_UPD + 2] * t[P_UPD + 2] / n;
        st->res = sqrt(fmax(rr / n, 0.0));
        st->qshift = (S.Q - t[P_UPD + 4]) / n;
        const bool first = st->cg_first != 0;
        if (first) {
            st->res0 = st->res;
        } else {
            st->iters += 1;
            st->iters_total += 1;
        }
        if (st->cg_last || st->res < ctl.tol) {
            st->done = 1;
            return;
        }
        if (st->iters >= ctl.maxit) {
            st->done = 1;
            atomicOr(&st->status, ST_NOCONV);
            return;
        }
        const double gam = t[P_UPD + 1], del = t[P_PRD + 0];
        const double beta = first ? 0.0 : gam / st->rho;
        const double den = first ? del : del - beta * gam / st->alpha;
        if (!(den > 0.0) || !(gam > 0.0)) {
            atomicOr(&st->status, ST_NOT_PD);
            st->done = 1;
            return;
        }
        const double alpha = gam / den;
        // sums of the new s = H y + beta s_old (m1^T s by its own recurrence:
        // an error in it only leaves m1^T r of the next residual slightly off
        // zero, and the next shift, from the measured m1^T r, removes that)
        const double m1s = first ? t[P_PRD + 1] : t[P_PRD + 1] + beta * st->m1s;
        const double rs = t[P_PRD + 2] + beta * t[P_UPD + 5];
        const double ss = t[P_PRD + 3] + 2.0 * beta * t[P_PRD + 4] + beta * beta * t[P_UPD + 6];
        const double sum_s = t[P_PRD + 5] + beta * t[P_UPD + 7];
        const double c = (t[P_UPD + 0] - alpha * m1s) / st->sdinv;
        const double rs_p = rs - t[P_UPD + 2] * sum_s / n;
        const double ss_p = ss - sum_s * sum_s / n;
        const double next2 = (rr - 2.0 * alpha * rs_p + alpha * alpha * ss_p) / n;
        st->cg_first = 0;
        st->m1s = m1s;
        st->rho = gam;
        st->alpha = alpha;
        st->beta = beta;
        st->w = c;
        st->mshift -= c;
        if (next2 < ctl.tol * ctl.tol) st->cg_last = 1;
    }
}

// Coulomb forces and energy at the equilibrated charges, plus the covalent
// forces and energies: writes F, q (user order) and the tile's energy.
template <typename R, int LPR>
__global__ void __launch_bounds__(TILE) k_force_coul(const Tile *tiles, Seg *segs, Params<double> PD, int gate)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (gate && (!S.sst->done || S.sst->forces_done)) return;
    __shared__ V4 dtab[NCODE];
    __shared__ double lds[4 * 3];
    load_dtab2<R>(S, dtab);
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    const auto qv = gbl(S.q);
    const double qsh = S.sst->qshift;
    const bool keep_hist = S.q_ring != nullptr;
    const int push = (S.sst->qhead + 1) % NHIST;       // ring slot that takes the previous solution
    constexpr int G = TILE / LPR;
    const int lane = threadIdx.x % LPR;
    const float ke32 = (float)PD.ke, irc32 = (float)PD.inv_rc;
    double esum = 0.0;
    // bond statistics of the step (for the measurement): bonds and ordered bond pairs
    double nb = 0.0, nt = 0.0;
    if (T.row0 + (int)threadIdx.x < S.n) {
        nb = (double)S.bcnt[T.row0 + threadIdx.x];
        nt = nb * (nb - 1.0);
    }
    for (int k = threadIdx.x / LPR; k < TILE; k += G) {
        const int s = T.row0 + k;
        if (s >= S.n) continue;
        const V4 li = xs[s];
        const int ti = (int)li.w;
        const double g3_0 = PD.g3[ti * 2], g3_1 = PD.g3[ti * 2 + 1];
        const float g3f_0 = (float)g3_0, g3f_1 = (float)g3_1;
        const int cnt = S.hcnt[s];
        const auto row = gbl(S.hidx + (size_t)s * S.Wl);
        double ec = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        for (int e = lane; e < cnt; e += LPR) {
            const uint32_t ent = row[e];
            const int j = (int)(ent & J_MASK);
            const V4 lj = ld4<R>(xs, j);
            const double qj = qv[j] + qsh;
            // every entry lies inside rc: the rows were selected by the
            // assembly's distance test (entry_r).  With FP32 pair terms the
            // distance is taken with the hardware square root (~1 ulp, as
            // close as the FP32 pair function itself) and needs no test; the
            // FP64 build keeps the test, as a select rather than a branch so
            // that the loop body stays one block and the charge load issues
            // beside the position load
            R3<R> d;
            double r;
            if constexpr (sizeof(R) == 4) {
                d = pair_vec<R>(li, lj, dtab[ent >> CODE_SHIFT]);
                r = (double)__builtin_amdgcn_sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
            } else {
                r = entry_r<R>(li, lj, dtab[ent >> CODE_SHIFT], d);
            }
            const bool in = sizeof(R) == 4 ? true : r < PD.rc;
            double dCr, c;
            if constexpr (sizeof(R) == 4) {
                float d32;
                c = (double)coul32_g(ke32, irc32, (int)lj.w ? g3f_1 : g3f_0, (float)r, d32);
                dCr = (double)d32;
            } else {
                c = coul64_g(PD, (int)lj.w ? g3_1 : g3_0, r, dCr);
            }
            c = in ? c : 0.0;
            dCr = in ? dCr : 0.0;
            ec += c * qj;
            if (j != s) {
                const double g = qj * dCr;
                fx += g * (double)d.x;
                fy += g * (double)d.y;
                fz += g * (double)d.z;
            }
        }
        ec = group_sum<LPR>(ec);
        fx = group_sum<LPR>(fx);
        fy = group_sum<LPR>(fy);
        fz = group_sum<LPR>(fz);
        if (lane == 0) {
            const double qs = S.q[s] + qsh;
            const int i = S.perm[s];
            S.F[i] = qs * fx + S.Fcov[s];
            S.F[S.n + i] = qs * fy + S.Fcov[S.npad + s];
            S.F[2 * S.n + i] = qs * fz + S.Fcov[2 * S.npad + s];
            S.q_out[i] = qs;
            if (keep_hist) S.q_ring[(size_t)push * S.n + i] = S.q_state[i];
            S.q_state[i] = qs;
            esum += PD.E0[ti] + PD.chi[ti] * qs + 0.5 * PD.J[ti] * qs * qs + 0.5 * qs * ec + S.ecov[s];
        }
    }
    double v[3] = {esum, nb, nt};
    tile_partials<3>(S, T.row0 / TILE, v, lds);
}

__global__ void k_fin_energy(const int *seg_ids, Seg *segs, int gate)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (gate && (!S.sst->done || S.sst->forces_done)) return;
    __shared__ double lds[4 * 3];
    double tot[3];
    seg_total<3>(S, lds, tot);
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        st->energy = tot[0];
        st->nbond = tot[1];
        st->ntrip = tot[2];
        if (S.E_out) *S.E_out = tot[0];
        st->mu_prev = st->mshift;
        st->nhist = st->nhist < NHIST + 1 ? st->nhist + 1 : NHIST + 1;
        if (S.q_ring) st->qhead = (st->qhead + 1) % NHIST;
        st->forces_done = 1;
    }
}

// serving: per-segment flags (done, forces_done, status, iterations)
__global__ void k_collect(const int *seg_ids, Seg *segs, int nseg, int4 *out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    const SegState *st = segs[seg_ids[k]].sst;
    out[k] = make_int4(st->done, st->forces_done, st->status, st->iters);
}

} // namespace ctbop
