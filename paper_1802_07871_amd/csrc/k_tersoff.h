// k_tersoff.h -- covalent part: bond pass and atomic-free force gather.
//
// Bond pass (one lane per sorted atom i): for every bond (i -> j), i.e. every
// covalent-list entry inside the cutoff S_ij, the environment sums of the two channels
//     zeta_l,ij = sum_{k != j} fc(r_ik) w_l(cos theta_ijk) exp[(alpha_l (r_ij - r_ik))^3]
// (Methods, Eq. 2, one per channel), the vectorised bond order
//     b_ij = G (sum_l (g_l + zeta_l^n_l)^-p)^(1/(2 sigma p))       (Eqs. 3-5, 7)
// and the bond energy 1/2 fc (fR - b fA).  Per entry it stores b_ij, the
// coefficients P_l = dE/dzeta_l,ij = -1/2 fc fA db/dzeta_l and the bond's
// attraction c_ij = fc b fA (which the charge coupling f_q scales).
//
// Force gather (one lane per sorted atom m) writes only F_m: every covalent
// term that moves with x_m, read back from the stored coefficients:
//   m as the centre i  : its own bonds (pair term) and their k environments;
//   m as the partner j : bonds (i -> m) of each neighbour i, found through the
//                        reverse-slot index, with i's environment k;
//   m as environment k : bonds (i -> k) of each neighbour i, with m in them.
// No atomics: each F_m is a plain sum in a fixed order (deterministic).
#pragma once
#include "ctbop_dev.h"

namespace ctbop {

template <typename R> struct R3 { R x, y, z; };

template <typename R>
__device__ __forceinline__ R dev_sqrt(R v) { return sqrt(v); }

// Reciprocal and square root of the covalent force terms: with FP32 terms the
// hardware instructions (~1 ulp, as close as the FP32 terms themselves),
// otherwise the correctly rounded operations.
__device__ __forceinline__ float term_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename R>
__device__ __forceinline__ R term_rcp(R x) { return (R)1 / x; }
__device__ __forceinline__ float term_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
template <typename R>
__device__ __forceinline__ R term_sqrt(R x) { return dev_sqrt(x); }

__device__ __forceinline__ void dev_sincos(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void dev_sincos(double a, double *s, double *c) { sincos(a, s, c); }

template <typename R>
__device__ __forceinline__ R cutoff(R r, R Rc, R Sc, R piSR, R &dfc)
{
    if (r <= Rc) { dfc = (R)0; return (R)1; }
    if (r >= Sc) { dfc = (R)0; return (R)0; }
    R sn, cs;
    dev_sincos(piSR * (r - Rc), &sn, &cs);
    dfc = (R)-0.5 * piSR * sn;
    return (R)0.5 + (R)0.5 * cs;
}

// angular function of channel l for centre species t (and d/dcos):
// w = gam (1 + (c^2/d^2) x^2 / (d^2 + x^2)), x = h - cos, one division
template <typename R>
__device__ __forceinline__ R angular(const Params<R> &P, int t, int l, R cs, R &dw)
{
    const R x = P.h[t][l] - cs;
    const R iden = term_rcp(P.d2[t][l] + x * x);
    const R w = P.gam[t][l] * ((R)1 + P.c2d2[t][l] * x * x * iden);
    dw = -P.gam[t][l] * P.c2[t][l] * (R)2 * x * iden * iden;
    return w;
}

template <typename R>
__device__ __forceinline__ R radial(const Params<R> &P, int t, int l, R dl, R &de)
{
    R a = P.alpha[t][l] * dl;
    R e = exp(a * a * a);
    de = (R)3 * P.alpha[t][l] * a * a * e;
    return e;
}

// vectorised bond order and its derivatives in zeta_1, zeta_2
template <typename R>
__device__ __forceinline__ R bond_order(const Params<R> &P, int t, R z1, R z2, R &db1, R &db2)
{
    R zn1 = z1 > (R)0 ? pow(z1, P.nn[t][0]) : (R)0;
    R zn2 = z2 > (R)0 ? pow(z2, P.nn[t][1]) : (R)0;
    R zh1 = P.g[t][0] + zn1, zh2 = P.g[t][1] + zn2;
    R a1, a2, S, b;
    if (P.p_is_2) {
        R i1 = (R)1 / zh1, i2 = (R)1 / zh2;
        a1 = i1 * i1;
        a2 = i2 * i2;
        S = a1 + a2;
        b = P.G[t] * pow(S, P.inv2sig[t] * (R)0.5);
        a1 *= i1;                    // zh^-p-1
        a2 *= i2;
    } else {
        a1 = pow(zh1, -P.p);
        a2 = pow(zh2, -P.p);
        S = a1 + a2;
        b = P.G[t] * pow(S, P.inv2sig[t] / P.p);
        a1 /= zh1;
        a2 /= zh2;
    }
    R k = -b * P.inv2sig[t] / S;
    db1 = z1 > (R)0 ? k * P.nn[t][0] * (zn1 / z1) * a1 : (R)0;
    db2 = z2 > (R)0 ? k * P.nn[t][1] * (zn2 / z2) * a2 : (R)0;
    return b;
}

// Gradients w.r.t. the bond partner (gj) and the environment atom (gk) of the
// zeta_l term of a triplet: centre species tc, bond vector db (length rb),
// environment vector de (length re), environment cutoff pair penv.
template <typename R>
__device__ __forceinline__ void trip_grad(const Params<R> &P, int tc, int penv, const R3<R> &db, R rb,
                                          const R3<R> &de, R re, R3<R> gj[2], R3<R> gk[2])
{
    const R ib = term_rcp(rb), ie = term_rcp(re);
    const R3<R> ub = {db.x * ib, db.y * ib, db.z * ib};
    const R3<R> ue = {de.x * ie, de.y * ie, de.z * ie};
    const R cs = ub.x * ue.x + ub.y * ue.y + ub.z * ue.z;
    const R3<R> cb = {(ue.x - cs * ub.x) * ib, (ue.y - cs * ub.y) * ib, (ue.z - cs * ub.z) * ib};
    const R3<R> ce = {(ub.x - cs * ue.x) * ie, (ub.y - cs * ue.y) * ie, (ub.z - cs * ue.z) * ie};
    R dfe;
    const R fe = cutoff(re, P.Rc[penv], P.Sc[penv], P.piSR[penv], dfe);
#pragma unroll
    for (int l = 0; l < 2; l++) {
        R dw, de_ = (R)0, ex = (R)1;
        const R w = angular(P, tc, l, cs, dw);
        if (!P.alpha_zero[tc]) ex = radial(P, tc, l, rb - re, de_);
        const R a = fe * dw * ex, bcoef = fe * w * de_, c = dfe * w * ex;
        gj[l].x = a * cb.x + bcoef * ub.x;
        gj[l].y = a * cb.y + bcoef * ub.y;
        gj[l].z = a * cb.z + bcoef * ub.z;
        gk[l].x = c * ue.x + a * ce.x - bcoef * ue.x;
        gk[l].y = c * ue.y + a * ce.y - bcoef * ue.y;
        gk[l].z = c * ue.z + a * ce.z - bcoef * ue.z;
    }
}

template <typename R>
__device__ __forceinline__ R3<R> pair_vec(const typename Vec4<R>::type &a, const typename Vec4<R>::type &b,
                                          const typename Vec4<R>::type &D)
{
    R3<R> v = {(b.x - a.x) + D.x, (b.y - a.y) + D.y, (b.z - a.z) + D.z};
    return v;
}

template <typename R>
__device__ __forceinline__ void load_dtab2(const Seg &S, typename Vec4<R>::type *tab)
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

constexpr int BOND_CACHE = 4;           // bonds per atom whose geometry the bond pass keeps in LDS

// The parameters in LDS: the triplet loops index them by species, and
// per-lane indexed reads of the kernel-argument copy go through the vector
// memory path (and are read again in every iteration for want of registers).
template <typename P>
__device__ __forceinline__ void stage_params(const P &src, P &dst)
{
    static_assert(sizeof(P) % 4 == 0, "parameter block of whole words");
    const int *a = reinterpret_cast<const int *>(&src);
    int *b = reinterpret_cast<int *>(&dst);
    for (int k = threadIdx.x; k < (int)(sizeof(P) / 4); k += blockDim.x) b[k] = a[k];
}

// Bond pass.  First the bonds of the step: the covalent-list entries inside
// S_ij, by the FP64 distance used below, compacted in list order (so every
// loop over bonds and triplets runs over bonds only; the skin shell of the
// covalent list, e.g. the twelve second neighbours of Si in SiC, drops out),
// with the slot map that lets the force gather find each bond's reverse.
// The bond pass runs in FP64 from the FP64 local coordinates: it is a small
// share of the step (a few bonds per atom), and FP64 keeps the energy free of
// FP32 rounding in zeta, b and the large, cancelling fR and b fA terms.  The
// coefficients are stored in the pair precision R for the force gather.
template <typename R>
__global__ void __launch_bounds__(TILE) k_bond(const Tile *tiles, Seg *segs, Params<double> Pk)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double4 dtab[NCODE];
    __shared__ Params<double> Pl;
    // the first BOND_CACHE bonds of each row of the tile: vector, length and
    // pair type, computed once for the triplet loop (the cutoff value is
    // recomputed from the length: 1 below R, which most bonds are, so the
    // block's LDS stays under a third of a CU's and three blocks fit)
    __shared__ double cbx[BOND_CACHE][TILE], cby[BOND_CACHE][TILE], cbz[BOND_CACHE][TILE];
    __shared__ double cbr[BOND_CACHE][TILE];
    __shared__ uint8_t cbp[BOND_CACHE][TILE];
    __shared__ int nb_lds[TILE];
    __shared__ uint8_t order[TILE];
    stage_params(Pk, Pl);
    load_dtab2<double>(S, dtab);            // (ends with a barrier)
    const Params<double> &P = Pl;
    const double4 *xs = S.xs64;
    const int Wb = S.Wb, Ws = S.Ws;
    // First, one row per lane (the sliced bond arrays are written a whole
    // segment per wave): the row's bonds, its bond count and the first
    // bonds' geometry.
    {
        const int s = T.row0 + threadIdx.x;
        int nb = -1;
        if (s < S.n) {
            const double4 li = ld4<double>(xs, s);
            const int ti = (int)li.w;
            const size_t rl = (size_t)s * Ws;
            const int ns = S.scnt[s];
            const auto sidx = gbl(S.sidx + rl);
            const auto srev = gbl(S.srev + rl);
            const auto bidx = gblw(S.bidx + slice_base(s, Wb));
            const auto bsrev = gblw(S.bsrev + slice_base(s, Wb));
            const auto cmap = gblw(S.cmap + slice_base(s, Ws));
            nb = 0;
            for (int e = 0; e < ns; e++) {
                const uint32_t ent = sidx[e];
                const double4 lj = ld4<double>(xs, ent & J_MASK);
                const int pp = ti * 2 + (int)lj.w;
                const R3<double> d = pair_vec<double>(li, lj, dtab[ent >> CODE_SHIFT]);
                const double r2 = d.x * d.x + d.y * d.y + d.z * d.z;
                uint8_t c = 255;
                if (r2 < P.Sc[pp] * P.Sc[pp]) {
                    if (nb < Wb) {
                        bidx[(size_t)nb * SLICE] = ent;
                        bsrev[(size_t)nb * SLICE] = srev[e];
                        c = (uint8_t)nb;
                        if (nb < BOND_CACHE) {
                            cbx[nb][threadIdx.x] = d.x;
                            cby[nb][threadIdx.x] = d.y;
                            cbz[nb][threadIdx.x] = d.z;
                            cbr[nb][threadIdx.x] = sqrt(r2);
                            cbp[nb][threadIdx.x] = (uint8_t)pp;
                        }
                    }
                    nb++;
                }
                cmap[(size_t)e * SLICE] = c;
            }
            if (nb > Wb) {
                atomicOr(&S.sst->status, ST_OVERFLOW);
                nb = Wb;
            }
            S.bcnt[s] = nb;
        } else if (s < S.npad) {
            S.ecov[s] = 0.0;
            S.bcnt[s] = 0;
        }
        nb_lds[threadIdx.x] = nb;
    }
    __syncthreads();
    // Then the triplet sums, bond orders and energies with the tile's rows
    // in order of decreasing bond count (ties by row): the loops run over
    // bond pairs, so the 64 rows a wave then holds have similar trip counts
    // (each row's results depend only on the row, not on the order).
    {
        const int own = nb_lds[threadIdx.x];
        int rank = 0;
        for (int k = 0; k < TILE; k++) {
            const int c = nb_lds[k];
            rank += (c > own || (c == own && k < (int)threadIdx.x)) ? 1 : 0;
        }
        order[rank] = (uint8_t)threadIdx.x;
    }
    __syncthreads();
    const int lr = order[threadIdx.x];
    const int s = T.row0 + lr;
    if (s >= S.n) return;
    const int nb = nb_lds[lr];
    const double4 li = ld4<double>(xs, s);
    const int ti = (int)li.w;
    V4 *slot = reinterpret_cast<V4 *>(S.slot) + slice_base(s, Wb);
    const auto row = gbl(S.bidx + slice_base(s, Wb));
    // bond e of the row: vector, length, cutoff value, pair type (the first
    // BOND_CACHE from LDS)
    auto bond = [&](int e, R3<double> &d, double &r, double &fcut, int &pp) {
        if (e < BOND_CACHE) {
            d.x = cbx[e][lr];
            d.y = cby[e][lr];
            d.z = cbz[e][lr];
            r = cbr[e][lr];
            pp = cbp[e][lr];
        } else {
            const uint32_t ent = row[(size_t)e * SLICE];
            const double4 lj = ld4<double>(xs, ent & J_MASK);
            pp = ti * 2 + (int)lj.w;
            d = pair_vec<double>(li, lj, dtab[ent >> CODE_SHIFT]);
            r = sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
        }
        double dummy;
        fcut = cutoff<double>(r, P.Rc[pp], P.Sc[pp], P.piSR[pp], dummy);
    };
    double ecov = 0.0;
    for (int e = 0; e < nb; e++) {
        R3<double> d;
        double r, fc;
        int pp;
        bond(e, d, r, fc, pp);
        double z1 = 0, z2 = 0;
        for (int e2 = 0; e2 < nb; e2++) {
            if (e2 == e) continue;
            R3<double> dk;
            double rk, fk;
            int pk;
            bond(e2, dk, rk, fk, pk);
            const double cs = (d.x * dk.x + d.y * dk.y + d.z * dk.z) / (r * rk);
            double dw, dex;
            double w1 = angular<double>(P, ti, 0, cs, dw), w2 = angular<double>(P, ti, 1, cs, dw);
            if (!P.alpha_zero[ti]) {
                w1 *= radial<double>(P, ti, 0, r - rk, dex);
                w2 *= radial<double>(P, ti, 1, r - rk, dex);
            }
            z1 += fk * w1;
            z2 += fk * w2;
        }
        double db1, db2;
        const double b = bond_order<double>(P, ti, z1, z2, db1, db2);
        const double fR = P.A[pp] * exp(-P.lam1[pp] * r), fA = P.B[pp] * exp(-P.lam2[pp] * r);
        ecov += 0.5 * fc * (fR - b * fA);
        V4 out;
        out.x = (R)b;
        out.y = (R)(-0.5 * fc * fA * db1);
        out.z = (R)(-0.5 * fc * fA * db2);
        out.w = (R)(fc * b * fA);                // the charge-free attraction (f_q coupling)
        st4<R>(slot, (size_t)e * SLICE, out);
    }
    S.ecov[s] = ecov;
}

// Bond index, in the partner i's row, of the reverse of bond (m, e)
__device__ __forceinline__ int reverse_bond(const Seg &S, int m, int e, int i)
{
    return S.cmap[sliced(i, S.bsrev[sliced(m, e, S.Wb)], S.Ws)];
}

// pair-term derivative dV/dr of 1/2 fc (fR - b fA) at fixed b
template <typename R>
__device__ __forceinline__ R pair_dvdr(const Params<R> &P, int pp, R r, R b)
{
    R dfc;
    const R fc = cutoff(r, P.Rc[pp], P.Sc[pp], P.piSR[pp], dfc);
    const R fR = P.A[pp] * exp(-P.lam1[pp] * r), fA = P.B[pp] * exp(-P.lam2[pp] * r);
    return (R)0.5 * (dfc * (fR - b * fA) + fc * (-P.lam1[pp] * fR + b * P.lam2[pp] * fA));
}

template <typename R>
__global__ void __launch_bounds__(TILE) k_force_cov(const Tile *tiles, Seg *segs, Params<R> Pk, int gate)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    // serving: only segments whose charge solve finished and whose forces are pending
    if (gate && (!S.sst->done || S.sst->forces_done)) return;
    __shared__ V4 dtab[NCODE];
    __shared__ Params<R> Pl;
    // the first BOND_CACHE bonds of each thread's atom: vector, length, pair type
    __shared__ R cbx[BOND_CACHE][TILE], cby[BOND_CACHE][TILE], cbz[BOND_CACHE][TILE], cbr[BOND_CACHE][TILE];
    __shared__ uint8_t cbp[BOND_CACHE][TILE];
    // the tile's atoms in order of decreasing bond count (ties by row): the
    // loops below run over the atom's bonds and its neighbours' bonds, so the
    // 64 atoms of a wave then have similar trip counts (each lane's result
    // depends only on its atom, not on the order)
    __shared__ uint8_t nb_lds[TILE];
    __shared__ uint8_t order[TILE];
    {
        const int mo = T.row0 + threadIdx.x;
        const int own = mo < S.n ? S.bcnt[mo] : -1;
        nb_lds[threadIdx.x] = (uint8_t)(own + 1);
        __syncthreads();
        int rank = 0;
        for (int k = 0; k < TILE; k++) {
            const int c = (int)nb_lds[k] - 1;
            rank += (c > own || (c == own && k < (int)threadIdx.x)) ? 1 : 0;
        }
        order[rank] = (uint8_t)threadIdx.x;
    }
    stage_params(Pk, Pl);
    load_dtab2<R>(S, dtab);                 // (ends with a barrier)
    const Params<R> &P = Pl;
    const int m = T.row0 + order[threadIdx.x];
    if (m >= S.n) return;
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    const V4 *slot = reinterpret_cast<const V4 *>(S.slot);
    const int Wb = S.Wb, Ws = S.Ws;
    const auto bcnt = gbl(S.bcnt);
    const auto bsrev = gbl(S.bsrev);
    const auto cmap = gbl(S.cmap);
    const V4 lm = ld4<R>(xs, m);
    const int tm = (int)lm.w;
    const int nb = bcnt[m];
    const auto row = gbl(S.bidx + slice_base(m, Wb));
    const size_t slm = slice_base(m, Wb);
    double fx = 0, fy = 0, fz = 0;
    // bond e of m: vector, length, pair type (the first BOND_CACHE from LDS)
    auto bond_geom = [&](int e, R3<R> &d, R &r, int &pp) {
        const uint32_t ent = row[(size_t)e * SLICE];
        const V4 lj = ld4<R>(xs, ent & J_MASK);
        pp = tm * 2 + (int)lj.w;
        d = pair_vec<R>(lm, lj, dtab[ent >> CODE_SHIFT]);
        r = term_sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
    };
    auto bond = [&](int e, R3<R> &d, R &r, int &pp) {
        if (e < BOND_CACHE) {
            d.x = cbx[e][threadIdx.x];
            d.y = cby[e][threadIdx.x];
            d.z = cbz[e][threadIdx.x];
            r = cbr[e][threadIdx.x];
            pp = cbp[e][threadIdx.x];
        } else {
            bond_geom(e, d, r, pp);
        }
    };
    for (int e = 0; e < min(nb, BOND_CACHE); e++) {
        R3<R> d;
        R r;
        int pp;
        bond_geom(e, d, r, pp);
        cbx[e][threadIdx.x] = d.x;
        cby[e][threadIdx.x] = d.y;
        cbz[e][threadIdx.x] = d.z;
        cbr[e][threadIdx.x] = r;
        cbp[e][threadIdx.x] = (uint8_t)pp;
    }
    // m as the centre of its own bonds
    for (int e = 0; e < nb; e++) {
        R3<R> d;
        R r;
        int pp;
        bond(e, d, r, pp);
        const R ir = term_rcp(r);
        const V4 sv = ld4<R>(slot, slm + (size_t)e * SLICE);
        const R dv = pair_dvdr(P, pp, r, sv.x) * ir;
        R ax = dv * d.x, ay = dv * d.y, az = dv * d.z;
        if (sv.y != (R)0 || sv.z != (R)0) {
            for (int e2 = 0; e2 < nb; e2++) {
                if (e2 == e) continue;
                R3<R> dk;
                R rk;
                int pk;
                bond(e2, dk, rk, pk);
                R3<R> gj[2], gk[2];
                trip_grad(P, tm, pk, d, r, dk, rk, gj, gk);
                ax += sv.y * (gj[0].x + gk[0].x) + sv.z * (gj[1].x + gk[1].x);
                ay += sv.y * (gj[0].y + gk[0].y) + sv.z * (gj[1].y + gk[1].y);
                az += sv.z * (gj[1].z + gk[1].z) + sv.y * (gj[0].z + gk[0].z);
            }
        }
        fx += (double)ax;
        fy += (double)ay;
        fz += (double)az;
    }
    // m as the partner j or the environment k of its neighbours' bonds
    for (int e = 0; e < nb; e++) {
        const uint32_t ent = row[(size_t)e * SLICE];
        const int i = (int)(ent & J_MASK);
        const V4 li = ld4<R>(xs, i);
        const int ti = (int)li.w, pp = ti * 2 + tm;
        const int ni = bcnt[i];
        // bond (i -> m) in row i
        const int rv = cmap[slice_base(i, Ws) + (size_t)bsrev[slm + (size_t)e * SLICE] * SLICE];
        if (rv >= ni) continue;                               // (a reverse always exists)
        const R3<R> dmi = pair_vec<R>(lm, li, dtab[ent >> CODE_SHIFT]);
        const R r = term_sqrt(dmi.x * dmi.x + dmi.y * dmi.y + dmi.z * dmi.z), ir = term_rcp(r);
        const R3<R> d = {-dmi.x, -dmi.y, -dmi.z};            // i -> m
        const size_t sli = slice_base(i, Wb);
        const V4 sv = ld4<R>(slot, sli + (size_t)rv * SLICE);
        const R dv = pair_dvdr(P, pp, r, sv.x) * ir;
        R ax = -dv * d.x, ay = -dv * d.y, az = -dv * d.z;
        const auto rowi = gbl(S.bidx + sli);
        for (int t = 0; t < ni; t++) {
            if (t == rv) continue;
            const uint32_t ent2 = rowi[(size_t)t * SLICE];
            const V4 lk = ld4<R>(xs, ent2 & J_MASK);
            const int pk = ti * 2 + (int)lk.w;
            const R3<R> dk = pair_vec<R>(li, lk, dtab[ent2 >> CODE_SHIFT]);   // i -> k
            const R rk = term_sqrt(dk.x * dk.x + dk.y * dk.y + dk.z * dk.z);
            R3<R> gj[2], gk[2];
            if (sv.y != (R)0 || sv.z != (R)0) {
                // bond (i -> m), environment k: m is the partner j
                trip_grad(P, ti, pk, d, r, dk, rk, gj, gk);
                ax -= sv.y * gj[0].x + sv.z * gj[1].x;
                ay -= sv.y * gj[0].y + sv.z * gj[1].y;
                az -= sv.y * gj[0].z + sv.z * gj[1].z;
            }
            const V4 sk = ld4<R>(slot, sli + (size_t)t * SLICE);   // bond (i -> k)
            if (sk.y != (R)0 || sk.z != (R)0) {
                // bond (i -> k), environment m: m is the environment atom
                trip_grad(P, ti, pp, dk, rk, d, r, gj, gk);
                ax -= sk.y * gk[0].x + sk.z * gk[1].x;
                ay -= sk.y * gk[0].y + sk.z * gk[1].y;
                az -= sk.y * gk[0].z + sk.z * gk[1].z;
            }
        }
        fx += (double)ax;
        fy += (double)ay;
        fz += (double)az;
    }
    S.Fcov[m] = fx;
    S.Fcov[S.npad + m] = fy;
    S.Fcov[2 * S.npad + m] = fz;
}

} // namespace ctbop
