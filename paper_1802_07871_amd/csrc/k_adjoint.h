// k_adjoint.h -- gradient of a loss L(E, F, q) with respect to the potential
// parameters, at the equilibrated charges of the last evaluation.
//
// With w = dL/dE, v = dL/dF, u = dL/dq (seeds given by the caller):
//   dL/dtheta = w dE/dtheta|_q + d(v.F)/dtheta|_q + a^T dq*/dtheta,
//   a = u + d(v.F)/dq.
// The charges satisfy H q* + chi = mu 1, sum q* = Q, so
//   a^T dq*/dtheta = -lambda^T (dH/dtheta q* + dchi/dtheta),
// where lambda solves the adjoint of the charge equilibration,
//   P H P lambda = P a, sum lambda = 0,
// with the same projected preconditioned CG (reverse mode through the
// charge solve: one extra solve for all parameters).  The explicit parameter
// dependence of the covalent and Coulomb terms is taken in forward mode, one
// parameter per pass, by evaluating the same bond, force and pair kernels in
// dual numbers (value + derivative along that parameter).  Since
// v.F = -dE/d(eps) along x + eps v, d(v.F)/dtheta is the derivative of v.F
// computed with dual parameters.  chi, J and E0 enter only the self energy
// and the diagonal, and are summed in closed form.
#pragma once
#include "ctbop_dev.h"
#include "dual.h"
#include "k_qeq.h"
#include "k_tersoff.h"

namespace ctbop {

struct AdjWs {
    double *v;        // dL/dF in the sorted frame, SoA [3 npad]
    double *a;        // adjoint charge source [npad]
    double *lam;      // adjoint charges [npad]
    double *scal;     // [0] q* re-projection, [1] lambda re-projection
    double *grad;     // dL/dtheta accumulators [64]
    double w;         // dL/dE
    // dual passes, a chunk of parameters per launch (blockIdx.y = member)
    const Params<Dual> *pk;   // the chunk's parameter sets, each seeded in its own parameter
    const int *kidx;          // the chunk's flat parameter indices
    double *slotd;            // dual bond coefficients (b, P1, P2 as value/derivative),
                              // [member][npad * Wb * 6]
    size_t slot_stride;       // doubles per member
    double *ppart;            // per-member tile partial sums [member][ptile]
    int ptile;
};

// The chunk member's parameter set, staged in LDS (buf) by the whole block
__device__ __forceinline__ const Params<Dual> &load_member_params(const AdjWs &A, unsigned char *buf)
{
    static_assert(sizeof(Params<Dual>) % 4 == 0, "copied as 32-bit words");
    const int *src = reinterpret_cast<const int *>(A.pk + blockIdx.y);
    int *dst = reinterpret_cast<int *>(buf);
    for (int i = threadIdx.x; i < (int)(sizeof(Params<Dual>) / 4); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return *reinterpret_cast<const Params<Dual> *>(buf);
}

// Block sum of one value per thread into the member's partial for this tile
__device__ __forceinline__ void member_partial(const AdjWs &A, int tile_local, double v, double *lds)
{
    double in[1] = {v}, out[1];
    block_sum<1>(in, lds, out);
    if (threadIdx.x == 0) A.ppart[(size_t)blockIdx.y * A.ptile + tile_local] = out[0];
}

// seeds into the sorted frame; keep the forward charges' re-projection
__global__ void __launch_bounds__(TILE) k_adj_seed(const Tile *tiles, Seg *segs, AdjWs A, const double *dLdF,
                                                   const double *dLdq)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    if (T.row0 == 0 && threadIdx.x == 0) A.scal[0] = S.sst->qshift;
    if (s < S.n) {
        const int i = S.perm[s];
        A.v[s] = dLdF[i];
        A.v[S.npad + s] = dLdF[S.n + i];
        A.v[2 * S.npad + s] = dLdF[2 * S.n + i];
        A.a[s] = dLdq ? dLdq[i] : 0.0;
    } else if (s < S.npad) {
        A.v[s] = A.v[S.npad + s] = A.v[2 * S.npad + s] = 0.0;
        A.a[s] = 0.0;
    }
}

// a_s = u_s + sum_j q_j C'(r_sj) (v_s - v_j) . r_hat_sj   (self images: v_s - v_s = 0)
template <typename R, int LPR>
__global__ void __launch_bounds__(TILE) k_adj_source(const Tile *tiles, Seg *segs, Params<double> PD, AdjWs A)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ V4 dtab[NCODE];
    load_dtab2<R>(S, dtab);
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    const double qsh = A.scal[0];
    constexpr int G = TILE / LPR;
    const int lane = threadIdx.x % LPR;
    for (int k = threadIdx.x / LPR; k < TILE; k += G) {
        const int s = T.row0 + k;
        if (s >= S.n) continue;
        const V4 li = xs[s];
        const int ti = (int)li.w;
        const double vx = A.v[s], vy = A.v[S.npad + s], vz = A.v[2 * S.npad + s];
        const int cnt = S.hcnt[s];
        const uint32_t *row = S.hidx + (size_t)s * S.Wl;
        double acc = 0.0;
        for (int e = lane; e < cnt; e += LPR) {
            const uint32_t ent = row[e];
            const int j = (int)(ent & J_MASK);
            if (j == s) continue;
            const V4 lj = xs[j];
            R3<R> d;
            const double r = entry_r<R>(li, lj, dtab[ent >> CODE_SHIFT], d);
            if (r >= PD.rc) continue;
            double dCr;
            coul64(PD, ti * 2 + (int)lj.w, r, dCr);
            const double dv = (vx - A.v[j]) * (double)d.x + (vy - A.v[S.npad + j]) * (double)d.y +
                              (vz - A.v[2 * S.npad + j]) * (double)d.z;
            acc += (S.q[j] + qsh) * dCr * dv;
        }
        acc = group_sum<LPR>(acc);
        if (lane == 0) A.a[s] += acc;
    }
}

// Start of the adjoint solve on the adjoint view (whose charge array is
// lambda): lambda = 0, r = a, p = 0; partial sums as the assembly writes them.
__global__ void __launch_bounds__(TILE) k_adj_init(const Tile *tiles, Seg *segs, AdjWs A)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[4 * 6];
    const int s = T.row0 + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (s < S.n) {
        const double r = A.a[s];
        S.q[s] = 0.0;          // the adjoint view's q is lambda
        S.r[s] = r;
        S.p[s] = 0.0;
        v[0] = r * S.m1[s];
        v[4] = S.m1[s];
    } else if (s < S.npad) {
        S.q[s] = 0.0;
    }
    tile_partials<6>(S, T.row0 / TILE, v, lds);
}

__global__ void k_adj_keep_lam_shift(const int *seg_ids, Seg *segs, AdjWs A)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (threadIdx.x == 0) A.scal[1] = S.sst->qshift;
}

// ---------------------------------------------------------------------------
// dual passes (a chunk of parameters per launch, one per blockIdx.y)
// ---------------------------------------------------------------------------

// Covalent bond pass in dual numbers: per-bond b, P1, P2 and the tile's
// w dEcov/dtheta, for the chunk member blockIdx.y.
__global__ void __launch_bounds__(TILE) k_bond_dual(const Tile *tiles, Seg *segs, AdjWs A)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double4 dtab[NCODE];
    __shared__ double lds[4];
    __shared__ __align__(16) unsigned char pbuf[sizeof(Params<Dual>)];
    const Params<Dual> &P = load_member_params(A, pbuf);
    load_dtab2<double>(S, dtab);
    const int s = T.row0 + threadIdx.x;
    double ew = 0.0;
    if (s < S.n) {
        const double4 *xs = S.xs64;
        const SRow<const uint32_t> row = srow<const uint32_t>(S.bidx, s, S.Wb);
        double *slot = A.slotd + blockIdx.y * A.slot_stride + (size_t)s * S.Wb * 6;
        const double4 li = xs[s];
        const int ti = (int)li.w;
        const int ns = S.bcnt[s];
        Dual ecov(0.0);
        for (int e = 0; e < ns; e++) {
            const uint32_t ent = row[e];
            const double4 lj = xs[ent & J_MASK];
            const int pp = ti * 2 + (int)lj.w;
            const R3<double> d = pair_vec<double>(li, lj, dtab[ent >> CODE_SHIFT]);
            const double r2 = d.x * d.x + d.y * d.y + d.z * d.z;
            Dual b(0.0), P1(0.0), P2(0.0);
            if (r2 < P.Sc[pp].v * P.Sc[pp].v) {
                const double r = ::sqrt(r2);
                Dual z1(0.0), z2(0.0);
                for (int e2 = 0; e2 < ns; e2++) {
                    if (e2 == e) continue;
                    const uint32_t ent2 = row[e2];
                    const double4 lk = xs[ent2 & J_MASK];
                    const int pk = ti * 2 + (int)lk.w;
                    const R3<double> dk = pair_vec<double>(li, lk, dtab[ent2 >> CODE_SHIFT]);
                    const double rk2 = dk.x * dk.x + dk.y * dk.y + dk.z * dk.z;
                    if (rk2 >= P.Sc[pk].v * P.Sc[pk].v) continue;
                    const double rk = ::sqrt(rk2);
                    const Dual cs((d.x * dk.x + d.y * dk.y + d.z * dk.z) / (r * rk));
                    Dual dummy, dw, dex;
                    const Dual fk = cutoff<Dual>(Dual(rk), P.Rc[pk], P.Sc[pk], P.piSR[pk], dummy);
                    Dual w1 = angular<Dual>(P, ti, 0, cs, dw), w2 = angular<Dual>(P, ti, 1, cs, dw);
                    if (!P.alpha_zero[ti]) {
                        w1 *= radial<Dual>(P, ti, 0, Dual(r - rk), dex);
                        w2 *= radial<Dual>(P, ti, 1, Dual(r - rk), dex);
                    }
                    z1 += fk * w1;
                    z2 += fk * w2;
                }
                Dual db1, db2, dfc;
                b = bond_order<Dual>(P, ti, z1, z2, db1, db2);
                const Dual fc = cutoff<Dual>(Dual(r), P.Rc[pp], P.Sc[pp], P.piSR[pp], dfc);
                const Dual fR = P.A[pp] * exp(-P.lam1[pp] * r), fA = P.B[pp] * exp(-P.lam2[pp] * r);
                ecov += 0.5 * fc * (fR - b * fA);
                P1 = -0.5 * fc * fA * db1;
                P2 = -0.5 * fc * fA * db2;
            }
            slot[6 * e + 0] = b.v;
            slot[6 * e + 1] = b.d;
            slot[6 * e + 2] = P1.v;
            slot[6 * e + 3] = P1.d;
            slot[6 * e + 4] = P2.v;
            slot[6 * e + 5] = P2.d;
        }
        ew = A.w * ecov.d;
    }
    member_partial(A, T.row0 / TILE, ew, lds);
}

__device__ __forceinline__ Dual slotd_get(const double *p) { return Dual(p[0], p[1]); }

// Covalent force gather in dual numbers; the tile's sum of v_m . dF_m/dtheta.
__global__ void __launch_bounds__(TILE) k_force_cov_dual(const Tile *tiles, Seg *segs, AdjWs A)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double4 dtab[NCODE];
    __shared__ double lds[4];
    __shared__ __align__(16) unsigned char pbuf[sizeof(Params<Dual>)];
    const Params<Dual> &P = load_member_params(A, pbuf);
    load_dtab2<double>(S, dtab);
    const double *slotd = A.slotd + blockIdx.y * A.slot_stride;
    const int m = T.row0 + threadIdx.x;
    double vf = 0.0;
    if (m < S.n) {
        const double4 *xs = S.xs64;
        const double4 lm = xs[m];
        const int tm = (int)lm.w;
        const int ns = S.bcnt[m];
        const SRow<const uint32_t> row = srow<const uint32_t>(S.bidx, m, S.Wb);
        Dual fx(0.0), fy(0.0), fz(0.0);
        for (int e = 0; e < ns; e++) {
            const uint32_t ent = row[e];
            const double4 lj = xs[ent & J_MASK];
            const int pp = tm * 2 + (int)lj.w;
            const R3<double> d = pair_vec<double>(lm, lj, dtab[ent >> CODE_SHIFT]);
            const double r2 = d.x * d.x + d.y * d.y + d.z * d.z;
            if (r2 >= P.Sc[pp].v * P.Sc[pp].v) continue;
            const double r = ::sqrt(r2), ir = 1.0 / r;
            const double *sv = slotd + ((size_t)m * S.Wb + e) * 6;
            const Dual b = slotd_get(sv), P1 = slotd_get(sv + 2), P2 = slotd_get(sv + 4);
            const Dual dv = pair_dvdr<Dual>(P, pp, Dual(r), b) * ir;
            Dual ax = dv * d.x, ay = dv * d.y, az = dv * d.z;
            for (int e2 = 0; e2 < ns; e2++) {
                if (e2 == e) continue;
                const uint32_t ent2 = row[e2];
                const double4 lk = xs[ent2 & J_MASK];
                const int pk = tm * 2 + (int)lk.w;
                const R3<double> dk = pair_vec<double>(lm, lk, dtab[ent2 >> CODE_SHIFT]);
                const double rk2 = dk.x * dk.x + dk.y * dk.y + dk.z * dk.z;
                if (rk2 >= P.Sc[pk].v * P.Sc[pk].v) continue;
                R3<Dual> gj[2], gk[2];
                const R3<Dual> dd = {Dual(d.x), Dual(d.y), Dual(d.z)}, ddk = {Dual(dk.x), Dual(dk.y), Dual(dk.z)};
                trip_grad<Dual>(P, tm, pk, dd, Dual(r), ddk, Dual(::sqrt(rk2)), gj, gk);
                ax += P1 * (gj[0].x + gk[0].x) + P2 * (gj[1].x + gk[1].x);
                ay += P1 * (gj[0].y + gk[0].y) + P2 * (gj[1].y + gk[1].y);
                az += P1 * (gj[0].z + gk[0].z) + P2 * (gj[1].z + gk[1].z);
            }
            fx += ax;
            fy += ay;
            fz += az;
        }
        for (int e = 0; e < ns; e++) {
            const uint32_t ent = row[e];
            const int i = (int)(ent & J_MASK);
            const double4 li = xs[i];
            const int ti = (int)li.w, pp = ti * 2 + tm;
            const R3<double> dmi = pair_vec<double>(lm, li, dtab[ent >> CODE_SHIFT]);
            const double r2 = dmi.x * dmi.x + dmi.y * dmi.y + dmi.z * dmi.z;
            if (r2 >= P.Sc[pp].v * P.Sc[pp].v) continue;
            const double r = ::sqrt(r2), ir = 1.0 / r;
            const R3<double> d = {-dmi.x, -dmi.y, -dmi.z};
            const int srev = reverse_bond(S, m, e, i);
            if (srev >= S.bcnt[i]) continue;                 // (a reverse always exists)
            const double *sv = slotd + ((size_t)i * S.Wb + srev) * 6;
            const Dual b = slotd_get(sv), P1 = slotd_get(sv + 2), P2 = slotd_get(sv + 4);
            const Dual dv = pair_dvdr<Dual>(P, pp, Dual(r), b) * ir;
            Dual ax = -dv * d.x, ay = -dv * d.y, az = -dv * d.z;
            const int ni = S.bcnt[i];
            const SRow<const uint32_t> rowi = srow<const uint32_t>(S.bidx, i, S.Wb);
            const R3<Dual> dd = {Dual(d.x), Dual(d.y), Dual(d.z)};
            for (int t = 0; t < ni; t++) {
                if (t == srev) continue;
                const uint32_t ent2 = rowi[t];
                const double4 lk = xs[ent2 & J_MASK];
                const int pk = ti * 2 + (int)lk.w;
                const R3<double> dk = pair_vec<double>(li, lk, dtab[ent2 >> CODE_SHIFT]);
                const double rk2 = dk.x * dk.x + dk.y * dk.y + dk.z * dk.z;
                if (rk2 >= P.Sc[pk].v * P.Sc[pk].v) continue;
                const double rk = ::sqrt(rk2);
                const R3<Dual> ddk = {Dual(dk.x), Dual(dk.y), Dual(dk.z)};
                R3<Dual> gj[2], gk[2];
                trip_grad<Dual>(P, ti, pk, dd, Dual(r), ddk, Dual(rk), gj, gk);
                ax -= P1 * gj[0].x + P2 * gj[1].x;
                ay -= P1 * gj[0].y + P2 * gj[1].y;
                az -= P1 * gj[0].z + P2 * gj[1].z;
                const double *sk = slotd + ((size_t)i * S.Wb + t) * 6;
                const Dual K1 = slotd_get(sk + 2), K2 = slotd_get(sk + 4);
                trip_grad<Dual>(P, ti, pp, ddk, Dual(rk), dd, Dual(r), gj, gk);
                ax -= K1 * gk[0].x + K2 * gk[1].x;
                ay -= K1 * gk[0].y + K2 * gk[1].y;
                az -= K1 * gk[0].z + K2 * gk[1].z;
            }
            fx += ax;
            fy += ay;
            fz += az;
        }
        vf = A.v[m] * fx.d + A.v[S.npad + m] * fy.d + A.v[2 * S.npad + m] * fz.d;
    }
    member_partial(A, T.row0 / TILE, vf, lds);
}

// Coulomb kernel in dual numbers (parameters gamma, ke, rc may carry the
// derivative)
__device__ __forceinline__ Dual coul_dual(const Params<Dual> &P, int pp, double r, Dual &dC)
{
    const Dual x = r * P.inv_rc, x2 = x * x, x3 = x2 * x;
    const Dual om = 1.0 - x, om2 = om * om;
    const Dual T = om2 * om2 * (1.0 + 4.0 * x + 10.0 * x2 + 20.0 * x3);
    const Dual dT = -140.0 * x3 * om2 * om;
    const Dual u = r * r * r + P.g3[pp];
    const Dual y = pow(u, -1.0 / 3.0);
    const Dual y2 = y * y;
    dC = P.ke * (dT * P.inv_rc * y - T * (r * r) * y2 * y2);
    return P.ke * T * y;
}

// Per row: w/2 q_s q_j dC/dtheta + q_s q_j d(C')/dtheta (v_s . r_hat) - lambda_s q_j dC/dtheta
template <typename R, int LPR>
__global__ void __launch_bounds__(TILE) k_coul_dual(const Tile *tiles, Seg *segs, AdjWs A)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ V4 dtab[NCODE];
    __shared__ double lds[4];
    __shared__ __align__(16) unsigned char pbuf[sizeof(Params<Dual>)];
    const Params<Dual> &P = load_member_params(A, pbuf);
    load_dtab2<R>(S, dtab);
    const V4 *xs = reinterpret_cast<const V4 *>(S.xs);
    const double qsh = A.scal[0], lsh = A.scal[1];
    constexpr int G = TILE / LPR;
    const int lane = threadIdx.x % LPR;
    double tot = 0.0;
    for (int k = threadIdx.x / LPR; k < TILE; k += G) {
        const int s = T.row0 + k;
        if (s >= S.n) continue;
        const V4 li = xs[s];
        const int ti = (int)li.w;
        const double qs = S.q[s] + qsh, ls = A.lam[s] + lsh;
        const double vx = A.v[s], vy = A.v[S.npad + s], vz = A.v[2 * S.npad + s];
        const int cnt = S.hcnt[s];
        const uint32_t *row = S.hidx + (size_t)s * S.Wl;
        double acc = 0.0;
        for (int e = lane; e < cnt; e += LPR) {
            const uint32_t ent = row[e];
            const int j = (int)(ent & J_MASK);
            const V4 lj = xs[j];
            R3<R> d;
            const double r = entry_r<R>(li, lj, dtab[ent >> CODE_SHIFT], d);
            if (r >= P.rc.v) continue;
            Dual dC;
            const Dual c = coul_dual(P, ti * 2 + (int)lj.w, r, dC);
            const double qj = S.q[j] + qsh;
            acc += (0.5 * A.w * qs - ls) * qj * c.d;
            if (j != s) acc += qs * qj * dC.d * (vx * (double)d.x + vy * (double)d.y + vz * (double)d.z) / r;
        }
        acc = group_sum<LPR>(acc);
        if (lane == 0) tot += acc;
    }
    member_partial(A, T.row0 / TILE, tot, lds);
}

// Closed-form self-energy and diagonal terms, per species t:
//   chi_t: w q_i - lambda_i;  J_t: w q_i^2 / 2 - lambda_i q_i;  E0_t: w
__global__ void __launch_bounds__(TILE) k_self_terms(const Tile *tiles, Seg *segs, AdjWs A)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[4 * 6];
    const int s = T.row0 + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (s < S.n) {
        const int t = (int)S.xs64[s].w;
        const double q = S.q[s] + A.scal[0], l = A.lam[s] + A.scal[1];
        v[3 * t + 0] = A.w * q - l;
        v[3 * t + 1] = 0.5 * A.w * q * q - l * q;
        v[3 * t + 2] = A.w;
    }
    tile_partials<6>(S, T.row0 / TILE, v, lds);
}

// Add the segment total of partial slots [0, K) to grad[idx[k]] (idx < 0: skip).
template <int K>
__global__ void k_fin_grad(const int *seg_ids, Seg *segs, AdjWs A, int i0, int i1, int i2, int i3, int i4, int i5)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[4 * K];
    double tot[K];
    seg_total<K>(S, lds, tot);
    if (threadIdx.x == 0) {
        const int idx[6] = {i0, i1, i2, i3, i4, i5};
#pragma unroll
        for (int k = 0; k < K; k++)
            if (idx[k] >= 0) A.grad[idx[k]] += tot[k];
    }
}

// Add each chunk member's total (its ptile partials, summed in a fixed order)
// to grad[kidx[member]]; one block per member.
__global__ void k_fin_grad_members(AdjWs A, int ntile)
{
    __shared__ double lds[4];
    double v[1] = {0.0}, tot[1];
    const double *pp = A.ppart + (size_t)blockIdx.x * A.ptile;
    for (int t = threadIdx.x; t < ntile; t += blockDim.x) v[0] += pp[t];
    block_sum<1>(v, lds, tot);
    if (threadIdx.x == 0) A.grad[A.kidx[blockIdx.x]] += tot[0];
}

__global__ void k_zero(double *p, int n)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0;
}

} // namespace ctbop
