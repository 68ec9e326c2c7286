// k_fq.h -- the charge-dependent coupling of the covalent part and the
// nonlinear charge minimisation it needs.
//
// The paper's potential gives its bonds a covalent-ionic mixed nature through
// a charge function f_q (Methods, first paragraph) whose form it leaves to its
// predecessor.  Stand-in: the attraction of bond (i,j) is scaled by
//     f_q = exp(-kappa (q_i - q_j)^2),
// so the covalent energy becomes E_cov(x) - 1/2 sum_(i,j) c_ij [f_q - 1] with
// c_ij = fc b_ij fA the charge-free attraction of the bond.  The energy is
// then no longer quadratic in q; the charges minimise it at fixed total
// charge (Methods: the energy is minimised over the charges by conjugate
// gradients at every step) by projected, block-Jacobi-preconditioned
// nonlinear CG:
//   r = -(chi + H q + g_c(q)) + shift,  g_c,m = -sum_j w_mj f_q'(q_m - q_j),
//   w_mj = (c_mj + c_jm)/2;  z = M (r - w 1);  p = z + beta p with the
//   Polak-Ribiere beta = z^T (r - r_old) / (z_old^T r_old), restarted at 0
//   when negative;  q += alpha p with alpha from two Newton steps on
//   phi'(alpha) = -p^T r + alpha p^T H p + [A(alpha) - A(0)],
//   phi''(alpha) = p^T H p + B(alpha),
//   A = -1/2 sum_bonds w delta f_q'(Delta + alpha delta),
//   B = -1/2 sum_bonds w delta^2 f_q''(Delta + alpha delta),
//   Delta = q_i - q_j, delta = p_i - p_j (sums over ordered bonds).
// The quadratic part of the residual is kept by recursion (rl -= alpha H p);
// the coupling's part is recomputed from the charges every iteration.  The
// matrix product, the block preconditioner, the projection and the stop test
// are the linear solve's.  After the solve every bond's coefficients (b and
// the two P_l) are scaled by its f_q, so the unchanged covalent force gather
// gives the forces at fixed charges, and each atom's bond energy gets its
// share of the coupling.
#pragma once
#include "ctbop_dev.h"
#include "k_tersoff.h"

namespace ctbop {

__device__ __forceinline__ double fq_d1(double k, double d) { return -2.0 * k * d * exp(-k * d * d); }
__device__ __forceinline__ double fq_d2(double k, double d) { return (4.0 * k * k * d * d - 2.0 * k) * exp(-k * d * d); }

// w per bond: the mean of the bond's attraction and its reverse's
template <typename R>
__global__ void __launch_bounds__(TILE) k_fq_weight(const Tile *tiles, Seg *segs)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int m = T.row0 + threadIdx.x;
    if (m >= S.n) return;
    const int Wb = S.Wb, Ws = S.Ws;
    const V4 *slot = reinterpret_cast<const V4 *>(S.slot);
    const auto bcnt = gbl(S.bcnt);
    const size_t bm = slice_base(m, Wb);
    const auto row = gbl(S.bidx + bm);
    const auto bsrev = gbl(S.bsrev + bm);
    const auto wq = gblw(S.wq + bm);
    const int nb = bcnt[m];
    for (int e = 0; e < nb; e++) {
        const int i = (int)(row[(size_t)e * SLICE] & J_MASK);
        const double c = (double)ld4<R>(slot, bm + (size_t)e * SLICE).w;
        const int rv = S.cmap[slice_base(i, Ws) + (size_t)bsrev[(size_t)e * SLICE] * SLICE];
        const double cr = rv < bcnt[i] ? (double)ld4<R>(slot, slice_base(i, Wb) + (size_t)rv * SLICE).w : c;
        wq[(size_t)e * SLICE] = 0.5 * (c + cr);
    }
}

// the coupling's share of the charge gradient of row m at charges q
__device__ __forceinline__ double fq_grad_row(const Seg &S, int m, double kq)
{
    const size_t bm = slice_base(m, S.Wb);
    const auto row = gbl(S.bidx + bm);
    const auto wq = gbl(S.wq + bm);
    const auto q = gbl(S.q);
    const double qm = q[m];
    const int nb = S.bcnt[m];
    double g = 0.0;
    for (int e = 0; e < nb; e++) {
        const int j = (int)(row[(size_t)e * SLICE] & J_MASK);
        g -= wq[(size_t)e * SLICE] * fq_d1(kq, qm - q[j]);
    }
    return g;
}

// start of the solve: rl = the quadratic residual from the assembly, r = rl - g_c(q0)
__global__ void __launch_bounds__(TILE) k_fq_r0(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n) {
        if (s < S.npad) S.rl[s] = 0.0;
        return;
    }
    const double rl = S.r[s];
    S.rl[s] = rl;
    S.r[s] = rl - fq_grad_row(S, s, S.fqk);
}

// line-search sums A(alpha), B(alpha) over the tile's bonds, written as
// partials k0, k0+1 (pass 0: alpha = 0)
__global__ void __launch_bounds__(TILE) k_fq_ls(const Tile *tiles, Seg *segs, int pass)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done) return;
    __shared__ double lds[4 * 2];
    const int s = T.row0 + threadIdx.x;
    const double a = pass ? S.sst->alpha : 0.0;
    const double kq = S.fqk;
    double A = 0.0, B = 0.0;
    if (s < S.n) {
        const size_t bm = slice_base(s, S.Wb);
        const auto row = gbl(S.bidx + bm);
        const auto wq = gbl(S.wq + bm);
        const auto q = gbl(S.q);
        const auto p = gbl(S.p);
        const double qs = q[s], ps = p[s];
        const int nb = S.bcnt[s];
        for (int e = 0; e < nb; e++) {
            const int j = (int)(row[(size_t)e * SLICE] & J_MASK);
            const double w = wq[(size_t)e * SLICE];
            const double d = ps - p[j];
            const double t = (qs - q[j]) + a * d;
            A -= 0.5 * w * d * fq_d1(kq, t);
            B -= 0.5 * w * d * d * fq_d2(kq, t);
        }
    }
    double v[2] = {A, B};
    tile_partials_at<2>(S, T.row0 / TILE, v, lds, pass ? 0 : 2);
}

// Newton steps on the step length.  Pass 0 also takes p^T H p and p^T r
// from the product's partials (0, 1); A(0), B(0) are partials 2, 3.
__global__ void k_fq_fin_ls(const int *seg_ids, Seg *segs, int pass)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (S.sst->done) return;
    __shared__ double lds[4 * 4];
    double tot[4];
    if (pass == 0) {
        seg_total<4>(S, lds, tot);
    } else {
        double t2[2];
        seg_total<2>(S, lds, t2);
        tot[0] = t2[0];
        tot[1] = t2[1];
    }
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        double d1, d2;
        if (pass == 0) {
            st->ps = tot[0];
            st->pr = tot[1];
            st->A0 = tot[2];
            st->alpha = 0.0;
            d1 = -tot[1];
            d2 = tot[0] + tot[3];
        } else {
            d1 = -st->pr + st->alpha * st->ps + (tot[0] - st->A0);
            d2 = st->ps + tot[1];
        }
        if (!(d2 > 0.0) || !(st->ps > 0.0)) {
            atomicOr(&st->status, ST_NOT_PD);
            st->done = 1;
            st->alpha = 0.0;
        } else {
            st->alpha -= d1 / d2;
        }
    }
}

// q += alpha p, rl -= alpha H p
__global__ void __launch_bounds__(TILE) k_fq_step(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done) return;
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n) return;
    const double a = S.sst->alpha;
    S.q[s] += a * S.p[s];
    S.rl[s] -= a * S.s[s];
}

// the full residual at the new charges, y = M r, and the tile's sums for w,
// rho, the stop test, the charge total and the Polak-Ribiere cross term
__global__ void __launch_bounds__(TILE) k_fq_resid(const Tile *tiles, Seg *segs)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    if (S.sst->done) return;
    __shared__ double lds[4 * 7];
    const int s = T.row0 + threadIdx.x;
    const bool live = s < S.n;
    double r = 0.0, ro = 0.0;
    if (live) {
        ro = S.r[s];
        r = S.rl[s] - fq_grad_row(S, s, S.fqk);
    }
    const double y = block_apply(S.binv, s, r);
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (live) {
        S.rold[s] = ro;
        S.r[s] = r;
        S.y[s] = y;
        const double m1 = S.m1[s];
        v[0] = r * m1;
        v[1] = r * y;
        v[2] = r;
        v[3] = r * r;
        v[4] = S.q[s];
        v[5] = y * ro;
        v[6] = m1 * ro;
    }
    tile_partials<7>(S, T.row0 / TILE, v, lds);
}

// w, rho, the Polak-Ribiere beta, the projected residual and the stop test
__global__ void k_fq_fin_update(const int *seg_ids, Seg *segs, CgCtl ctl)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    if (S.sst->done) return;
    __shared__ double lds[4 * 7];
    double tot[7];
    seg_total<7>(S, lds, tot);
    if (threadIdx.x == 0) {
        SegState *st = S.sst;
        const double w = tot[0] / st->sdinv;
        const double rho = tot[1] - w * tot[0];          // z^T r
        const double cross = tot[5] - w * tot[6];        // z^T r_old
        const double res2 = (tot[3] - tot[2] * tot[2] / S.n) / S.n;
        const double beta = (rho - cross) / st->rho;
        st->beta = beta > 0.0 ? beta : 0.0;
        st->rho = rho;
        st->w = w;
        st->mshift -= w;
        st->res = sqrt(fmax(res2, 0.0));
        st->iters += 1;
        st->iters_total += 1;
        st->qshift = (S.Q - tot[4]) / S.n;
        if (st->res < ctl.tol) st->done = 1;
        else if (st->iters >= ctl.maxit) { st->done = 1; atomicOr(&st->status, ST_NOCONV); }
    }
}

// after the solve: scale each bond's b, P_1, P_2 by its f_q (the force gather
// then gives the forces at fixed charges) and add the coupling's share
// 1/2 sum_j c_ij (1 - f_q) to the atom's bond energy
template <typename R>
__global__ void __launch_bounds__(TILE) k_fq_scale(const Tile *tiles, Seg *segs)
{
    using V4 = typename Vec4<R>::type;
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int s = T.row0 + threadIdx.x;
    if (s >= S.n) return;
    const size_t bm = slice_base(s, S.Wb);
    const auto row = gbl(S.bidx + bm);
    const auto q = gbl(S.q);
    V4 *slot = reinterpret_cast<V4 *>(S.slot);
    const double kq = S.fqk, qs = q[s];
    const int nb = S.bcnt[s];
    double corr = 0.0;
    for (int e = 0; e < nb; e++) {
        const int j = (int)(row[(size_t)e * SLICE] & J_MASK);
        const double d = qs - q[j];
        const double f = exp(-kq * d * d);
        V4 sv = ld4<R>(slot, bm + (size_t)e * SLICE);
        corr += 0.5 * (double)sv.w * (1.0 - f);
        sv.x = (R)((double)sv.x * f);
        sv.y = (R)((double)sv.y * f);
        sv.z = (R)((double)sv.z * f);
        st4<R>(slot, bm + (size_t)e * SLICE, sv);
    }
    S.ecov[s] += corr;
}

} // namespace ctbop
