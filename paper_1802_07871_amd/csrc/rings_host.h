// rings_host.h -- ring statistics entry points (included by ctbop.hip).
#pragma once
#include "k_rings.h"

namespace {

// workspace: counters, histogram, then the per-row C adjacency
struct RingLayout {
    size_t off_cnt, off_hist, off_adj, off_deg, off_mark, bytes;
};

RingLayout ring_layout(int npad, int nbins)
{
    RingLayout R;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align_up(o + b, 256);
        return at;
    };
    R.off_cnt = take(sizeof(unsigned long long) * RC_N);
    R.off_hist = take(sizeof(unsigned long long) * (size_t)nbins);
    R.off_adj = take(sizeof(uint32_t) * RING_DEG * (size_t)npad);
    R.off_deg = take(sizeof(int) * (size_t)npad);
    R.off_mark = take(sizeof(uint32_t) * RING_DEG * (size_t)npad);
    R.bytes = o;
    return R;
}

// smallest distance between opposite faces of the cell along each periodic direction
double min_periodic_width(const double *box, const int *pbc)
{
    const double *a[3] = {box, box + 3, box + 6};
    auto cross = [](const double *u, const double *v, double *w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double c[3];
    cross(a[1], a[2], c);
    const double vol = fabs(a[0][0] * c[0] + a[0][1] * c[1] + a[0][2] * c[2]);
    double wmin = INFINITY;
    for (int d = 0; d < 3; d++) {
        if (!pbc[d]) continue;
        cross(a[(d + 1) % 3], a[(d + 2) % 3], c);
        wmin = std::min(wmin, vol / sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
    }
    return wmin;
}

} // namespace

extern "C" {

int ctbop_rings_bytes(ctbop_ctx *ctx, int n, const double *box, const int *pbc, int nbins, size_t *bytes)
{
    if (!ctx || !box || !pbc || !bytes) return fail(CTBOP_E_INVAL, "null argument");
    if (nbins < 1 || nbins > 4096) return fail(CTBOP_E_INVAL, "nbins must be 1..4096");
    Layout L;
    int rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    *bytes = ring_layout(L.seg.npad, nbins).bytes;
    return CTBOP_OK;
}

int ctbop_rings(ctbop_ctx *ctx, int n, const double *x, const int32_t *types, const double *box, const int *pbc,
                void *sys, size_t sys_bytes, double r_bond, int max_size, const double *normal, const double *ref,
                double max_tilt_deg, int nbins, void *ws, size_t ws_bytes, int64_t *counts, int64_t *bonds,
                int64_t *hist, int32_t *ring_list, double *ring_orient, int64_t ring_cap, int64_t *n_rings,
                void *stream)
{
    if (!ctx || !x || !types || !box || !pbc || !ws || !counts || !bonds || !normal || !ref)
        return fail(CTBOP_E_INVAL, "null argument");
    if (max_size < 3 || max_size > RING_MAX) return fail(CTBOP_E_INVAL, "max_size must be 3..8");
    if (nbins < 1 || nbins > 4096) return fail(CTBOP_E_INVAL, "nbins must be 1..4096");
    if (ring_cap < 0 || (ring_cap > 0 && !ring_list)) return fail(CTBOP_E_INVAL, "ring list capacity without a list");
    const double S_cc = ctx->theta[26 + 5];
    if (!(r_bond > 0.0) || r_bond > S_cc)
        return fail(CTBOP_E_INVAL, "r_bond must lie in (0, S_CC] (the covalent list holds bonds up to S_CC)");
    if (min_periodic_width(box, pbc) < max_size * r_bond)
        return fail(CTBOP_E_INVAL, "periodic width below max_size * r_bond: rings could wind around the cell");
    // reference frame of the orientation
    RingCfg c;
    memset(&c, 0, sizeof c);
    const double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
    if (!(nn > 0.0)) return fail(CTBOP_E_INVAL, "zero plane normal");
    for (int d = 0; d < 3; d++) c.n[d] = normal[d] / nn;
    const double un = ref[0] * c.n[0] + ref[1] * c.n[1] + ref[2] * c.n[2];
    for (int d = 0; d < 3; d++) c.u[d] = ref[d] - un * c.n[d];
    const double uu = sqrt(c.u[0] * c.u[0] + c.u[1] * c.u[1] + c.u[2] * c.u[2]);
    if (!(uu > 1e-9 * sqrt(ref[0] * ref[0] + ref[1] * ref[1] + ref[2] * ref[2])))
        return fail(CTBOP_E_INVAL, "reference direction parallel to the normal");
    for (int d = 0; d < 3; d++) c.u[d] /= uu;
    c.w[0] = c.n[1] * c.u[2] - c.n[2] * c.u[1];
    c.w[1] = c.n[2] * c.u[0] - c.n[0] * c.u[2];
    c.w[2] = c.n[0] * c.u[1] - c.n[1] * c.u[0];
    c.rb2 = r_bond * r_bond;
    c.max_size = max_size;
    c.nbins = nbins;
    c.cos_tilt_min = max_tilt_deg >= 90.0 ? -2.0 : cos(max_tilt_deg * M_PI / 180.0);

    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    const RingLayout RL = ring_layout(P.L.seg.npad, nbins);
    if (ws_bytes < RL.bytes) return fail(CTBOP_E_NOMEM, "workspace smaller than ctbop_rings_bytes()");
    Seg S = P.L.seg;
    S.x = const_cast<double *>(x);
    S.type = types;
    S.F = nullptr;
    S.q_out = nullptr;
    S.E_out = nullptr;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    lists_any(ctx, P, 0);
    char *w = (char *)ws;
    RingWs W;
    W.adj = (uint32_t *)(w + RL.off_adj);
    W.deg = (int *)(w + RL.off_deg);
    W.mark = (uint32_t *)(w + RL.off_mark);
    W.cnt = (unsigned long long *)(w + RL.off_cnt);
    W.hist = (unsigned long long *)(w + RL.off_hist);
    W.list = ring_cap > 0 ? ring_list : nullptr;
    W.orient = ring_cap > 0 ? ring_orient : nullptr;
    W.cap = ring_cap;
    HIPCHK(hipMemsetAsync(w, 0, RL.off_adj, P.st));
    const dim3 g(P.L.ntile), b(TILE);
    {
        Timed t(ctx, 9, P.st);
        hipLaunchKernelGGL(k_ring_adj, g, b, 0, P.st, P.dtiles, P.dseg, W, c);
    }
    {
        Timed t(ctx, 10, P.st);
        hipLaunchKernelGGL(k_rings, g, b, 0, P.st, P.dtiles, P.dseg, W, c);
    }
    {
        Timed t(ctx, 11, P.st);
        hipLaunchKernelGGL(k_ring_chain, g, b, 0, P.st, P.dtiles, P.dseg, W);
    }
    HIPCHK(hipGetLastError());
    std::vector<unsigned long long> cnt(RC_N), h(nbins);
    HIPCHK(hipMemcpyAsync(cnt.data(), W.cnt, sizeof(unsigned long long) * RC_N, hipMemcpyDeviceToHost, P.st));
    HIPCHK(hipMemcpyAsync(h.data(), W.hist, sizeof(unsigned long long) * nbins, hipMemcpyDeviceToHost, P.st));
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, &P.L.seg.sst->status, sizeof(int), hipMemcpyDeviceToHost, P.st));
    HIPCHK(hipStreamSynchronize(P.st));
    if (st) return fail(map_status(st), status_text(st));
    if (cnt[RC_OVERFLOW])
        return fail(CTBOP_E_NEIGH_OVERFLOW, std::to_string(cnt[RC_OVERFLOW]) + " C atoms with more than 12 C neighbours");
    for (int k = 0; k <= RING_MAX; k++) counts[k] = (int64_t)cnt[k];
    bonds[0] = (int64_t)cnt[RC_BONDS];
    bonds[1] = (int64_t)cnt[RC_CHAIN];
    if (hist)
        for (int k = 0; k < nbins; k++) hist[k] = (int64_t)h[k];
    if (n_rings) *n_rings = (int64_t)cnt[RC_LISTED];
    return CTBOP_OK;
}

} // extern "C"
