// adjoint_host.h -- host side of ctbop_param_grad (included by ctbop.hip).
#pragma once
#include "dual.h"
#include "k_adjoint.h"

namespace {

// Parameters in dual numbers with parameter k seeded (derivative 1): the
// mixing rules and G carry the derivative to every derived constant.
void fill_params_dual(const double *theta, int k, const ctbop_opts &o, Params<Dual> &P)
{
    memset(&P, 0, sizeof P);
    Dual t[CTBOP_N_PARAMS];
    for (int i = 0; i < CTBOP_N_PARAMS; i++) t[i] = Dual(theta[i], i == k ? 1.0 : 0.0);
    const Dual *s[2] = {t, t + 26};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            const int pp = a * 2 + b;
            P.A[pp] = sqrt(s[a][0] * s[b][0]);
            P.B[pp] = sqrt(s[a][1] * s[b][1]) * (a != b ? t[52] : Dual(1.0));
            P.lam1[pp] = 0.5 * (s[a][2] + s[b][2]);
            P.lam2[pp] = 0.5 * (s[a][3] + s[b][3]);
            const Dual Rc = sqrt(s[a][4] * s[b][4]), Sc = sqrt(s[a][5] * s[b][5]);
            P.Rc[pp] = Rc;
            P.Sc[pp] = Sc;
            P.piSR[pp] = M_PI / (Sc - Rc);
            P.g3[pp] = pow(s[a][23] * s[b][23], -1.5);
            P.s_cut2[pp] = (float)((Sc.v + o.skin) * (Sc.v + o.skin));
        }
    const Dual p = t[55];
    for (int a = 0; a < 2; a++) {
        const Dual *c = s[a];
        const Dual sig = c[6];
        P.G[a] = pow(pow(c[7 + 5], -p) + pow(c[14 + 5], -p), -1.0 / (2.0 * sig * p));
        P.inv2sig[a] = 1.0 / (2.0 * sig);
        for (int l = 0; l < 2; l++) {
            const Dual *ch = c + 7 + 7 * l;
            P.gam[a][l] = ch[0];
            P.c2[a][l] = ch[1] * ch[1];
            P.d2[a][l] = ch[2] * ch[2];
            P.c2d2[a][l] = (ch[1] / ch[2]) * (ch[1] / ch[2]);
            P.h[a][l] = ch[3];
            P.nn[a][l] = ch[4];
            P.g[a][l] = ch[5];
            P.alpha[a][l] = ch[6];
        }
        // the alpha terms are evaluated whenever alpha is the seeded parameter
        P.alpha_zero[a] = (c[13].v == 0.0 && c[20].v == 0.0 && c[13].d == 0.0 && c[20].d == 0.0) ? 1 : 0;
        P.chi[a] = c[21].v;
        P.J[a] = c[22].v;
        P.E0[a] = c[24].v;
        P.mass[a] = c[25].v;
    }
    P.p = p;
    P.p_is_2 = (p.v == 2.0 && p.d == 0.0) ? 1 : 0;
    P.ke = t[53];
    P.rc = t[54];
    P.inv_rc = 1.0 / t[54];
    P.l_cut2 = (float)((theta[54] + o.skin) * (theta[54] + o.skin));
    P.close2 = 0.25f;
}

// parameter classes of the flat layout
bool is_covalent(int k)
{
    if (k == 52 || k == 55) return true;
    if (k >= 52) return false;
    return (k % 26) <= 20;
}
bool is_coulomb(int k) { return k == 53 || k == 54 || (k < 52 && k % 26 == 23); }
constexpr int N_COVALENT = 44, N_COULOMB = 4;

// The dual passes take a chunk of parameters per launch; the chunk is as
// large as fits this budget of dual bond coefficients (all 44 covalent
// parameters for a few thousand atoms, one at a time at a million).
constexpr size_t DUAL_SLOT_BUDGET = size_t(512) << 20;

struct AdjLayout {
    size_t off_v, off_a, off_lam, off_slot, off_scal, off_grad, off_seg, off_sst, off_pk, off_kidx, off_ppart, bytes;
    size_t slot_stride;   // doubles per chunk member
    int chunk;            // covalent parameters per launch
    int cap;              // parameter sets held (>= chunk, >= N_COULOMB)
};

AdjLayout adj_layout(const Layout &L)
{
    AdjLayout A;
    const size_t np = L.seg.npad;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t at = o;
        o = align_up(o + b, 256);
        return at;
    };
    A.slot_stride = 6 * np * (size_t)L.seg.Wb;
    A.chunk = (int)std::max<size_t>(1, std::min<size_t>(N_COVALENT, DUAL_SLOT_BUDGET / (8 * A.slot_stride)));
    A.cap = std::max(A.chunk, N_COULOMB);
    A.off_v = take(8 * 3 * np);
    A.off_a = take(8 * np);
    A.off_lam = take(8 * np);
    A.off_slot = take(8 * A.slot_stride * (size_t)A.chunk);
    A.off_pk = take(sizeof(Params<Dual>) * (size_t)A.cap);
    A.off_kidx = take(sizeof(int) * (size_t)A.cap);
    A.off_ppart = take(8 * (size_t)L.seg.ntile * (size_t)A.cap);
    A.off_scal = take(8 * 8);
    A.off_grad = take(8 * 64);
    A.off_seg = take(sizeof(Seg));
    A.off_sst = take(sizeof(SegState));
    A.bytes = o;
    return A;
}

template <typename R>
int launch_param_grad(ctbop_ctx *ctx, Prep &P, const Params<R> &prm, char *adj, size_t adj_bytes, double dLdE,
                      const double *dLdF, const double *dLdq, double *grad_host, int *cg_iters)
{
    const AdjLayout AL = adj_layout(P.L);
    if (adj_bytes < AL.bytes) return fail(CTBOP_E_NOMEM, "adjoint workspace smaller than ctbop_param_grad_bytes()");
    AdjWs A;
    A.v = (double *)(adj + AL.off_v);
    A.a = (double *)(adj + AL.off_a);
    A.lam = (double *)(adj + AL.off_lam);
    A.slotd = (double *)(adj + AL.off_slot);
    A.slot_stride = AL.slot_stride;
    A.pk = (const Params<Dual> *)(adj + AL.off_pk);
    A.kidx = (const int *)(adj + AL.off_kidx);
    A.ppart = (double *)(adj + AL.off_ppart);
    A.ptile = P.L.ntile;
    A.scal = (double *)(adj + AL.off_scal);
    A.grad = (double *)(adj + AL.off_grad);
    A.w = dLdE;
    Seg *dadj = (Seg *)(adj + AL.off_seg);
    const dim3 g(P.L.ntile), b(TILE), g1(1);
    hipStream_t st = P.st;
    const int *sid = P.dsegid;
    hipLaunchKernelGGL(k_zero, g1, dim3(64), 0, st, A.grad, 64);
    hipLaunchKernelGGL(k_adj_seed, g, b, 0, st, P.dtiles, P.dseg, A, dLdF, dLdq);
    hipLaunchKernelGGL((k_adj_source<R, LPR>), g, b, 0, st, P.dtiles, P.dseg, ctx->pd, A);
    // adjoint view: the solver's charge array is lambda, total charge 0, and
    // its own solver state (the forward state and charges stay untouched)
    SegState *asst = (SegState *)(adj + AL.off_sst);
    static_assert(sizeof(SegState) % sizeof(double) == 0, "SegState is cleared as doubles");
    hipLaunchKernelGGL(k_zero, g1, dim3(64), 0, st, (double *)asst, (int)(sizeof(SegState) / sizeof(double)));
    Seg Sa = P.L.seg;
    Sa.q = A.lam;
    Sa.Q = 0.0;
    Sa.sst = asst;
    hipLaunchKernelGGL(k_set_seg, g1, g1, 0, st, dadj, Sa);
    hipLaunchKernelGGL(k_adj_init, g, b, 0, st, P.dtiles, dadj, A);
    // the stop test is relative to the starting projected residual of the
    // source a (whose scale is the caller's): first read that residual
    CgCtl ctl{1e-300, ctx->opts.cg_maxit};
    hipLaunchKernelGGL(k_fin_w0, g1, b, 0, st, sid, dadj);
    hipLaunchKernelGGL(k_shift_stats, g, b, 0, st, P.dtiles, dadj);
    hipLaunchKernelGGL(k_fin_assemble, g1, b, 0, st, sid, dadj, ctl);
    HIPCHK(hipGetLastError());
    double res0 = 0.0;
    HIPCHK(hipMemcpyAsync(&res0, &asst->res0, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctl.tol = std::max(ctx->opts.cg_tol * res0, 1e-300);
    // the single-reduction solve of the forward one (its first finalize
    // counts no iteration)
    hipLaunchKernelGGL((k_cg1_update<true>), g, b, 0, st, P.dtiles, dadj);
    int done_it = 0;
    for (;;) {
        for (int c = 0; c < ctx->opts.cg_check; c++) {
            hipLaunchKernelGGL((k_spmv<R, SPMV_U, SP_CG1>), g, b, 0, st, P.dtiles, dadj);
            hipLaunchKernelGGL(k_cg1_sum, dim3(FIN_SPLIT), b, 0, st, sid, dadj);
            hipLaunchKernelGGL(k_cg1_fin, g1, b, 0, st, sid, dadj, ctl);
            hipLaunchKernelGGL((k_cg1_update<false>), g, b, 0, st, P.dtiles, dadj);
        }
        done_it += ctx->opts.cg_check;
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ctx->host_flag, &asst->done, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (ctx->host_flag[0] || done_it >= ctx->opts.cg_maxit + 2) break;
    }
    if (cg_iters) *cg_iters = ctx->host_flag[1];
    hipLaunchKernelGGL(k_adj_keep_lam_shift, g1, dim3(64), 0, st, sid, dadj, A);
    // closed-form chi, J, E0 terms
    hipLaunchKernelGGL(k_self_terms, g, b, 0, st, P.dtiles, P.dseg, A);
    hipLaunchKernelGGL(k_fin_grad<6>, g1, b, 0, st, sid, P.dseg, A, 21, 22, 24, 26 + 21, 26 + 22, 26 + 24);
    // forward-mode passes over the explicit dependence, a chunk of parameters
    // per launch (blockIdx.y = member); every set is filled on the host first
    std::vector<int> cov, coul;
    for (int k = 0; k < CTBOP_N_PARAMS; k++) {
        if (is_covalent(k)) cov.push_back(k);
        else if (is_coulomb(k)) coul.push_back(k);
    }
    std::vector<Params<Dual>> hpk(cov.size() + coul.size());
    std::vector<int> hk(cov.size() + coul.size());
    for (size_t m = 0; m < cov.size(); m++) {
        fill_params_dual(ctx->theta, cov[m], ctx->opts, hpk[m]);
        hk[m] = cov[m];
    }
    for (size_t m = 0; m < coul.size(); m++) {
        fill_params_dual(ctx->theta, coul[m], ctx->opts, hpk[cov.size() + m]);
        hk[cov.size() + m] = coul[m];
    }
    Params<Dual> *dpk = (Params<Dual> *)(adj + AL.off_pk);
    int *dk = (int *)(adj + AL.off_kidx);
    for (size_t c0 = 0; c0 < cov.size(); c0 += AL.chunk) {
        const int m = (int)std::min<size_t>(AL.chunk, cov.size() - c0);
        HIPCHK(hipMemcpyAsync(dpk, &hpk[c0], sizeof(Params<Dual>) * m, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dk, &hk[c0], sizeof(int) * m, hipMemcpyHostToDevice, st));
        const dim3 gm(P.L.ntile, m);
        hipLaunchKernelGGL(k_bond_dual, gm, b, 0, st, P.dtiles, P.dseg, A);
        hipLaunchKernelGGL(k_fin_grad_members, dim3(m), b, 0, st, A, P.L.ntile);
        hipLaunchKernelGGL(k_force_cov_dual, gm, b, 0, st, P.dtiles, P.dseg, A);
        hipLaunchKernelGGL(k_fin_grad_members, dim3(m), b, 0, st, A, P.L.ntile);
    }
    {
        const int m = (int)coul.size();
        HIPCHK(hipMemcpyAsync(dpk, &hpk[cov.size()], sizeof(Params<Dual>) * m, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dk, &hk[cov.size()], sizeof(int) * m, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL((k_coul_dual<R, LPR>), dim3(P.L.ntile, m), b, 0, st, P.dtiles, P.dseg, A);
        hipLaunchKernelGGL(k_fin_grad_members, dim3(m), b, 0, st, A, P.L.ntile);
    }
    HIPCHK(hipGetLastError());
    int status = 0;
    HIPCHK(hipMemcpyAsync(grad_host, A.grad, sizeof(double) * CTBOP_N_PARAMS, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&status, &asst->status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (status) return fail(map_status(status), "adjoint charge solve: " + status_text(status));
    return CTBOP_OK;
}

} // namespace

extern "C" {

int ctbop_param_grad_bytes(ctbop_ctx *ctx, int n, const double *box, const int *pbc, size_t *bytes)
{
    if (!ctx || !bytes) return fail(CTBOP_E_INVAL, "null argument");
    Layout L;
    int rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    *bytes = adj_layout(L).bytes;
    return CTBOP_OK;
}

int ctbop_param_grad(ctbop_ctx *ctx, int n, const double *box, const int *pbc, void *sys, size_t sys_bytes,
                     void *adj_ws, size_t adj_bytes, double dL_dE, const double *dL_dF_dev, const double *dL_dq_dev,
                     double *grad_host, int *cg_iters, void *stream)
{
    if (!ctx || !sys || !adj_ws || !dL_dF_dev || !grad_host) return fail(CTBOP_E_INVAL, "null argument");
    if (ctx->opts.fq_kappa > 0.0) return fail(CTBOP_E_INVAL, "parameter adjoint: not available with fq_kappa > 0");
    auto it = ctx->seen.find(sys);
    auto ge = ctx->eval_gen.find(sys);
    if (it == ctx->seen.end() || it->second.n != n || ge == ctx->eval_gen.end() || ge->second != ctx->param_gen)
        return fail(CTBOP_E_INVAL, "param_grad needs a preceding evaluation on this system buffer with the current parameters");
    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    if (P.fresh) return fail(CTBOP_E_INVAL, "param_grad: the system buffer's geometry changed since the evaluation");
    if (!ctx->host_flag) HIPCHK(hipHostMalloc((void **)&ctx->host_flag, 64, hipHostMallocDefault));
    if (ctx->opts.fp64)
        return launch_param_grad<double>(ctx, P, ctx->pd, (char *)adj_ws, adj_bytes, dL_dE, dL_dF_dev, dL_dq_dev,
                                         grad_host, cg_iters);
    return launch_param_grad<float>(ctx, P, ctx->pf, (char *)adj_ws, adj_bytes, dL_dE, dL_dF_dev, dL_dq_dev,
                                    grad_host, cg_iters);
}

} // extern "C"
