// ctbop.hip -- host side of the C ABI (include/ctbop.h): contexts, layout of
// the caller-owned per-system buffer, and the launch sequence of one
// energy/force/charge evaluation and of the MD loop.  All device work is in
// the kernels included below; this file only validates, lays out memory and
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ctbop.h"
#include "ctbop_dev.h"
#include "k_lists.h"
#include "k_tersoff.h"
#include "k_qeq.h"
#include "k_md.h"
#include "k_fq.h"

using namespace ctbop;

namespace {

constexpr int LPR = 16;             // lanes per Coulomb row (assembly, force gather)
constexpr int BUILD_L = 4;          // lanes per atom in the list build (tuned: 2, 4, 8, 16 lanes)
constexpr int SPMV_U = 8;           // list entries in flight per row in the charge-solve product (tuned)

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) return fail(CTBOP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Sig {
    int n;
    double box[9];
    int pbc[3];
    int fp64;
    size_t bytes;
    bool operator==(const Sig &o) const
    {
        return n == o.n && fp64 == o.fp64 && bytes == o.bytes && !memcmp(box, o.box, sizeof box) &&
               !memcmp(pbc, o.pbc, sizeof pbc);
    }
};

struct Layout {
    Seg seg;               // with device addresses filled in
    size_t off_seg, off_sst, off_tiles, off_segid, off_ke;
    size_t bytes;
    int ntile;
};

} // namespace

struct ctbop_ctx {
    double theta[CTBOP_N_PARAMS];
    ctbop_opts opts;
    Params<float> pf;
    Params<double> pd;
    std::unordered_map<void *, Sig> seen;
    std::unordered_map<void *, int> last_iters;
    // parameter set generation, and the generation each system buffer was
    // last evaluated with (the adjoint needs the evaluation it differentiates)
    unsigned long param_gen = 0;
    std::unordered_map<void *, unsigned long> eval_gen;
    std::atomic<int> servers{0};  // live servers on this context
    int *host_flag = nullptr;    // pinned: done, iters
    // second stream (default priority) for the covalent terms, which overlap
    // the Coulomb chain of an evaluation; events fork it off the caller's
    // stream after the lists and join it back before the Coulomb forces
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // tiles per launch of the side stream's kernels: two blocks per CU, so
    // that they leave room for the solve's product beside them
    int side_chunk = 512;
    // optional per-kernel timing with HIP events on the caller's stream
    int profile = 0;
    unsigned profile_mask = 0xffffu;   // kernel classes timed while profiling is on
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_ms[16] = {0};
    long prof_n[16] = {0};
};

namespace {

template <typename R>
void fill_params(const double *t, const ctbop_opts &o, Params<R> &P)
{
    memset(&P, 0, sizeof P);
    const double *s[2] = {t, t + 26};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            int pp = a * 2 + b;
            P.A[pp] = (R)std::sqrt(s[a][0] * s[b][0]);
            P.B[pp] = (R)(std::sqrt(s[a][1] * s[b][1]) * (a != b ? t[52] : 1.0));
            P.lam1[pp] = (R)(0.5 * (s[a][2] + s[b][2]));
            P.lam2[pp] = (R)(0.5 * (s[a][3] + s[b][3]));
            double Rc = std::sqrt(s[a][4] * s[b][4]), Sc = std::sqrt(s[a][5] * s[b][5]);
            P.Rc[pp] = (R)Rc;
            P.Sc[pp] = (R)Sc;
            P.piSR[pp] = (R)(M_PI / (Sc - Rc));
            P.g3[pp] = (R)std::pow(s[a][23] * s[b][23], -1.5);
            P.s_cut2[pp] = (float)((Sc + o.skin) * (Sc + o.skin));
        }
    const double p = t[55];
    for (int a = 0; a < 2; a++) {
        const double *c = s[a];
        double sig = c[6];
        double g1 = c[7 + 5], g2 = c[14 + 5];
        P.G[a] = (R)std::pow(std::pow(g1, -p) + std::pow(g2, -p), -1.0 / (2.0 * sig * p));
        P.inv2sig[a] = (R)(1.0 / (2.0 * sig));
        for (int l = 0; l < 2; l++) {
            const double *ch = c + 7 + 7 * l;
            P.gam[a][l] = (R)ch[0];
            P.c2[a][l] = (R)(ch[1] * ch[1]);
            P.d2[a][l] = (R)(ch[2] * ch[2]);
            P.c2d2[a][l] = (R)((ch[1] / ch[2]) * (ch[1] / ch[2]));
            P.h[a][l] = (R)ch[3];
            P.nn[a][l] = (R)ch[4];
            P.g[a][l] = (R)ch[5];
            P.alpha[a][l] = (R)ch[6];
        }
        P.alpha_zero[a] = (c[7 + 6] == 0.0 && c[14 + 6] == 0.0) ? 1 : 0;
        P.chi[a] = c[21];
        P.J[a] = c[22];
        P.E0[a] = c[24];
        P.mass[a] = c[25];
    }
    P.p = (R)p;
    P.p_is_2 = (p == 2.0) ? 1 : 0;
    P.ke = (R)t[53];
    P.rc = (R)t[54];
    P.inv_rc = (R)(1.0 / t[54]);
    P.l_cut2 = (float)((t[54] + o.skin) * (t[54] + o.skin));
    P.close2 = 0.25f;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Geometry of the cell grid and the byte layout of the per-system buffer.
// The list build's cell culling (Seg::cwi, Seg::cull2): the inverse of the
// cell-grid matrix, and rl^2 over the smallest eigenvalue of its metric
// (cyclic Jacobi rotations on the 3x3 symmetric matrix), widened by 1e-4
// relative plus 1e-3 cell^2 for the FP32 arithmetic of the test.
void cell_cull(Seg &S, double rl)
{
    const double(*c)[3] = S.cw;
    const double det = c[0][0] * (c[1][1] * c[2][2] - c[1][2] * c[2][1]) -
                       c[0][1] * (c[1][0] * c[2][2] - c[1][2] * c[2][0]) +
                       c[0][2] * (c[1][0] * c[2][1] - c[1][1] * c[2][0]);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            // (c^-1)[a][b] = cofactor(b, a) / det
            const int r0 = (b + 1) % 3, r1 = (b + 2) % 3, q0 = (a + 1) % 3, q1 = (a + 2) % 3;
            S.cwi[a][b] = (float)((c[r0][q0] * c[r1][q1] - c[r0][q1] * c[r1][q0]) / det);
        }
    double g[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) g[a][b] = c[a][0] * c[b][0] + c[a][1] * c[b][1] + c[a][2] * c[b][2];
    for (int sweep = 0; sweep < 50; sweep++) {
        const double off = g[0][1] * g[0][1] + g[0][2] * g[0][2] + g[1][2] * g[1][2];
        if (off <= 1e-30 * (g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2])) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                if (g[p][q] == 0.0) continue;
                const double th = 0.5 * std::atan2(2.0 * g[p][q], g[q][q] - g[p][p]);
                const double cs = std::cos(th), sn = std::sin(th);
                for (int k = 0; k < 3; k++) {          // columns p, q
                    const double gp = g[k][p], gq = g[k][q];
                    g[k][p] = cs * gp - sn * gq;
                    g[k][q] = sn * gp + cs * gq;
                }
                for (int k = 0; k < 3; k++) {          // rows p, q
                    const double gp = g[p][k], gq = g[q][k];
                    g[p][k] = cs * gp - sn * gq;
                    g[q][k] = sn * gp + cs * gq;
                }
            }
    }
    const double lam = std::min(g[0][0], std::min(g[1][1], g[2][2]));
    S.cull2 = (float)(rl * rl / lam * (1.0 + 1e-4) + 1e-3);
}

int make_layout(const ctbop_ctx *ctx, int n, const double *box, const int *pbc, char *base, Layout &L)
{
    if (n <= 0 || n > MAX_ATOMS) return fail(CTBOP_E_INVAL, "atom count out of range");
    Seg &S = L.seg;
    memset(&S, 0, sizeof S);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) S.h[a][b] = box[3 * a + b];
    const double(*h)[3] = S.h;
    double det = h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[2][1]) - h[0][1] * (h[1][0] * h[2][2] - h[1][2] * h[2][0]) +
                 h[0][2] * (h[1][0] * h[2][1] - h[1][1] * h[2][0]);
    if (!(det > 0.0)) return fail(CTBOP_E_INVAL, "box must be right-handed with positive volume");
    S.hi[0][0] = (h[1][1] * h[2][2] - h[1][2] * h[2][1]) / det;
    S.hi[0][1] = (h[0][2] * h[2][1] - h[0][1] * h[2][2]) / det;
    S.hi[0][2] = (h[0][1] * h[1][2] - h[0][2] * h[1][1]) / det;
    S.hi[1][0] = (h[1][2] * h[2][0] - h[1][0] * h[2][2]) / det;
    S.hi[1][1] = (h[0][0] * h[2][2] - h[0][2] * h[2][0]) / det;
    S.hi[1][2] = (h[0][2] * h[1][0] - h[0][0] * h[1][2]) / det;
    S.hi[2][0] = (h[1][0] * h[2][1] - h[1][1] * h[2][0]) / det;
    S.hi[2][1] = (h[0][1] * h[2][0] - h[0][0] * h[2][1]) / det;
    S.hi[2][2] = (h[0][0] * h[1][1] - h[0][1] * h[1][0]) / det;
    const double rl = ctx->theta[54] + ctx->opts.skin;
    double w[3];
    for (int a = 0; a < 3; a++) {
        const double *u = h[(a + 1) % 3], *v = h[(a + 2) % 3];
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        w[a] = det / std::sqrt(cx * cx + cy * cy + cz * cz);
        S.pbc[a] = pbc[a] ? 1 : 0;
        S.nb[a] = std::max(1, (int)std::floor(w[a] / (0.5 * rl)));
    }
    // keep the grid at most a few cells per atom (huge vacuum boxes)
    const long cap = std::max<long>(4096, 8L * n);
    while ((long)S.nb[0] * S.nb[1] * S.nb[2] > cap) {
        int a = (S.nb[0] >= S.nb[1] && S.nb[0] >= S.nb[2]) ? 0 : (S.nb[1] >= S.nb[2] ? 1 : 2);
        S.nb[a] = std::max(1, S.nb[a] / 2);
    }
    for (int a = 0; a < 3; a++) {
        int st = (int)std::ceil(rl * S.nb[a] / w[a] - 1e-12);
        if (S.pbc[a]) {
            if (st > 3) return fail(CTBOP_E_INVAL, "periodic cell narrower than (rc_coul + skin)/3");
        } else {
            st = std::min(st, S.nb[a] - 1);
        }
        S.st[a] = st;
        for (int b = 0; b < 3; b++) S.cw[a][b] = h[a][b] / S.nb[a];
    }
    cell_cull(S, rl);
    S.ncell = S.nb[0] * S.nb[1] * S.nb[2];
    S.n = n;
    S.npad = (n + TILE - 1) / TILE * TILE;
    S.ntile = S.npad / TILE;
    S.tile0 = 0;
    S.Wl = ctx->opts.long_cap;
    S.Ws = ctx->opts.short_cap;
    S.Wb = std::min(S.Ws, WB);
    S.skin = ctx->opts.skin;
    const int fp64 = ctx->opts.fp64;
    const size_t rsz = fp64 ? 8 : 4, v4 = fp64 ? 32 : 16;
    const size_t np = S.npad;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.off_seg = take(sizeof(Seg));
    L.off_sst = take(sizeof(SegState));
    L.off_tiles = take(sizeof(Tile) * S.ntile);
    L.off_segid = take(sizeof(int));
    L.off_ke = take(8 * sizeof(double));
    size_t o_perm = take(4 * np), o_permt = take(4 * np), o_cellof = take(4 * (size_t)n), o_csort = take(4 * np);
    size_t o_cs = take(4 * ((size_t)S.ncell + 1)), o_cc = take(4 * (size_t)S.ncell);
    size_t o_off = take(8 * 3 * np), o_ref = take(8 * 3 * (size_t)n), o_xs = take(v4 * np);
    size_t o_xs64 = fp64 ? o_xs : take(32 * np);
    size_t o_lcnt = take(4 * np), o_lidx = take(4 * np * S.Wl), o_H = take(rsz * np * S.Wl);
    size_t o_hcnt = take(4 * np), o_hidx = take(4 * np * S.Wl), o_Hr = take(rsz * np * S.Wl);
    size_t o_hsidx = take(4 * np * S.Wl), o_hs16 = take(2 * np * S.Wl), o_hwide = take(np), o_swide = take(np / SLICE);
    size_t o_hperm = take(np);
    const size_t nt = (size_t)S.ntile;
    size_t o_halo = take(4 * nt * HALO_MAX), o_nhalo = take(4 * nt), o_hbits = take(8 * nt * HALO_WORDS),
           o_hpre = take(2 * nt * HALO_WORDS);
    size_t o_scnt = take(4 * np), o_sidx = take(4 * np * S.Ws), o_srev = take(np * S.Ws);
    size_t o_bcnt = take(4 * np), o_bidx = take(4 * np * S.Wb), o_bsrev = take(np * S.Wb), o_cmap = take(np * S.Ws),
           o_slot = take(v4 * np * S.Wb);
    size_t o_ecov = take(8 * np), o_fcov = take(8 * 3 * np);
    size_t o_q = take(8 * np), o_r = take(8 * np), o_p = take(8 * np), o_s = take(8 * np), o_jd = take(8 * np);
    size_t o_binv = take(2 * np * BK), o_m1 = take(8 * np), o_y = take(8 * np), o_hz = take(8 * np);
    size_t o_qs = take(8 * (size_t)n), o_qring = take(8 * (size_t)NHIST * n);
    size_t o_part = take(8 * (NPART * (size_t)S.ntile + 16 * FIN_SPLIT));
    const bool fq = ctx->opts.fq_kappa > 0.0;
    size_t o_rl = 0, o_rold = 0, o_wq = 0;
    if (fq) {
        o_rl = take(8 * np);
        o_rold = take(8 * np);
        o_wq = take(8 * np * S.Wb);
    }
    S.fqk = ctx->opts.fq_kappa;
    L.bytes = o;
    L.ntile = S.ntile;
    if (base) {
        S.perm = (int *)(base + o_perm);
        S.perm_tmp = (int *)(base + o_permt);
        S.cell_of = (int *)(base + o_cellof);
        S.csort = (int *)(base + o_csort);
        S.cell_start = (int *)(base + o_cs);
        S.cell_cnt = (int *)(base + o_cc);
        S.off = (double *)(base + o_off);
        S.ref_x = (double *)(base + o_ref);
        S.xs = base + o_xs;
        S.xs64 = (double4 *)(base + o_xs64);
        S.lcnt = (int *)(base + o_lcnt);
        S.lidx = (uint32_t *)(base + o_lidx);
        S.H = base + o_H;
        S.hcnt = (int *)(base + o_hcnt);
        S.hidx = (uint32_t *)(base + o_hidx);
        S.Hr = base + o_Hr;
        S.hsidx = (uint32_t *)(base + o_hsidx);
        S.hs16 = (uint16_t *)(base + o_hs16);
        S.hwide = (uint8_t *)(base + o_hwide);
        S.swide = (uint8_t *)(base + o_swide);
        S.hperm = (uint8_t *)(base + o_hperm);
        S.halo = (uint32_t *)(base + o_halo);
        S.nhalo = (int *)(base + o_nhalo);
        S.hbits = (unsigned long long *)(base + o_hbits);
        S.hpre = (uint16_t *)(base + o_hpre);
        S.scnt = (int *)(base + o_scnt);
        S.sidx = (uint32_t *)(base + o_sidx);
        S.srev = (uint8_t *)(base + o_srev);
        S.bcnt = (int *)(base + o_bcnt);
        S.bidx = (uint32_t *)(base + o_bidx);
        S.bsrev = (uint8_t *)(base + o_bsrev);
        S.cmap = (uint8_t *)(base + o_cmap);
        S.slot = base + o_slot;
        S.ecov = (double *)(base + o_ecov);
        S.Fcov = (double *)(base + o_fcov);
        S.q = (double *)(base + o_q);
        S.r = (double *)(base + o_r);
        S.p = (double *)(base + o_p);
        S.s = (double *)(base + o_s);
        S.binv = (_Float16 *)(base + o_binv);
        S.m1 = (double *)(base + o_m1);
        S.y = (double *)(base + o_y);
        S.hz = (double *)(base + o_hz);
        S.jd = (double *)(base + o_jd);
        S.q_state = (double *)(base + o_qs);
        S.q_ring = (double *)(base + o_qring);
        S.part = (double *)(base + o_part);
        S.sst = (SegState *)(base + L.off_sst);
        if (fq) {
            S.rl = (double *)(base + o_rl);
            S.rold = (double *)(base + o_rold);
            S.wq = (double *)(base + o_wq);
        }
    }
    return CTBOP_OK;
}

__global__ void k_reset_state(SegState *st, Tile *tiles, int ntile, int *segid)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        memset(st, 0, sizeof(SegState));
        *segid = 0;
    }
    if (t < ntile) {
        tiles[t].seg = 0;
        tiles[t].row0 = t * TILE;
    }
}

hipEvent_t ev_get(ctbop_ctx *ctx)
{
    if (ctx->ev_free.empty()) {
        // timing only: no system-scope fence (cache writeback and invalidate)
        // when the event is recorded, which would slow the work it brackets;
        // the stream is synchronised before any time is read
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    return e;
}

// Launch wrapper: with profiling on, bracket the launch with events
// (kernel class k) on the same stream.
struct Timed {
    ctbop_ctx *ctx;
    int k;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(ctbop_ctx *c, int kk, hipStream_t s) : ctx(c), k(kk), st(s)
    {
        if (ctx->profile && ((ctx->profile_mask >> k) & 1u)) {
            a = ev_get(ctx);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~Timed()
    {
        if (a) {
            hipEvent_t b = ev_get(ctx);
            if (b) {
                (void)hipEventRecord(b, st);
                ctx->ev_pending.push_back({k, {a, b}});
            }
        }
    }
};

// after a stream synchronisation: fold completed event pairs into totals
// (pairs on another stream that have not completed yet stay pending)
void ev_harvest(ctbop_ctx *ctx)
{
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> keep;
    for (auto &p : ctx->ev_pending) {
        if (hipEventQuery(p.second.second) == hipErrorNotReady) {
            keep.push_back(p);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            ctx->prof_ms[p.first] += ms;
            ctx->prof_n[p.first] += 1;
        }
        ctx->ev_free.push_back(p.second.first);
        ctx->ev_free.push_back(p.second.second);
    }
    ctx->ev_pending.swap(keep);
}

// the side stream and its two events, created on first use
int side_stream(ctbop_ctx *ctx)
{
    if (ctx->side) return CTBOP_OK;
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu > 0) ctx->side_chunk = 2 * ncu;
    HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    return CTBOP_OK;
}

int map_status(int st)
{
    if (st & ST_TOO_CLOSE) return CTBOP_E_TOO_CLOSE;
    if (st & ST_OVERFLOW) return CTBOP_E_NEIGH_OVERFLOW;
    if (st & ST_REV) return CTBOP_E_NEIGH_OVERFLOW;
    if (st & ST_NOT_PD) return CTBOP_E_QEQ_NOT_PD;
    if (st & ST_NOCONV) return CTBOP_E_QEQ_NOCONV;
    return CTBOP_OK;
}

std::string status_text(int st)
{
    std::string s;
    if (st & ST_TOO_CLOSE) s += "atoms closer than 0.5 A; ";
    if (st & ST_OVERFLOW) s += "neighbour list overflow (raise long_cap/short_cap); ";
    if (st & ST_REV) s += "covalent list not symmetric; ";
    if (st & ST_NOT_PD) s += "charge matrix not positive definite; ";
    if (st & ST_NOCONV) s += "charge solve did not converge; ";
    return s;
}

struct Prep {
    Layout L;
    char *base;
    Seg *dseg;
    Tile *dtiles;
    int *dsegid;
    double *dke;
    hipStream_t st;
    bool fresh;
    // false for the allocation-free entry point: no side stream (the
    // covalent kernels then run on the caller's stream; results do not
    // depend on it), the solver flag read into flag_host, and no record of
    // the buffer in the context's maps
    bool own = true;
    int *flag_host = nullptr;
};

// validate, lay out, and (re)initialise the system buffer when it is new to
// this context or its geometry changed
int prepare(ctbop_ctx *ctx, int n, const double *box, const int *pbc, void *sys, size_t sys_bytes, void *stream,
            Prep &P)
{
    if (!ctx || !box || !pbc || !sys) return fail(CTBOP_E_INVAL, "null argument");
    P.base = (char *)sys;
    int rc = make_layout(ctx, n, box, pbc, P.base, P.L);
    if (rc) return rc;
    if (sys_bytes < P.L.bytes) return fail(CTBOP_E_NOMEM, "system buffer smaller than ctbop_system_bytes()");
    P.dseg = (Seg *)(P.base + P.L.off_seg);
    P.dtiles = (Tile *)(P.base + P.L.off_tiles);
    P.dsegid = (int *)(P.base + P.L.off_segid);
    P.dke = (double *)(P.base + P.L.off_ke);
    P.st = (hipStream_t)stream;
    Sig sig;
    memset(&sig, 0, sizeof sig);
    sig.n = n;
    memcpy(sig.box, box, sizeof sig.box);
    for (int a = 0; a < 3; a++) sig.pbc[a] = pbc[a] ? 1 : 0;
    sig.fp64 = ctx->opts.fp64;
    sig.bytes = P.L.bytes;
    auto it = ctx->seen.find(sys);
    P.fresh = (it == ctx->seen.end() || !(it->second == sig));
    if (!ctx->host_flag) HIPCHK(hipHostMalloc((void **)&ctx->host_flag, 64, hipHostMallocDefault));
    P.flag_host = ctx->host_flag;
    if (P.fresh) {
        hipLaunchKernelGGL(k_reset_state, dim3((P.L.ntile + 255) / 256), dim3(256), 0, P.st, P.L.seg.sst, P.dtiles,
                           P.L.ntile, P.dsegid);
        HIPCHK(hipGetLastError());
        ctx->seen[sys] = sig;
        ctx->last_iters[sys] = 0;
    }
    return CTBOP_OK;
}

// Sorted frame and neighbour lists for the current positions (the lists are
// rebuilt when an atom has moved more than half the skin, or on request).
template <typename R>
void launch_lists(ctbop_ctx *ctx, Prep &P, const Params<R> &prm, int flags)
{
    const int nt = P.L.ntile;
    const dim3 g(nt), b(TILE), g1(1);
    hipStream_t st = P.st;
    const int force = (flags & CTBOP_FLAG_FORCE_REBUILD) || P.fresh;
    int warm = 0;
    if ((flags & CTBOP_FLAG_WARM_START) && !P.fresh) warm = (flags & CTBOP_FLAG_EXTRAPOLATE) ? 2 : 1;
    const int *sid = P.dsegid;
    hipLaunchKernelGGL(k_call_init, g1, dim3(64), 0, st, sid, P.dseg, 1, force);
    hipLaunchKernelGGL(k_check_disp, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_bin_clear, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_bin, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_scan_part, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_scan_mid, g1, b, 0, st, sid, P.dseg);
    hipLaunchKernelGGL(k_scan_fin, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_scatter, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_cell_sort, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_gather<R>, g, b, 0, st, P.dtiles, P.dseg, warm);
    hipLaunchKernelGGL(k_fin_qshift, g1, b, 0, st, sid, P.dseg);
    hipLaunchKernelGGL(k_qfix, g, b, 0, st, P.dtiles, P.dseg);
    {
        Timed t(ctx, 7, st);
        hipLaunchKernelGGL((k_build<R, BUILD_L>), g, b, 0, st, P.dtiles, P.dseg, prm);
    }
    hipLaunchKernelGGL(k_rev, g, b, 0, st, P.dtiles, P.dseg);
    hipLaunchKernelGGL(k_mark_built, g1, dim3(64), 0, st, sid, P.dseg, 1);
}

// One evaluation: sorted frame and lists, bond pass, Coulomb rows, charge
// solve, forces and energy.
template <typename R>
int launch_eval(ctbop_ctx *ctx, Prep &P, const Params<R> &prm, int flags, int *iters_out)
{
    const int nt = P.L.ntile;
    const dim3 g(nt), b(TILE), g1(1);
    hipStream_t st = P.st;
    const int *sid = P.dsegid;
    launch_lists<R>(ctx, P, prm, flags);
    // covalent terms on the side stream: they need only the lists, and run
    // beside the charge solve and its host round trips, forked after the
    // sliced copy (beside the assembly and the copy they slowed both by more
    // than the solve loses).  With the charge coupling the covalent gather
    // needs the charges: the side stream then runs the bond pass and the
    // coupling weights only, forked before the assembly since the starting
    // residual needs those weights, and the gather follows the solve on the
    // caller's stream.
    const bool fq = ctx->opts.fq_kappa > 0.0;
    auto side_launch = [&]() -> int {
        hipStream_t cst = st;
        if (P.own) {
            int rc = side_stream(ctx);
            if (rc) return rc;
            HIPCHK(hipEventRecord(ctx->ev_fork, st));
            HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
            cst = ctx->side;
        }
        // beside the solve, in chunks of side_chunk tiles one after another,
        // so that at most two of their blocks per CU take room from the
        // product (all at once they slowed its launches 1.6x; chunks of 1, 1.5,
        // 2, 3 and 4 blocks per CU: the step 12.96, 11.61, 10.97, 11.05 and
        // 11.15 ms against 11.13); with the charge coupling, whose assembly
        // waits for them, and alone on the caller's stream, one launch
        const int chunk = P.own && !fq ? ctx->side_chunk : nt;
        {
            Timed t(ctx, 3, cst);
            for (int t0 = 0; t0 < nt; t0 += chunk)
                hipLaunchKernelGGL((k_bond<R>), dim3(std::min(chunk, nt - t0)), b, 0, cst, P.dtiles + t0, P.dseg,
                                   ctx->pd);
        }
        if (fq) {
            hipLaunchKernelGGL((k_fq_weight<R>), g, b, 0, cst, P.dtiles, P.dseg);
        } else {
            Timed t(ctx, 4, cst);
            for (int t0 = 0; t0 < nt; t0 += chunk)
                hipLaunchKernelGGL((k_force_cov<R>), dim3(std::min(chunk, nt - t0)), b, 0, cst, P.dtiles + t0,
                                   P.dseg, prm, 0);
        }
        if (P.own) HIPCHK(hipEventRecord(ctx->ev_join, ctx->side));
        return CTBOP_OK;
    };
    if (fq) {
        const int rc = side_launch();
        if (rc) return rc;
    }
    CgCtl ctl{ctx->opts.cg_tol, ctx->opts.cg_maxit};
    {
        Timed t(ctx, 2, st);
        hipLaunchKernelGGL((k_assemble<R, LPR>), g, b, 0, st, P.dtiles, P.dseg, ctx->pd);
    }
    if (fq) {
        // the starting residual needs the coupling weights of this step
        if (P.own) HIPCHK(hipStreamWaitEvent(st, ctx->ev_join, 0));
        hipLaunchKernelGGL(k_fq_r0, g, b, 0, st, P.dtiles, P.dseg);
    }
    {
        Timed t(ctx, 8, st);
        hipLaunchKernelGGL((k_hslice<R>), g, b, 0, st, P.dtiles, P.dseg);
    }
    if (!fq) {
        const int rc = side_launch();
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_fin_w0, g1, b, 0, st, sid, P.dseg);
    if (fq) {
        hipLaunchKernelGGL(k_shift_stats, g, b, 0, st, P.dtiles, P.dseg);
        hipLaunchKernelGGL(k_fin_assemble, g1, b, 0, st, sid, P.dseg, ctl);
    } else {
        // the single-reduction solve's start: the residual's shift, y = M r
        Timed t(ctx, 6, st);
        hipLaunchKernelGGL((k_cg1_update<true>), g, b, 0, st, P.dtiles, P.dseg);
    }
    HIPCHK(hipGetLastError());
    // charge solve: launch iterations in batches, then read the convergence flag
    int done_it = 0;
    int chunk = ctx->opts.cg_check;
    // (the single-reduction solve's first finalize counts no iteration: n
    // iterations take n + 1 rounds)
    if (P.own) chunk = std::max(chunk, std::min(ctx->last_iters[P.base], ctx->opts.cg_maxit) + (fq ? 0 : 1));
    int *flag = P.flag_host;
    for (;;) {
        for (int c = 0; c < chunk; c++) {
            if (!fq) {
                {
                    Timed t(ctx, 0, st);
                    hipLaunchKernelGGL((k_spmv<R, SPMV_U, SP_CG1>), g, b, 0, st, P.dtiles, P.dseg);
                }
                hipLaunchKernelGGL(k_cg1_sum, dim3(FIN_SPLIT), b, 0, st, sid, P.dseg);
                hipLaunchKernelGGL(k_cg1_fin, g1, b, 0, st, sid, P.dseg, ctl);
                Timed t(ctx, 5, st);
                hipLaunchKernelGGL((k_cg1_update<false>), g, b, 0, st, P.dtiles, P.dseg);
                continue;
            }
            {
                Timed t(ctx, 6, st);
                hipLaunchKernelGGL(k_cg_dir, g, b, 0, st, P.dtiles, P.dseg);
            }
            {
                Timed t(ctx, 0, st);
                hipLaunchKernelGGL((k_spmv<R, SPMV_U, SP_FQ>), g, b, 0, st, P.dtiles, P.dseg);
            }
            // two Newton steps on the step length
            for (int pass = 0; pass < 2; pass++) {
                hipLaunchKernelGGL(k_fq_ls, g, b, 0, st, P.dtiles, P.dseg, pass);
                hipLaunchKernelGGL(k_fq_fin_ls, g1, b, 0, st, sid, P.dseg, pass);
            }
            hipLaunchKernelGGL(k_fq_step, g, b, 0, st, P.dtiles, P.dseg);
            {
                Timed t(ctx, 5, st);
                hipLaunchKernelGGL(k_fq_resid, g, b, 0, st, P.dtiles, P.dseg);
            }
            hipLaunchKernelGGL(k_fq_fin_update, g1, b, 0, st, sid, P.dseg, ctl);
        }
        done_it += chunk;
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(flag, &P.L.seg.sst->done, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (ctx->profile) ev_harvest(ctx);
        // (the single-reduction solve's first finalize counts no iteration)
        if (flag[0] || done_it >= ctx->opts.cg_maxit + 2) break;
        chunk = ctx->opts.cg_check;
    }
    if (P.own) ctx->last_iters[P.base] = flag[1];
    if (iters_out) *iters_out = flag[1];
    if (P.own && !fq) HIPCHK(hipStreamWaitEvent(st, ctx->ev_join, 0));
    if (fq) {
        hipLaunchKernelGGL((k_fq_scale<R>), g, b, 0, st, P.dtiles, P.dseg);
        Timed t(ctx, 4, st);
        hipLaunchKernelGGL((k_force_cov<R>), g, b, 0, st, P.dtiles, P.dseg, prm, 0);
    }
    {
        Timed t(ctx, 1, st);
        hipLaunchKernelGGL((k_force_coul<R, LPR>), g, b, 0, st, P.dtiles, P.dseg, ctx->pd, 0);
    }
    hipLaunchKernelGGL(k_fin_energy, g1, b, 0, st, sid, P.dseg, 0);
    HIPCHK(hipGetLastError());
    return CTBOP_OK;
}

void lists_any(ctbop_ctx *ctx, Prep &P, int flags)
{
    if (ctx->opts.fp64) launch_lists<double>(ctx, P, ctx->pd, flags);
    else launch_lists<float>(ctx, P, ctx->pf, flags);
}

int eval_any(ctbop_ctx *ctx, Prep &P, int flags, int *iters)
{
    if (P.own) ctx->eval_gen[P.base] = ctx->param_gen;
    if (ctx->opts.fp64) return launch_eval<double>(ctx, P, ctx->pd, flags, iters);
    return launch_eval<float>(ctx, P, ctx->pf, flags, iters);
}

int check_params(const double *params, int n_params)
{
    if (!params) return fail(CTBOP_E_INVAL, "null argument");
    if (n_params != CTBOP_N_PARAMS) return fail(CTBOP_E_INVAL, "expected 56 parameters");
    for (int t = 0; t < 2; t++) {
        const double *s = params + 26 * t;
        if (!(s[6] > 0) || !(s[11] > 0) || !(s[18] > 0) || !(s[12] > 0) || !(s[19] > 0) || !(s[22] > 0) ||
            !(s[5] > s[4]) || !(s[23] > 0))
            return fail(CTBOP_E_INVAL, "parameters: need sigma, n_l, g_l, J, gamma_coul > 0 and S > R");
    }
    if (!(params[55] > 0) || !(params[54] > 0)) return fail(CTBOP_E_INVAL, "parameters: need p > 0, rc > 0");
    return CTBOP_OK;
}

int fill_info(ctbop_ctx *ctx, Prep &P, ctbop_info *info)
{
    SegState ss;
    HIPCHK(hipMemcpyAsync(&ss, P.L.seg.sst, sizeof ss, hipMemcpyDeviceToHost, P.st));
    HIPCHK(hipStreamSynchronize(P.st));
    if (ctx->profile) ev_harvest(ctx);
    info->energy = ss.energy;
    info->cg_residual = ss.res;
    info->mu = ss.mu_prev;
    info->cg_iters = ss.iters;
    info->rebuilt = ss.rebuild;
    info->status = map_status(ss.status);
    info->max_long = ss.maxl;
    info->max_short = ss.maxs;
    info->nnz_long = ss.nnz_long;
    info->nnz_short = ss.nnz_short;
    info->n_rebuild = ss.nrebuild;
    info->cg_iters_total = ss.iters_total;
    info->cg_res0 = ss.res0;
    info->nnz_coul = (unsigned long long)ss.nnz_coul;
    info->nnz_coul_wide = (unsigned long long)ss.nnz_wide;
    info->nnz_coul_slots = (unsigned long long)ss.nnz_slots;
    info->nnz_coul_halo = (unsigned long long)ss.nnz_halo;
    info->n_bonds = (unsigned long long)ss.nbond;
    info->n_triplets = (unsigned long long)ss.ntrip;
    if (ss.status) return fail(info->status, status_text(ss.status));
    return CTBOP_OK;
}

} // namespace

extern "C" {

void ctbop_default_opts(ctbop_opts *o)
{
    o->cg_tol = 1e-9;
    o->cg_maxit = 500;
    o->skin = 0.6;
    o->long_cap = 512;
    o->short_cap = 64;
    o->fp64 = 0;
    o->cg_check = 4;
    o->fq_kappa = 0.0;
}

int ctbop_create(const double *params, int n_params, const ctbop_opts *opts, ctbop_ctx **out)
{
    if (!out) return fail(CTBOP_E_INVAL, "null argument");
    int prc = check_params(params, n_params);
    if (prc) return prc;
    ctbop_ctx *c = new ctbop_ctx();
    memcpy(c->theta, params, sizeof c->theta);
    ctbop_default_opts(&c->opts);
    if (opts) {
        c->opts = *opts;
        ctbop_opts d;
        ctbop_default_opts(&d);
        if (c->opts.cg_tol <= 0) c->opts.cg_tol = d.cg_tol;
        if (c->opts.cg_maxit <= 0) c->opts.cg_maxit = d.cg_maxit;
        if (c->opts.skin < 0) c->opts.skin = d.skin;
        if (c->opts.long_cap <= 0) c->opts.long_cap = d.long_cap;
        if (c->opts.short_cap <= 0) c->opts.short_cap = d.short_cap;
        if (c->opts.cg_check <= 0) c->opts.cg_check = d.cg_check;
    }
    if (c->opts.short_cap > 255) {
        delete c;
        return fail(CTBOP_E_INVAL, "short_cap must be <= 255");
    }
    if (!(c->opts.fq_kappa >= 0.0)) {
        delete c;
        return fail(CTBOP_E_INVAL, "fq_kappa must be >= 0");
    }
    fill_params<float>(c->theta, c->opts, c->pf);
    fill_params<double>(c->theta, c->opts, c->pd);
    *out = c;
    return CTBOP_OK;
}

int ctbop_set_params(ctbop_ctx *ctx, const double *params, int n_params)
{
    if (!ctx) return fail(CTBOP_E_INVAL, "null argument");
    int rc = check_params(params, n_params);
    if (rc) return rc;
    if (ctx->servers.load() > 0) return fail(CTBOP_E_BUSY, "a server is running on this context");
    memcpy(ctx->theta, params, sizeof ctx->theta);
    fill_params<float>(ctx->theta, ctx->opts, ctx->pf);
    fill_params<double>(ctx->theta, ctx->opts, ctx->pd);
    ctx->param_gen++;
    // list radii may have changed: every system buffer starts over
    ctx->seen.clear();
    ctx->last_iters.clear();
    ctx->eval_gen.clear();
    return CTBOP_OK;
}

int ctbop_destroy(ctbop_ctx *ctx)
{
    if (!ctx) return CTBOP_OK;
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
        (void)hipEventDestroy(ctx->ev_fork);
        (void)hipEventDestroy(ctx->ev_join);
    }
    if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
    for (auto &p : ctx->ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    delete ctx;
    return CTBOP_OK;
}

int ctbop_system_bytes(ctbop_ctx *ctx, int n, const double *box, const int *pbc, size_t *bytes)
{
    if (!ctx || !box || !pbc || !bytes) return fail(CTBOP_E_INVAL, "null argument");
    Layout L;
    int rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    *bytes = L.bytes;
    return CTBOP_OK;
}

int ctbop_system_reset(ctbop_ctx *ctx, void *sys)
{
    if (!ctx || !sys) return fail(CTBOP_E_INVAL, "null argument");
    ctx->seen.erase(sys);
    ctx->last_iters.erase(sys);
    ctx->eval_gen.erase(sys);
    return CTBOP_OK;
}

int ctbop_compute_energy_forces_charges(ctbop_ctx *ctx, int n, const double *pos, const int32_t *types,
                                        const double *box, const int *pbc, double Q, int flags, void *sys,
                                        size_t sys_bytes, double *E, double *F, double *q, ctbop_info *info,
                                        void *stream)
{
    if (!pos || !types || !F || !q) return fail(CTBOP_E_INVAL, "null array argument");
    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    Seg S = P.L.seg;
    S.x = pos;
    S.type = types;
    S.F = F;
    S.q_out = q;
    S.E_out = E;
    S.Q = Q;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    int iters = 0;
    rc = eval_any(ctx, P, flags, &iters);
    if (rc) return rc;
    if (info) return fill_info(ctx, P, info);
    return CTBOP_OK;
}

int ctbop_md_run(ctbop_ctx *ctx, int n, double *x, double *v, const int32_t *types, const uint8_t *fixed,
                 const double *box, const int *pbc, double Q, double dt, int nsteps, int every, void *sys,
                 size_t sys_bytes, double *F, double *q, double *thermo, ctbop_info *info, void *stream)
{
    if (!x || !v || !types || !F || !q || nsteps < 0) return fail(CTBOP_E_INVAL, "bad argument");
    if (every <= 0) every = 1;
    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    Seg S = P.L.seg;
    S.x = x;
    S.type = types;
    S.F = F;
    S.q_out = q;
    S.E_out = nullptr;
    S.Q = Q;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    MdIO io;
    io.x = x;
    io.v = v;
    io.F = F;
    io.fixed = fixed;
    io.dt = dt;
    io.mass[0] = ctx->theta[25];
    io.mass[1] = ctx->theta[26 + 25];
    const dim3 g(P.L.ntile), b(TILE);
    int iters = 0, status_acc = 0;
    // forces at the start
    const int mdflags = CTBOP_FLAG_WARM_START | CTBOP_FLAG_EXTRAPOLATE;
    rc = eval_any(ctx, P, mdflags, &iters);
    if (rc) return rc;
    hipLaunchKernelGGL(k_md_kick, g, b, 0, P.st, P.dtiles, P.dseg, MdIO{x, v, F, fixed, 0.0, {io.mass[0], io.mass[1]}});
    hipLaunchKernelGGL(k_fin_ke, dim3(1), b, 0, P.st, P.dsegid, P.dseg, P.dke);
    for (int s = 0; s <= nsteps; s++) {
        if (s > 0) {
            hipLaunchKernelGGL(k_md_kick_drift, g, b, 0, P.st, P.dtiles, P.dseg, io);
            rc = eval_any(ctx, P, mdflags, &iters);
            if (rc) return rc;
            hipLaunchKernelGGL(k_md_kick, g, b, 0, P.st, P.dtiles, P.dseg, io);
            hipLaunchKernelGGL(k_fin_ke, dim3(1), b, 0, P.st, P.dsegid, P.dseg, P.dke);
            HIPCHK(hipGetLastError());
        }
        if (thermo && s % every == 0) {
            double kv[2];
            HIPCHK(hipMemcpyAsync(kv, P.dke, sizeof kv, hipMemcpyDeviceToHost, P.st));
            HIPCHK(hipStreamSynchronize(P.st));
            thermo[2 * (s / every)] = kv[1];
            thermo[2 * (s / every) + 1] = kv[0];
        }
        if (s % 64 == 0 || s == nsteps) {
            int code = 0;
            HIPCHK(hipMemcpyAsync(&code, &P.L.seg.sst->status, sizeof(int), hipMemcpyDeviceToHost, P.st));
            HIPCHK(hipStreamSynchronize(P.st));
            status_acc |= code;
            if (code) return fail(map_status(code), status_text(code));
        }
    }
    (void)status_acc;
    if (info) return fill_info(ctx, P, info);
    HIPCHK(hipStreamSynchronize(P.st));
    return CTBOP_OK;
}

int ctbop_md_run_nvt(ctbop_ctx *ctx, int n, double *x, double *v, const int32_t *types, const uint8_t *fixed,
                     const double *box, const int *pbc, double Q, double dt, int nsteps, int every, double T_K,
                     double tau_fs, int chain_len, double *chain, void *sys, size_t sys_bytes, double *F, double *q,
                     double *thermo, ctbop_info *info, void *stream)
{
    if (!x || !v || !types || !F || !q || !chain || nsteps < 0) return fail(CTBOP_E_INVAL, "bad argument");
    if (chain_len < 1 || chain_len > NHC_MAX) return fail(CTBOP_E_INVAL, "chain length must be 1..8");
    if (!(T_K > 0) || !(tau_fs > 0) || !(dt > 0)) return fail(CTBOP_E_INVAL, "need T, tau, dt > 0");
    if (every <= 0) every = 1;
    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    Seg S = P.L.seg;
    S.x = x;
    S.type = types;
    S.F = F;
    S.q_out = q;
    S.E_out = nullptr;
    S.Q = Q;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    const dim3 g(P.L.ntile), b(TILE), g1(1);
    // degrees of freedom of the mobile atoms (momentum conserved only if none is fixed)
    hipLaunchKernelGGL(k_count_fixed, g, b, 0, P.st, P.dtiles, P.dseg, fixed);
    hipLaunchKernelGGL(k_fin_ke, g1, b, 0, P.st, P.dsegid, P.dseg, P.dke + 6);
    double nfix = 0.0;
    HIPCHK(hipMemcpyAsync(&nfix, P.dke + 6, sizeof(double), hipMemcpyDeviceToHost, P.st));
    HIPCHK(hipStreamSynchronize(P.st));
    const int nmob = n - (int)llround(nfix);
    if (nmob < 2) return fail(CTBOP_E_INVAL, "NVT needs at least two mobile atoms");
    NhcCfg c;
    memset(&c, 0, sizeof c);
    c.M = chain_len;
    c.dt = dt;
    c.kT = 8.617333262e-5 * T_K;
    c.Nf = 3.0 * nmob - (nmob == n ? 3.0 : 0.0);
    for (int k = 0; k < chain_len; k++) c.Qm[k] = (k == 0 ? c.Nf : 1.0) * c.kT * tau_fs * tau_fs;
    MdIO io;
    io.x = x;
    io.v = v;
    io.F = F;
    io.fixed = fixed;
    io.dt = dt;
    io.mass[0] = ctx->theta[25];
    io.mass[1] = ctx->theta[26 + 25];
    io.vscale = P.dke + 2;
    io.ke_mobile = 1;
    MdIO io0 = io;
    io0.dt = 0.0;
    int iters = 0;
    const int mdflags = CTBOP_FLAG_WARM_START | CTBOP_FLAG_EXTRAPOLATE;
    rc = eval_any(ctx, P, mdflags, &iters);
    if (rc) return rc;
    hipLaunchKernelGGL(k_md_kick, g, b, 0, P.st, P.dtiles, P.dseg, io0);
    hipLaunchKernelGGL(k_fin_ke, g1, b, 0, P.st, P.dsegid, P.dseg, P.dke);
    hipLaunchKernelGGL(k_nhc, g1, dim3(64), 0, P.st, P.dke, chain, c, nsteps > 0 ? 0 : 3);
    for (int s = 0; s <= nsteps; s++) {
        if (s > 0) {
            hipLaunchKernelGGL(k_md_kick_drift, g, b, 0, P.st, P.dtiles, P.dseg, io);
            rc = eval_any(ctx, P, mdflags, &iters);
            if (rc) return rc;
            hipLaunchKernelGGL(k_md_kick, g, b, 0, P.st, P.dtiles, P.dseg, io);
            hipLaunchKernelGGL(k_fin_ke, g1, b, 0, P.st, P.dsegid, P.dseg, P.dke);
            hipLaunchKernelGGL(k_nhc, g1, dim3(64), 0, P.st, P.dke, chain, c, s < nsteps ? 1 : 2);
            HIPCHK(hipGetLastError());
        }
        if (thermo && s % every == 0) {
            double kv[5];
            HIPCHK(hipMemcpyAsync(kv, P.dke, sizeof kv, hipMemcpyDeviceToHost, P.st));
            HIPCHK(hipStreamSynchronize(P.st));
            thermo[3 * (s / every)] = kv[1];
            thermo[3 * (s / every) + 1] = kv[3];
            thermo[3 * (s / every) + 2] = kv[1] + kv[3] + kv[4];
        }
        if (s % 64 == 0 || s == nsteps) {
            int code = 0;
            HIPCHK(hipMemcpyAsync(&code, &P.L.seg.sst->status, sizeof(int), hipMemcpyDeviceToHost, P.st));
            HIPCHK(hipStreamSynchronize(P.st));
            if (code) return fail(map_status(code), status_text(code));
        }
    }
    // the last thermostat half step's scale
    if (nsteps > 0) hipLaunchKernelGGL(k_md_scale, g, b, 0, P.st, P.dtiles, P.dseg, io);
    HIPCHK(hipGetLastError());
    if (info) return fill_info(ctx, P, info);
    HIPCHK(hipStreamSynchronize(P.st));
    return CTBOP_OK;
}

int ctbop_relax_fire(ctbop_ctx *ctx, int n, double *x, double *v, const int32_t *types, const uint8_t *fixed,
                     const double *box, const int *pbc, double Q, double fmax, int max_steps, double dt0,
                     double dtmax, void *sys, size_t sys_bytes, double *F, double *q, double *E_trace,
                     int *steps_out, double *fmax_out, int *converged, ctbop_info *info, void *stream)
{
    if (!x || !v || !types || !F || !q || max_steps < 0) return fail(CTBOP_E_INVAL, "bad argument");
    if (!(fmax > 0) || !(dt0 > 0) || !(dtmax >= dt0)) return fail(CTBOP_E_INVAL, "need fmax, dt0 > 0, dtmax >= dt0");
    // the published FIRE constants
    const int n_min = 5;
    const double f_inc = 1.1, f_dec = 0.5, alpha_start = 0.1, f_alpha = 0.99;
    Prep P;
    int rc = prepare(ctx, n, box, pbc, sys, sys_bytes, stream, P);
    if (rc) return rc;
    Seg S = P.L.seg;
    S.x = x;
    S.type = types;
    S.F = F;
    S.q_out = q;
    S.E_out = nullptr;
    S.Q = Q;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    HIPCHK(hipMemsetAsync(v, 0, 3 * sizeof(double) * (size_t)n, P.st));
    const dim3 g(P.L.ntile), b(TILE), g1(1);
    MdIO io;
    io.x = x;
    io.v = v;
    io.F = F;
    io.fixed = fixed;
    io.dt = 0.0;
    io.mass[0] = ctx->theta[25];
    io.mass[1] = ctx->theta[26 + 25];
    // the charge solve starts from the polynomial extrapolation of the last
    // solutions, as in MD: the minimiser's path is no time series, but it is
    // smooth between restarts (measured: 3 % faster per iteration than
    // starting from the last charges)
    const int flags = CTBOP_FLAG_WARM_START | CTBOP_FLAG_EXTRAPOLATE;
    int iters = 0;
    double red[6];
    auto evaluate = [&]() -> int {
        int r = eval_any(ctx, P, flags, &iters);
        if (r) return r;
        hipLaunchKernelGGL(k_fire_kick, g, b, 0, P.st, P.dtiles, P.dseg, io);
        hipLaunchKernelGGL(k_fire_fin, g1, b, 0, P.st, P.dsegid, P.dseg, P.dke);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(red, P.dke, sizeof red, hipMemcpyDeviceToHost, P.st));
        HIPCHK(hipStreamSynchronize(P.st));
        const int code = (int)red[5];
        if (code) return fail(map_status(code), status_text(code));
        return CTBOP_OK;
    };
    rc = evaluate();
    if (rc) return rc;
    double dt = dt0, alpha = alpha_start;
    int n_pos = 0, s = 0, conv = 0;
    for (;;) {
        if (E_trace) E_trace[s] = red[4];
        const double fm = sqrt(red[3]);
        if (fmax_out) *fmax_out = fm;
        if (fm < fmax) {
            conv = 1;
            break;
        }
        if (s == max_steps) break;
        double cv = 1.0, cf = 0.0;
        if (s > 0) {
            cv = 1.0 - alpha;
            cf = red[2] > 0.0 ? alpha * sqrt(red[1]) / sqrt(red[2]) : 0.0;
            if (red[0] > 0.0) {
                if (++n_pos > n_min) {
                    dt = std::min(dt * f_inc, dtmax);
                    alpha *= f_alpha;
                }
            } else {
                dt *= f_dec;
                cv = cf = 0.0;
                alpha = alpha_start;
                n_pos = 0;
            }
        }
        io.dt = dt;
        hipLaunchKernelGGL(k_fire_kick_drift, g, b, 0, P.st, P.dtiles, P.dseg, io, cv, cf);
        rc = evaluate();
        if (rc) return rc;
        s++;
    }
    if (steps_out) *steps_out = s;
    if (converged) *converged = conv;
    if (info) return fill_info(ctx, P, info);
    return CTBOP_OK;
}

int ctbop_status(ctbop_ctx *ctx, void *sys, size_t sys_bytes, void *stream, int *code)
{
    if (!ctx || !sys || !code) return fail(CTBOP_E_INVAL, "null argument");
    auto it = ctx->seen.find(sys);
    if (it == ctx->seen.end()) return fail(CTBOP_E_INVAL, "system buffer not used with this context");
    Layout L;
    int rc = make_layout(ctx, it->second.n, it->second.box, it->second.pbc, (char *)sys, L);
    if (rc) return rc;
    if (sys_bytes < L.bytes) return fail(CTBOP_E_NOMEM, "system buffer too small");
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, &L.seg.sst->status, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    *code = map_status(st);
    return CTBOP_OK;
}

const char *ctbop_last_error(void) { return g_err.c_str(); }

int ctbop_profile(ctbop_ctx *ctx, int enable, int reset, void *stream, double *ms_out, long *count_out, int nk)
{
    if (!ctx) return fail(CTBOP_E_INVAL, "null context");
    if (stream || !ctx->ev_pending.empty()) {
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        ev_harvest(ctx);
    }
    for (int k = 0; k < nk && k < 16; k++) {
        if (ms_out) ms_out[k] = ctx->prof_ms[k];
        if (count_out) count_out[k] = ctx->prof_n[k];
    }
    if (reset)
        for (int k = 0; k < 16; k++) {
            ctx->prof_ms[k] = 0.0;
            ctx->prof_n[k] = 0;
        }
    ctx->profile = enable ? 1 : 0;
    return CTBOP_OK;
}

int ctbop_profile_classes(ctbop_ctx *ctx, unsigned mask)
{
    if (!ctx) return fail(CTBOP_E_INVAL, "null context");
    ctx->profile_mask = mask & 0xffffu;
    return CTBOP_OK;
}

int ctbop_debug_lists(ctbop_ctx *ctx, int n, void *sys, size_t sys_bytes, int long_cap, int short_cap,
                      int *cl, int *jl, double *dl, int *cs, int *js, double *ds, void *stream)
{
    if (!ctx || !sys) return fail(CTBOP_E_INVAL, "null argument");
    auto it = ctx->seen.find(sys);
    if (it == ctx->seen.end() || it->second.n != n) return fail(CTBOP_E_INVAL, "system buffer not set up for n atoms");
    Layout L;
    int rc = make_layout(ctx, n, it->second.box, it->second.pbc, (char *)sys, L);
    if (rc) return rc;
    const Seg &S = L.seg;
    hipStream_t st = (hipStream_t)stream;
    const size_t np = S.npad;
    std::vector<int> perm(np), lcnt(np), scnt(np);
    std::vector<uint32_t> lidx(np * S.Wl), sidx(np * S.Ws);
    std::vector<double> off(3 * np);
    const size_t v4 = ctx->opts.fp64 ? 32 : 16;
    std::vector<char> xs(v4 * np);
    HIPCHK(hipMemcpyAsync(perm.data(), S.perm, 4 * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(lcnt.data(), S.lcnt, 4 * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(scnt.data(), S.scnt, 4 * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(lidx.data(), S.lidx, 4 * np * S.Wl, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sidx.data(), S.sidx, 4 * np * S.Ws, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(xs.data(), S.xs, v4 * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    auto pos = [&](int s, int a) -> double {
        if (ctx->opts.fp64) return ((const double *)xs.data())[4 * s + a];
        return (double)((const float *)xs.data())[4 * s + a];
    };
    auto emit = [&](int s, const uint32_t *row, size_t stride, int cnt, int cap, int *counts, int *jj, double *dd) {
        const int i = perm[s];
        counts[i] = std::min(cnt, cap);
        for (int e = 0; e < counts[i]; e++) {
            const uint32_t ent = row[(size_t)e * stride];
            const int j = (int)(ent & J_MASK), c = (int)(ent >> CODE_SHIFT);
            const int d0 = c / 49 - 3, d1 = (c / 7) % 7 - 3, d2 = c % 7 - 3;
            jj[(size_t)i * cap + e] = perm[j];
            for (int a = 0; a < 3; a++)
                dd[3 * ((size_t)i * cap + e) + a] =
                    pos(j, a) - pos(s, a) + (d0 * S.cw[0][a] + d1 * S.cw[1][a] + d2 * S.cw[2][a]);
        }
    };
    for (int s = 0; s < n; s++) {
        if (cl) emit(s, &lidx[(size_t)s * S.Wl], 1, lcnt[s], long_cap, cl, jl, dl);
        if (cs) emit(s, &sidx[(size_t)s * S.Ws], 1, scnt[s], short_cap, cs, js, ds);
    }
    return CTBOP_OK;
}

} // extern "C"

#include "static_entry.h"
#include "server.h"
#include "removal.h"
#include "adjoint_host.h"
#include "rings_host.h"
