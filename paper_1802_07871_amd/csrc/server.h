// server.h -- continuous-batching serving engine (host side), included by
// ctbop.hip after the single-system path.
//
// Every admitted request is a segment: one region of the caller's arena holds
// its inputs, outputs and the same per-system layout the single-system path
// uses, and one entry of a device table holds its descriptor.  A scheduler
// thread runs ticks on one stream:
//   1. admit pending requests in arrival order while slots and arena bytes
//      allow (a request that does not fit waits; retained systems are evicted
//      least recently used first);
//   2. set-up kernels (bins, lists, bond pass, Coulomb assembly) over the new
//      segments' tiles, all in one launch per kernel;
//   3. K charge-solve iterations over every active segment's tiles, again one
//      launch per kernel; each segment stops on its own test;
//   4. force and energy kernels over the same tiles, gated per segment on
//      "solve finished, forces pending";
//   5. read the per-segment flags, copy finished results to the caller's host
//      buffers and free (or retain) their regions.
// Requests that arrive during a tick join at the next one, so work of
// requests of any size and phase overlaps on the device.  Each segment's
// arithmetic and reduction order do not depend on the other segments, so a
// result is bitwise the same alone and in the mix.
#pragma once
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SrvReq {
    long ticket;
    int n;
    std::vector<double> pos;
    std::vector<int32_t> types;
    double box[9];
    int pbc[3];
    double Q;
    long sys_id;
    std::vector<double> q0;         // starting charges (user order), or empty
    double *E_out, *F_out, *q_out;
    double t_submit, t_admit;
};

enum SlotState { FREE = 0, ACTIVE = 1, RETAINED = 2 };

struct SrvSlot {
    int state = FREE;
    SrvReq req;
    size_t off = 0, bytes = 0;      // region in the arena
    Layout L;
    size_t io_off = 0;              // I/O arrays at the start of the region
    int phase = 0;                  // 0 = needs set-up, 1 = solving/finishing
    long sys_id = -1;
    double last_use = 0;
    Sig sig;
};

} // namespace

struct ctbop_server {
    ctbop_ctx *ctx = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0;
    int cg_per_tick = 8;
    int iters_hint = 0;      // solver iterations of the last finished request (tick thread only)
    int device = 0;
    hipStream_t stream = nullptr;
    // the covalent kernels of newly set-up systems run on a stream of the
    // server's own beside the assembly and the solve, joined before the
    // Coulomb forces (as the single-system path does)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // device tables at the head of the arena
    Seg *dsegs = nullptr;
    Tile *dtiles_setup = nullptr, *dtiles_act = nullptr;
    int *dids_setup = nullptr, *dids_act = nullptr;
    int4 *dflags = nullptr;
    int max_tiles = 0;
    // host mirrors (pinned)
    Tile *htiles = nullptr;
    int *hids = nullptr;
    int4 *hflags = nullptr;
    // regions
    std::map<size_t, size_t> free_ranges;   // offset -> size
    std::vector<SrvSlot> slots;
    std::deque<SrvReq> pending;
    std::deque<ctbop_result> done;
    long next_ticket = 1;
    size_t max_pending = 1 << 20;
    // thread
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    int error = 0;
    std::string errmsg;
    // statistics
    long ticks = 0, admitted = 0, completed = 0;
    double busy_s = 0;
    size_t peak_bytes = 0, used_bytes = 0;
};

namespace {

size_t io_bytes(int n) { return align_up(8 * 3 * (size_t)n, 256) + align_up(4 * (size_t)n, 256) +
                                align_up(8 * 3 * (size_t)n, 256) + align_up(8 * (size_t)n, 256) + 256; }

bool range_alloc(ctbop_server *S, size_t bytes, size_t &off)
{
    for (auto it = S->free_ranges.begin(); it != S->free_ranges.end(); ++it) {
        if (it->second >= bytes) {
            off = it->first;
            size_t rest = it->second - bytes;
            S->free_ranges.erase(it);
            if (rest) S->free_ranges[off + bytes] = rest;
            S->used_bytes += bytes;
            S->peak_bytes = std::max(S->peak_bytes, S->used_bytes);
            return true;
        }
    }
    return false;
}

void range_free(ctbop_server *S, size_t off, size_t bytes)
{
    S->used_bytes -= bytes;
    auto it = S->free_ranges.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != S->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        S->free_ranges.erase(nx);
    }
    if (it != S->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            S->free_ranges.erase(it);
        }
    }
}

Sig req_sig(const ctbop_ctx *ctx, const SrvReq &r, size_t bytes)
{
    Sig g;
    memset(&g, 0, sizeof g);
    g.n = r.n;
    memcpy(g.box, r.box, sizeof g.box);
    for (int a = 0; a < 3; a++) g.pbc[a] = r.pbc[a] ? 1 : 0;
    g.fp64 = ctx->opts.fp64;
    g.bytes = bytes;
    return g;
}

// place a request into a slot: region, descriptor, inputs.  Returns false if
// it does not fit right now.
int admit_one(ctbop_server *S, SrvReq &r, bool &placed)
{
    placed = false;
    ctbop_ctx *ctx = S->ctx;
    // a retained system with the same id and geometry keeps its lists and charges
    int reuse = -1, freeslot = -1;
    for (int k = 0; k < S->max_slots; k++) {
        SrvSlot &sl = S->slots[k];
        if (sl.state == RETAINED && r.sys_id >= 0 && sl.sys_id == r.sys_id) reuse = k;
        if (sl.state == FREE && freeslot < 0) freeslot = k;
    }
    Layout L;
    int rc = make_layout(ctx, r.n, r.box, r.pbc, nullptr, L);
    if (rc) return rc;
    const size_t iob = io_bytes(r.n);
    const size_t need = iob + L.bytes;
    Sig sg = req_sig(ctx, r, L.bytes);
    int k = -1;
    bool fresh = true;
    if (reuse >= 0 && S->slots[reuse].sig == sg) {
        k = reuse;
        fresh = false;
    } else {
        if (reuse >= 0) {                  // same id, new geometry: drop the old state
            range_free(S, S->slots[reuse].off, S->slots[reuse].bytes);
            S->slots[reuse].state = FREE;
            if (freeslot < 0) freeslot = reuse;
        }
        size_t off;
        while (!range_alloc(S, need, off)) {
            // evict the least recently used retained system, if any
            int lru = -1;
            for (int j = 0; j < S->max_slots; j++)
                if (S->slots[j].state == RETAINED && (lru < 0 || S->slots[j].last_use < S->slots[lru].last_use)) lru = j;
            if (lru < 0) return CTBOP_OK;  // wait for running requests to finish
            range_free(S, S->slots[lru].off, S->slots[lru].bytes);
            S->slots[lru].state = FREE;
            if (freeslot < 0) freeslot = lru;
        }
        if (freeslot < 0) {
            range_free(S, off, need);
            return CTBOP_OK;
        }
        k = freeslot;
        S->slots[k].off = off;
        S->slots[k].bytes = need;
    }
    SrvSlot &sl = S->slots[k];
    char *base = S->arena + sl.off;
    rc = make_layout(ctx, r.n, r.box, r.pbc, base + iob, sl.L);
    if (rc) return rc;
    sl.io_off = 0;
    sl.sig = sg;
    sl.sys_id = r.sys_id;
    sl.state = ACTIVE;
    sl.phase = 0;
    sl.req = std::move(r);
    sl.req.t_admit = now_s();
    sl.last_use = sl.req.t_admit;
    const int n = sl.req.n;
    double *x = (double *)base;
    int32_t *ty = (int32_t *)(base + align_up(8 * 3 * (size_t)n, 256));
    double *F = (double *)((char *)ty + align_up(4 * (size_t)n, 256));
    double *q = (double *)((char *)F + align_up(8 * 3 * (size_t)n, 256));
    double *E = (double *)((char *)q + align_up(8 * (size_t)n, 256));
    Seg sd = sl.L.seg;
    sd.x = x;
    sd.type = ty;
    sd.F = F;
    sd.q_out = q;
    sd.E_out = E;
    sd.Q = sl.req.Q;
    HIPCHK(hipMemcpyAsync(x, sl.req.pos.data(), 8 * 3 * (size_t)n, hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(ty, sl.req.types.data(), 4 * (size_t)n, hipMemcpyHostToDevice, S->stream));
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, S->stream, S->dsegs + k, sd);
    if (fresh)
        hipLaunchKernelGGL(k_reset_state, dim3((sl.L.ntile + 255) / 256), dim3(256), 0, S->stream, sd.sst,
                           (Tile *)(base + iob + sl.L.off_tiles), sl.L.ntile, (int *)(base + iob + sl.L.off_segid));
    // starting charges given with the request replace the warm-start state;
    // a retained system otherwise starts from its last charges
    const bool given = !sl.req.q0.empty();
    if (given)
        HIPCHK(hipMemcpyAsync(sd.q_state, sl.req.q0.data(), 8 * (size_t)n, hipMemcpyHostToDevice, S->stream));
    hipLaunchKernelGGL(k_set_warm, dim3(1), dim3(1), 0, S->stream, sd.sst, (fresh && !given) ? 0 : 1);
    HIPCHK(hipGetLastError());
    S->admitted++;
    placed = true;
    return CTBOP_OK;
}

// One tick: set up the newly admitted systems, run cg_iters solver
// iterations over every active system, then the (gated) force kernels and
// the harvest.  With poll set (nobody waiting for admission when the tick
// began) the iterations go in chunks, the first as long as the last finished
// request needed, then cg_check each, with a convergence check after each
// chunk: the tick goes on until an active system has converged (or the
// iteration limit), so that it is harvested at once, unless a request
// arrives, which ends it at the next check once cg_iters have run.  A lone
// request is then served in one tick, like a plain call.
template <typename R>
int server_tick(ctbop_server *S, const Params<R> &prm, int cg_iters, bool poll)
{
    ctbop_ctx *ctx = S->ctx;
    hipStream_t st = S->stream;
    // tables: set-up tiles/ids and active tiles/ids
    int nts = 0, nis = 0, nta = 0, nia = 0;
    std::vector<int> act;
    for (int k = 0; k < S->max_slots; k++) {
        SrvSlot &sl = S->slots[k];
        if (sl.state != ACTIVE) continue;
        act.push_back(k);
    }
    if (act.empty()) return CTBOP_OK;
    int total_tiles = 0;
    for (int k : act) total_tiles += S->slots[k].L.ntile;
    if (total_tiles > S->max_tiles) return fail(CTBOP_E_NOMEM, "server tile table too small");
    Tile *hts = S->htiles, *hta = S->htiles + S->max_tiles;
    int *his = S->hids, *hia = S->hids + S->max_slots;
    for (int k : act) {
        SrvSlot &sl = S->slots[k];
        for (int t = 0; t < sl.L.ntile; t++) {
            Tile tt;
            tt.seg = k;
            tt.row0 = t * TILE;
            if (sl.phase == 0) hts[nts++] = tt;
            hta[nta++] = tt;
        }
        if (sl.phase == 0) his[nis++] = k;
        hia[nia++] = k;
    }
    HIPCHK(hipMemcpyAsync(S->dtiles_setup, hts, sizeof(Tile) * std::max(nts, 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(S->dtiles_act, hta, sizeof(Tile) * nta, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(S->dids_setup, his, sizeof(int) * std::max(nis, 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(S->dids_act, hia, sizeof(int) * nia, hipMemcpyHostToDevice, st));
    const dim3 b(TILE);
    if (nts) {
        const dim3 g(nts), gs(nis);
        const int *sid = S->dids_setup;
        Tile *T = S->dtiles_setup;
        hipLaunchKernelGGL(k_call_init, dim3((nis + 63) / 64), dim3(64), 0, st, sid, S->dsegs, nis, 0);
        hipLaunchKernelGGL(k_check_disp, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_bin_clear, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_bin, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_scan_part, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_scan_mid, gs, b, 0, st, sid, S->dsegs);
        hipLaunchKernelGGL(k_scan_fin, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_scatter, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_cell_sort, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_gather<R>, g, b, 0, st, T, S->dsegs, -1);
        hipLaunchKernelGGL(k_fin_qshift, gs, b, 0, st, sid, S->dsegs);
        hipLaunchKernelGGL(k_qfix, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL((k_build<R, BUILD_L>), g, b, 0, st, T, S->dsegs, prm);
        hipLaunchKernelGGL(k_rev, g, b, 0, st, T, S->dsegs);
        hipLaunchKernelGGL(k_mark_built, dim3((nis + 63) / 64), dim3(64), 0, st, sid, S->dsegs, nis);
        hipLaunchKernelGGL((k_assemble<R, LPR>), g, b, 0, st, T, S->dsegs, ctx->pd);
        hipLaunchKernelGGL((k_hslice<R>), g, b, 0, st, T, S->dsegs);
        // covalent energy and forces need only the lists: side stream, forked
        // after the sliced copy so that they run beside the solve
        HIPCHK(hipEventRecord(S->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(S->side, S->ev_fork, 0));
        hipLaunchKernelGGL((k_bond<R>), g, b, 0, S->side, T, S->dsegs, ctx->pd);
        hipLaunchKernelGGL((k_force_cov<R>), g, b, 0, S->side, T, S->dsegs, prm, 0);
        HIPCHK(hipEventRecord(S->ev_join, S->side));
        hipLaunchKernelGGL(k_fin_w0, gs, b, 0, st, sid, S->dsegs);
        hipLaunchKernelGGL((k_cg1_update<true>), g, b, 0, st, T, S->dsegs);
    }
    {
        const dim3 g(nta), gs(nia);
        const int *sid = S->dids_act;
        Tile *T = S->dtiles_act;
        CgCtl ctl{ctx->opts.cg_tol, ctx->opts.cg_maxit};
        // single-reduction solve: a solve of n iterations takes n + 1 rounds
        // (its first finalize counts none)
        const int limit = poll ? ctx->opts.cg_maxit + 2 : cg_iters;
        for (int c = 0; c < limit;) {
            const int first = std::max(ctx->opts.cg_check, std::min(S->iters_hint, ctx->opts.cg_maxit) + 1);
            const int chunk = poll ? std::min(limit - c, c == 0 ? first : ctx->opts.cg_check) : cg_iters;
            for (int k = 0; k < chunk; k++) {
                hipLaunchKernelGGL((k_spmv<R, SPMV_U, SP_CG1>), g, b, 0, st, T, S->dsegs);
                hipLaunchKernelGGL(k_cg1_sum, dim3(nia * FIN_SPLIT), b, 0, st, sid, S->dsegs);
                hipLaunchKernelGGL(k_cg1_fin, gs, b, 0, st, sid, S->dsegs, ctl);
                hipLaunchKernelGGL((k_cg1_update<false>), g, b, 0, st, T, S->dsegs);
            }
            c += chunk;
            if (!poll || c >= limit) break;
            hipLaunchKernelGGL(k_collect, dim3((nia + 63) / 64), dim3(64), 0, st, sid, S->dsegs, nia, S->dflags);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(S->hflags, S->dflags, sizeof(int4) * nia, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            bool any_done = false;
            for (int a = 0; a < nia; a++) any_done = any_done || S->hflags[a].x != 0;
            if (any_done) break;
            if (c >= cg_iters) {
                std::lock_guard<std::mutex> lk(S->mu);
                if (!S->pending.empty()) break;
            }
        }
        if (nts) HIPCHK(hipStreamWaitEvent(st, S->ev_join, 0));
        hipLaunchKernelGGL((k_force_coul<R, LPR>), g, b, 0, st, T, S->dsegs, ctx->pd, 1);
        hipLaunchKernelGGL(k_fin_energy, gs, b, 0, st, sid, S->dsegs, 1);
        hipLaunchKernelGGL(k_collect, dim3((nia + 63) / 64), dim3(64), 0, st, sid, S->dsegs, nia, S->dflags);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(S->hflags, S->dflags, sizeof(int4) * nia, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    // harvest
    std::vector<int> fin;
    for (int a = 0; a < nia; a++) {
        SrvSlot &sl = S->slots[hia[a]];
        sl.phase = 1;
        if (S->hflags[a].y) fin.push_back(a);
    }
    for (int a : fin) {
        SrvSlot &sl = S->slots[hia[a]];
        const int n = sl.req.n;
        char *base = S->arena + sl.off;
        double *F = (double *)(base + align_up(8 * 3 * (size_t)n, 256) + align_up(4 * (size_t)n, 256));
        double *q = (double *)((char *)F + align_up(8 * 3 * (size_t)n, 256));
        double *E = (double *)((char *)q + align_up(8 * (size_t)n, 256));
        if (sl.req.F_out) HIPCHK(hipMemcpyAsync(sl.req.F_out, F, 8 * 3 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (sl.req.q_out) HIPCHK(hipMemcpyAsync(sl.req.q_out, q, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (sl.req.E_out) HIPCHK(hipMemcpyAsync(sl.req.E_out, E, 8, hipMemcpyDeviceToHost, st));
    }
    if (!fin.empty()) HIPCHK(hipStreamSynchronize(st));
    const double t = now_s();
    std::vector<ctbop_result> res;
    for (int a : fin) {
        SrvSlot &sl = S->slots[hia[a]];
        ctbop_result r;
        r.ticket = sl.req.ticket;
        r.status = map_status(S->hflags[a].z);
        r.cg_iters = S->hflags[a].w;
        S->iters_hint = r.cg_iters;
        r.n_atoms = sl.req.n;
        r.t_submit = sl.req.t_submit;
        r.t_admit = sl.req.t_admit;
        r.t_done = t;
        res.push_back(r);
        sl.last_use = t;
        if (sl.sys_id >= 0) {
            sl.state = RETAINED;
        } else {
            range_free(S, sl.off, sl.bytes);
            sl.state = FREE;
        }
        sl.req.pos.clear();
        sl.req.pos.shrink_to_fit();
        sl.req.types.clear();
        sl.req.types.shrink_to_fit();
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &r : res) S->done.push_back(r);
        S->completed += (long)res.size();
        S->ticks++;
    }
    if (!res.empty()) S->cv.notify_all();
    return CTBOP_OK;
}

// the server's stream, events and pinned tables (whichever exist)
void release_handles(ctbop_server *S)
{
    if (S->side) {
        (void)hipStreamSynchronize(S->side);
        (void)hipStreamDestroy(S->side);
    }
    if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
    if (S->ev_join) (void)hipEventDestroy(S->ev_join);
    if (S->htiles) (void)hipHostFree(S->htiles);
    if (S->hids) (void)hipHostFree(S->hids);
    if (S->hflags) (void)hipHostFree(S->hflags);
}

void server_loop(ctbop_server *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        // solver iterations of this tick: with nobody waiting for admission,
        // iterate until the active systems converge (checked between chunks),
        // so a lone request finishes in one tick (each tick costs table
        // uploads, host round trips and the gated force launches)
        int cg_iters = S->cg_per_tick;
        bool poll = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            bool any_active = false;
            for (auto &sl : S->slots)
                if (sl.state == ACTIVE) any_active = true;
            S->cv.wait(lk, [&] { return S->stop || !S->pending.empty() || any_active; });
            if (S->stop) return;
            // admission in arrival order
            while (!S->pending.empty()) {
                bool placed = false;
                int rc = admit_one(S, S->pending.front(), placed);
                if (rc) {
                    S->error = rc;
                    S->errmsg = g_err;
                    ctbop_result r;
                    memset(&r, 0, sizeof r);
                    r.ticket = S->pending.front().ticket;
                    r.status = rc;
                    r.n_atoms = S->pending.front().n;
                    r.t_submit = S->pending.front().t_submit;
                    r.t_admit = r.t_done = now_s();
                    S->done.push_back(r);
                    S->pending.pop_front();
                    continue;
                }
                if (!placed) break;
                S->pending.pop_front();
            }
            if (S->pending.empty()) poll = true;
        }
        const double t0 = now_s();
        int rc = S->ctx->opts.fp64 ? server_tick<double>(S, S->ctx->pd, cg_iters, poll)
                                   : server_tick<float>(S, S->ctx->pf, cg_iters, poll);
        S->busy_s += now_s() - t0;
        if (rc) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->error = rc;
            S->errmsg = g_err;
            S->stop = true;
            S->cv.notify_all();
            return;
        }
    }
}

} // namespace

extern "C" {

size_t ctbop_server_table_bytes(int max_slots, int max_tiles)
{
    return align_up(sizeof(Seg) * max_slots, 256) + 2 * align_up(sizeof(Tile) * max_tiles, 256) +
           2 * align_up(sizeof(int) * max_slots, 256) + align_up(sizeof(int4) * max_slots, 256);
}

int ctbop_server_request_bytes(ctbop_ctx *ctx, int n, const double *box, const int *pbc, size_t *bytes)
{
    if (!ctx || !bytes) return fail(CTBOP_E_INVAL, "null argument");
    Layout L;
    int rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    *bytes = io_bytes(n) + L.bytes;
    return CTBOP_OK;
}

int ctbop_server_create(ctbop_ctx *ctx, void *arena, size_t arena_bytes, int max_slots, int cg_per_tick,
                        void *stream, ctbop_server **out)
{
    if (!ctx || !arena || !out || max_slots <= 0) return fail(CTBOP_E_INVAL, "bad argument");
    if (ctx->opts.fq_kappa > 0.0) return fail(CTBOP_E_INVAL, "server: not available with fq_kappa > 0");
    ctbop_server *S = new ctbop_server();
    S->ctx = ctx;
    S->arena = (char *)arena;
    S->arena_bytes = arena_bytes;
    S->max_slots = max_slots;
    S->cg_per_tick = cg_per_tick > 0 ? cg_per_tick : 8;
    S->stream = (hipStream_t)stream;
    S->max_tiles = 2 * (int)std::min<size_t>(arena_bytes / ((size_t)TILE * 1024) + max_slots, 1 << 22);
    const size_t tb = ctbop_server_table_bytes(max_slots, S->max_tiles);
    if (tb + (1 << 20) > arena_bytes) {
        delete S;
        return fail(CTBOP_E_NOMEM, "arena too small for the server tables");
    }
    char *p = S->arena;
    S->dsegs = (Seg *)p;
    p += align_up(sizeof(Seg) * max_slots, 256);
    S->dtiles_setup = (Tile *)p;
    p += align_up(sizeof(Tile) * S->max_tiles, 256);
    S->dtiles_act = (Tile *)p;
    p += align_up(sizeof(Tile) * S->max_tiles, 256);
    S->dids_setup = (int *)p;
    p += align_up(sizeof(int) * max_slots, 256);
    S->dids_act = (int *)p;
    p += align_up(sizeof(int) * max_slots, 256);
    S->dflags = (int4 *)p;
    p += align_up(sizeof(int4) * max_slots, 256);
    S->free_ranges[tb] = arena_bytes - tb;
    S->slots.resize(max_slots);
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&S->htiles, sizeof(Tile) * 2 * S->max_tiles, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&S->hids, sizeof(int) * 2 * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&S->hflags, sizeof(int4) * max_slots, hipHostMallocDefault) != hipSuccess) {
        release_handles(S);
        delete S;
        return fail(CTBOP_E_HIP, "server stream, events or pinned host tables");
    }
    S->th = std::thread(server_loop, S);
    ctx->servers++;
    *out = S;
    return CTBOP_OK;
}

int ctbop_server_submit(ctbop_server *S, const ctbop_request *rq, long *ticket)
{
    if (!S || !rq || !rq->pos_host || !rq->types_host || rq->n <= 0) return fail(CTBOP_E_INVAL, "bad request");
    size_t need;
    int rc = ctbop_server_request_bytes(S->ctx, rq->n, rq->box, rq->pbc, &need);
    if (rc) return rc;
    if (need + ctbop_server_table_bytes(S->max_slots, S->max_tiles) > S->arena_bytes)
        return fail(CTBOP_E_NOMEM, "request larger than the serving arena");
    SrvReq r;
    r.n = rq->n;
    r.pos.assign(rq->pos_host, rq->pos_host + 3 * (size_t)rq->n);
    r.types.assign(rq->types_host, rq->types_host + rq->n);
    memcpy(r.box, rq->box, sizeof r.box);
    for (int a = 0; a < 3; a++) r.pbc[a] = rq->pbc[a];
    r.Q = rq->total_charge;
    r.sys_id = rq->system_id;
    if (rq->q0_host) r.q0.assign(rq->q0_host, rq->q0_host + rq->n);
    r.E_out = rq->E_host;
    r.F_out = rq->F_host;
    r.q_out = rq->q_host;
    r.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(S->error ? S->error : CTBOP_E_INVAL, "server stopped: " + S->errmsg);
        if (S->pending.size() >= S->max_pending) return fail(CTBOP_E_BUSY, "pending queue full");
        r.ticket = S->next_ticket++;
        if (ticket) *ticket = r.ticket;
        S->pending.push_back(std::move(r));
    }
    S->cv.notify_all();
    return CTBOP_OK;
}

int ctbop_server_poll(ctbop_server *S, ctbop_result *out, int max, double wait_s, int *n_done)
{
    if (!S || !n_done) return fail(CTBOP_E_INVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && wait_s > 0)
        S->cv.wait_for(lk, std::chrono::duration<double>(wait_s), [&] { return !S->done.empty() || S->stop; });
    int k = 0;
    while (k < max && !S->done.empty()) {
        out[k++] = S->done.front();
        S->done.pop_front();
    }
    *n_done = k;
    if (S->stop && S->error) return fail(S->error, "server stopped: " + S->errmsg);
    return CTBOP_OK;
}

int ctbop_server_stats(ctbop_server *S, double *out, int nout)
{
    if (!S || !out) return fail(CTBOP_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int active = 0, retained = 0;
    for (auto &sl : S->slots) {
        active += sl.state == ACTIVE;
        retained += sl.state == RETAINED;
    }
    double v[9] = {(double)S->ticks, (double)S->admitted, (double)S->completed, (double)S->pending.size(),
                   (double)active, (double)retained, (double)S->used_bytes, (double)S->peak_bytes, S->busy_s};
    for (int k = 0; k < nout && k < 9; k++) out[k] = v[k];
    return CTBOP_OK;
}

int ctbop_server_destroy(ctbop_server *S)
{
    if (!S) return CTBOP_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    (void)hipStreamSynchronize(S->stream);
    release_handles(S);
    S->ctx->servers--;
    delete S;
    return CTBOP_OK;
}

} // extern "C"
