// removal.h -- removal energies of single atoms (included by ctbop.hip after
// server.h): the full system once, then every leave-one-out system as a
// continuous batch through a server on the rest of the caller's arena.
#pragma once

namespace {

constexpr int REMOVAL_MAX_SLOTS = 64;       // leave-one-out systems in flight at most

// bytes of the full system's inputs/outputs and buffer at the head of the arena
size_t removal_head_bytes(const Layout &L, int n)
{
    return io_bytes(n) + L.bytes;
}

} // namespace

extern "C" {

int ctbop_removal_bytes(ctbop_ctx *ctx, int n, const double *box, const int *pbc, int m, size_t *bytes)
{
    if (!ctx || !box || !pbc || !bytes) return fail(CTBOP_E_INVAL, "null argument");
    if (n < 2 || m < 0) return fail(CTBOP_E_INVAL, "need n >= 2 and m >= 0");
    if (ctx->opts.fq_kappa > 0.0) return fail(CTBOP_E_INVAL, "removal energies: not available with fq_kappa > 0");
    Layout L;
    int rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    size_t req;
    rc = ctbop_server_request_bytes(ctx, n - 1, box, pbc, &req);
    if (rc) return rc;
    const int conc = std::max(1, std::min(m, 16));
    const size_t work = (size_t)conc * (req + 256);
    const int slots = std::max(conc, std::min(std::max(m, 1), REMOVAL_MAX_SLOTS));
    const int tiles = 2 * (int)std::min<size_t>(work / ((size_t)TILE * 1024) + slots + 64, 1 << 22);
    *bytes = align_up(removal_head_bytes(L, n), 256) + ctbop_server_table_bytes(slots, tiles) + work + (4 << 20);
    return CTBOP_OK;
}

int ctbop_removal_energies(ctbop_ctx *ctx, int n, const double *pos_host, const int32_t *types_host,
                           const double *box, const int *pbc, double Q, const int *cand_host, int m,
                           void *arena_dev, size_t arena_bytes, double *E_host, double *dE_host, int *iters_host,
                           void *stream)
{
    if (!ctx || !pos_host || !types_host || !box || !pbc || !arena_dev || !E_host || (m > 0 && (!cand_host || !dE_host)))
        return fail(CTBOP_E_INVAL, "null argument");
    if (n < 2 || m < 0) return fail(CTBOP_E_INVAL, "need n >= 2 and m >= 0");
    for (int k = 0; k < m; k++)
        if (cand_host[k] < 0 || cand_host[k] >= n) return fail(CTBOP_E_INVAL, "candidate index out of range");
    size_t need;
    int rc = ctbop_removal_bytes(ctx, n, box, pbc, std::min(m, 1), &need);
    if (rc) return rc;
    if (arena_bytes < need) return fail(CTBOP_E_NOMEM, "arena smaller than ctbop_removal_bytes()");
    hipStream_t st = (hipStream_t)stream;
    // full system at the head of the arena
    Layout L;
    rc = make_layout(ctx, n, box, pbc, nullptr, L);
    if (rc) return rc;
    char *a = (char *)arena_dev;
    double *x = (double *)a;
    int32_t *ty = (int32_t *)(a + align_up(8 * 3 * (size_t)n, 256));
    double *F = (double *)((char *)ty + align_up(4 * (size_t)n, 256));
    double *q = (double *)((char *)F + align_up(8 * 3 * (size_t)n, 256));
    double *E = (double *)((char *)q + align_up(8 * (size_t)n, 256));
    char *sys = a + io_bytes(n);
    const size_t head = align_up(removal_head_bytes(L, n), 256);
    HIPCHK(hipMemcpyAsync(x, pos_host, 8 * 3 * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ty, types_host, 4 * (size_t)n, hipMemcpyHostToDevice, st));
    ctbop_info info;
    rc = ctbop_compute_energy_forces_charges(ctx, n, x, ty, box, pbc, Q, CTBOP_FLAG_FORCE_REBUILD, sys, L.bytes,
                                             E, F, q, &info, stream);
    // the buffer is not kept for a later call
    ctx->seen.erase(sys);
    ctx->last_iters.erase(sys);
    ctx->eval_gen.erase(sys);
    if (rc) return rc;
    std::vector<double> qh(n);
    HIPCHK(hipMemcpyAsync(qh.data(), q, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(E_host, E, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (m == 0) return CTBOP_OK;
    // leave-one-out systems, each starting from the full system's charges
    ctbop_server *srv = nullptr;
    const int slots = std::max(1, std::min(m, REMOVAL_MAX_SLOTS));
    rc = ctbop_server_create(ctx, a + head, arena_bytes - head, slots, 8, stream, &srv);
    if (rc) return rc;
    std::vector<double> Ek(m, 0.0);
    std::vector<int> status(m, -1), iters(m, 0);
    std::unordered_map<long, int> which;
    std::vector<double> xs(3 * (size_t)(n - 1)), q0(n - 1);
    std::vector<int32_t> ts(n - 1);
    const int window = 4 * slots;              // requests pending in the server at most
    int next = 0, done = 0, err = CTBOP_OK;
    std::vector<ctbop_result> res(slots);
    while (done < m && err == CTBOP_OK) {
        while (next < m && next - done < window) {
            const int i = cand_host[next];
            for (int d = 0; d < 3; d++) {
                const double *src = pos_host + (size_t)d * n;
                double *dst = xs.data() + (size_t)d * (n - 1);
                std::copy(src, src + i, dst);
                std::copy(src + i + 1, src + n, dst + i);
            }
            std::copy(types_host, types_host + i, ts.begin());
            std::copy(types_host + i + 1, types_host + n, ts.begin() + i);
            std::copy(qh.begin(), qh.begin() + i, q0.begin());
            std::copy(qh.begin() + i + 1, qh.end(), q0.begin() + i);
            ctbop_request r;
            memset(&r, 0, sizeof r);
            r.n = n - 1;
            r.pos_host = xs.data();
            r.types_host = ts.data();
            memcpy(r.box, box, sizeof r.box);
            for (int d = 0; d < 3; d++) r.pbc[d] = pbc[d];
            r.total_charge = Q;
            r.system_id = -1;
            r.E_host = &Ek[next];
            r.q0_host = q0.data();
            long t;
            const int s = ctbop_server_submit(srv, &r, &t);
            if (s == CTBOP_E_BUSY) break;
            if (s) {
                err = s;
                break;
            }
            which[t] = next++;
        }
        if (err) break;
        int got = 0;
        const int p = ctbop_server_poll(srv, res.data(), slots, 0.05, &got);
        if (p) err = p;
        for (int k = 0; k < got; k++) {
            const int c = which[res[k].ticket];
            status[c] = res[k].status;
            iters[c] = res[k].cg_iters;
            done++;
        }
    }
    ctbop_server_destroy(srv);
    if (err) return err;
    for (int k = 0; k < m; k++) {
        if (status[k] != CTBOP_OK)
            return fail(status[k], "removal of atom " + std::to_string(cand_host[k]) + " failed");
        dE_host[k] = Ek[k] - *E_host;
        if (iters_host) iters_host[k] = iters[k];
    }
    return CTBOP_OK;
}

} // extern "C"
