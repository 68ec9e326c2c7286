// static_entry.h -- the allocation-free form of the energy/force/charge
// evaluation (ctbop_compute_energy_forces_charges_static in ctbop.h).
//
// The per-system buffer (lists, sort order, Coulomb rows, solver vectors,
// partial sums) lives in a file-scope device array instead of caller memory,
// so the call needs no device allocation from anyone.  Each device holds its
// own copy of the array, at its own address, for the life of the process.
// Host code never passes the array's name to a kernel or a copy (in host
// code it names a host-side stand-in): the device address is taken once per
// device with hipGetSymbolAddress and kept in static_ptr[].
//
// Included once, from ctbop.hip, after the launch sequence it reuses.
#pragma once

#include <mutex>

#define CTBOP_STATIC_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[CTBOP_STATIC_SCRATCH_BYTES];

namespace {

std::mutex static_mu;
void *static_ptr[CTBOP_STATIC_MAX_DEVICES] = {nullptr};

// Device address of this device's copy of the scratch array, looked up on
// the first call made with the device current.
int static_scratch(void **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= CTBOP_STATIC_MAX_DEVICES) return fail(CTBOP_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(static_mu);
    if (!static_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CTBOP_E_HIP, "hipGetSymbolAddress returned a null address for the scratch array");
        static_ptr[dev] = p;
    }
    *out = static_ptr[dev];
    return CTBOP_OK;
}

} // namespace

extern "C" int ctbop_compute_energy_forces_charges_static(ctbop_ctx *ctx, int n, const double *pos,
                                                          const int32_t *types, const double *box, const int *pbc,
                                                          double Q, double *E, double *F, double *q,
                                                          ctbop_info *info, void *stream)
{
    if (!ctx || !box || !pbc) return fail(CTBOP_E_INVAL, "null argument");
    if (!pos || !types || !F || !q) return fail(CTBOP_E_INVAL, "null array argument");
    // size check first: it needs no device
    Prep P;
    int rc = make_layout(ctx, n, box, pbc, nullptr, P.L);
    if (rc) return rc;
    if (P.L.bytes > (size_t)CTBOP_STATIC_SCRATCH_BYTES)
        return fail(CTBOP_E_NOMEM, "system needs " + std::to_string(P.L.bytes) +
                                       " bytes of scratch; the static scratch holds " +
                                       std::to_string((size_t)CTBOP_STATIC_SCRATCH_BYTES) +
                                       " (use ctbop_compute_energy_forces_charges with a caller buffer)");
    void *sys = nullptr;
    rc = static_scratch(&sys);
    if (rc) return rc;
    P.base = (char *)sys;
    rc = make_layout(ctx, n, box, pbc, P.base, P.L);
    if (rc) return rc;
    P.dseg = (Seg *)(P.base + P.L.off_seg);
    P.dtiles = (Tile *)(P.base + P.L.off_tiles);
    P.dsegid = (int *)(P.base + P.L.off_segid);
    P.dke = (double *)(P.base + P.L.off_ke);
    P.st = (hipStream_t)stream;
    // the array keeps whatever the last call (of any context) left in it:
    // every call starts over (state cleared, lists rebuilt, cold charges)
    P.fresh = true;
    P.own = false;
    int flag[2] = {0, 0};
    P.flag_host = flag;
    hipLaunchKernelGGL(k_reset_state, dim3((P.L.ntile + 255) / 256), dim3(256), 0, P.st, P.L.seg.sst, P.dtiles,
                       P.L.ntile, P.dsegid);
    HIPCHK(hipGetLastError());
    Seg S = P.L.seg;
    S.x = pos;
    S.type = types;
    S.F = F;
    S.q_out = q;
    S.E_out = E;
    S.Q = Q;
    hipLaunchKernelGGL(k_set_seg, dim3(1), dim3(1), 0, P.st, P.dseg, S);
    // no timing events here (creating one may allocate)
    const int prof = ctx->profile;
    ctx->profile = 0;
    int iters = 0;
    rc = eval_any(ctx, P, 0, &iters);
    ctx->profile = prof;
    if (rc) return rc;
    if (info) return fill_info(ctx, P, info);
    return CTBOP_OK;
}
