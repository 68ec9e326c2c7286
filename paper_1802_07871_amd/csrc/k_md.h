// k_md.h -- velocity-Verlet integration (user atom order), NVE or NVT with a
// Nose-Hoover chain thermostat, and FIRE structure relaxation.
//
// Half kick + drift before the force evaluation, half kick after it.  Atoms
// with a nonzero fixed flag neither move nor change velocity (the paper holds
// the bottom of its SiC slab fixed during growth runs) but keep interacting.
#pragma once
#include "ctbop_dev.h"

namespace ctbop {

constexpr double ACC_UNIT = 9.648533212e-3;   // (eV/Angstrom)/amu in Angstrom/fs^2

struct MdIO {
    double *x, *v;
    const double *F;
    const uint8_t *fixed;
    double dt;
    double mass[2];
    const double *vscale = nullptr;   // NVT: thermostat scaling of the mobile velocities before the kick
    int ke_mobile = 0;                // kinetic energy of the mobile atoms only
};

__global__ void __launch_bounds__(TILE) k_md_kick_drift(const Tile *tiles, Seg *segs, MdIO io)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    if (io.fixed && io.fixed[i]) return;
    const double a = 0.5 * io.dt * ACC_UNIT / io.mass[S.type[i]];
    const double sc = io.vscale ? *io.vscale : 1.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double v = sc * io.v[d * S.n + i] + a * io.F[d * S.n + i];
        io.v[d * S.n + i] = v;
        io.x[d * S.n + i] += io.dt * v;
    }
}

// second half kick and the tile's kinetic energy
__global__ void __launch_bounds__(TILE) k_md_kick(const Tile *tiles, Seg *segs, MdIO io)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[4];
    const int i = T.row0 + threadIdx.x;
    double ke = 0.0;
    if (i < S.n) {
        const double m = io.mass[S.type[i]];
        const bool mob = !(io.fixed && io.fixed[i]);
        const double a = 0.5 * io.dt * ACC_UNIT / m;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            double v = io.v[d * S.n + i];
            if (mob) {
                v += a * io.F[d * S.n + i];
                io.v[d * S.n + i] = v;
            }
            if (mob || !io.ke_mobile) ke += 0.5 * m * v * v / ACC_UNIT;
        }
    }
    double v1[1] = {ke};
    tile_partials<1>(S, T.row0 / TILE, v1, lds);
}

// kinetic and potential energy of the step
__global__ void k_fin_ke(const int *seg_ids, Seg *segs, double *ke_out)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[4];
    double tot[1];
    seg_total<1>(S, lds, tot);
    if (threadIdx.x == 0) {
        ke_out[0] = tot[0];
        ke_out[1] = S.sst->energy;
    }
}

// ---------------------------------------------------------------------------
// NVT: Nose-Hoover chain of M thermostats on the mobile atoms.  With K their
// kinetic energy and Nf their degrees of freedom,
//   m dv/dt = F - m vxi_1 v,   Q_1 dvxi_1/dt = 2K - Nf kT - Q_1 vxi_1 vxi_2,
//   Q_k dvxi_k/dt = Q_{k-1} vxi_{k-1}^2 - kT - Q_k vxi_k vxi_{k+1},  dxi_k/dt = vxi_k,
// Q_1 = Nf kT tau^2, Q_k = kT tau^2; conserved: E_pot + K + sum Q_k vxi_k^2/2
// + Nf kT xi_1 + kT sum_{k>1} xi_k.  A step is a thermostat half step, velocity
// Verlet and a thermostat half step; the half step propagates the chain
// velocities from the last member to the first, scales the particle
// velocities by exp(-vxi_1 dt/2), advances the xi, and propagates the chain
// back up (the split flows are exact, so the step is time reversible).
// ---------------------------------------------------------------------------
constexpr int NHC_MAX = 8;
struct NhcCfg {
    int M;
    double dt, kT, Nf;
    double Qm[NHC_MAX];
};

__device__ double nhc_g(const NhcCfg &c, int k, double K, const double *vxi)
{
    return k == 0 ? (2.0 * K - c.Nf * c.kT) / c.Qm[0] : (c.Qm[k - 1] * vxi[k - 1] * vxi[k - 1] - c.kT) / c.Qm[k];
}

// one thermostat half step (length dt/2); K is scaled with the velocities,
// the returned factor applies to the mobile velocities
__device__ double nhc_half(const NhcCfg &c, double &K, double *xi, double *vxi)
{
    const double h = 0.5 * c.dt;
    const int M = c.M;
    vxi[M - 1] += 0.5 * h * nhc_g(c, M - 1, K, vxi);
    for (int k = M - 2; k >= 0; k--) {
        const double damp = exp(-0.25 * h * vxi[k + 1]);
        vxi[k] = (vxi[k] * damp + 0.5 * h * nhc_g(c, k, K, vxi)) * damp;
    }
    const double sc = exp(-h * vxi[0]);
    K *= sc * sc;
    for (int k = 0; k < M; k++) xi[k] += h * vxi[k];
    for (int k = 0; k < M - 1; k++) {
        const double damp = exp(-0.25 * h * vxi[k + 1]);
        vxi[k] = (vxi[k] * damp + 0.5 * h * nhc_g(c, k, K, vxi)) * damp;
    }
    vxi[M - 1] += 0.5 * h * nhc_g(c, M - 1, K, vxi);
    return sc;
}

// One thread.  ke[0] holds K after the step's second half kick (or of the
// initial velocities).  mode 0: start (first half step of the next step only);
// 1: end of a step (second half step) and the next step's first half step;
// 2: end of the last step; 3: report only.  Writes ke[2] = the velocity scale
// still to apply (by the next kick-drift, or by k_md_scale after the last
// step), ke[3] = K of the step's final velocities, ke[4] = the chain's energy.
__global__ void k_nhc(double *ke, double *chain, NhcCfg c, int mode)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double *xi = chain, *vxi = chain + c.M;
    double K = ke[0], scale = 1.0;
    if (mode == 1 || mode == 2) scale = nhc_half(c, K, xi, vxi);
    double eth = c.Nf * c.kT * xi[0];
    for (int k = 0; k < c.M; k++) eth += 0.5 * c.Qm[k] * vxi[k] * vxi[k] + (k > 0 ? c.kT * xi[k] : 0.0);
    ke[3] = K;
    ke[4] = eth;
    if (mode == 0 || mode == 1) scale *= nhc_half(c, K, xi, vxi);
    ke[2] = scale;
}

// apply the pending thermostat scale to the mobile velocities
__global__ void __launch_bounds__(TILE) k_md_scale(const Tile *tiles, Seg *segs, MdIO io)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n || (io.fixed && io.fixed[i])) return;
    const double sc = *io.vscale;
#pragma unroll
    for (int d = 0; d < 3; d++) io.v[d * S.n + i] *= sc;
}

// number of fixed atoms (tile partials)
__global__ void __launch_bounds__(TILE) k_count_fixed(const Tile *tiles, Seg *segs, const uint8_t *fixed)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[4];
    const int i = T.row0 + threadIdx.x;
    double v[1] = {(i < S.n && fixed && fixed[i]) ? 1.0 : 0.0};
    tile_partials<1>(S, T.row0 / TILE, v, lds);
}

// ---------------------------------------------------------------------------
// Structure relaxation by FIRE (Bitzek et al., Phys. Rev. Lett. 97, 170201,
// 2006): velocity-Verlet steps whose velocities are mixed towards the force
// direction, v <- cv v + cf F, between steps (cv = 1 - alpha, cf = alpha
// |v| / |F|; both 0 stop the system after an uphill step).  The host holds
// the FIRE state (dt, alpha, the count of downhill steps) and reads the four
// reductions of each step: P = F.v, |v|^2, |F|^2 and max_i |F_i|^2 over the
// mobile atoms.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(TILE) k_fire_kick_drift(const Tile *tiles, Seg *segs, MdIO io, double cv,
                                                          double cf)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    if (io.fixed && io.fixed[i]) return;
    const double a = 0.5 * io.dt * ACC_UNIT / io.mass[S.type[i]];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double f = io.F[d * S.n + i];
        double v = cv * io.v[d * S.n + i] + cf * f;
        v += a * f;
        io.v[d * S.n + i] = v;
        io.x[d * S.n + i] += io.dt * v;
    }
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// max over the block (result valid in thread 0)
__device__ __forceinline__ double block_max(double v, double *lds /* 4 */)
{
    const double m = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    const double r = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
    __syncthreads();
    return r;
}

// second half kick (skipped with dt = 0) and the tile's FIRE reductions:
// partials 0..2 = P, |v|^2, |F|^2 (sums), 3 = max |F_i|^2
__global__ void __launch_bounds__(TILE) k_fire_kick(const Tile *tiles, Seg *segs, MdIO io)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    __shared__ double lds[12];
    __shared__ double ldm[4];
    const int i = T.row0 + threadIdx.x;
    double r[3] = {0.0, 0.0, 0.0}, f2 = 0.0;
    if (i < S.n && !(io.fixed && io.fixed[i])) {
        const double a = 0.5 * io.dt * ACC_UNIT / io.mass[S.type[i]];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double f = io.F[d * S.n + i];
            double v = io.v[d * S.n + i];
            if (io.dt != 0.0) {
                v += a * f;
                io.v[d * S.n + i] = v;
            }
            r[0] += f * v;
            r[1] += v * v;
            f2 += f * f;
        }
        r[2] = f2;
    }
    tile_partials<3>(S, T.row0 / TILE, r, lds);
    const double m = block_max(f2, ldm);
    if (threadIdx.x == 0) S.part[(size_t)3 * S.ntile + T.row0 / TILE] = m;
}

// out[0..3] = P, |v|^2, |F|^2, max |F_i|^2; out[4] = potential energy;
// out[5] = the segment's status word
__global__ void k_fire_fin(const int *seg_ids, Seg *segs, double *out)
{
    const Seg &S = segs[seg_ids[blockIdx.x]];
    __shared__ double lds[12];
    __shared__ double ldm[4];
    double tot[3];
    seg_total<3>(S, lds, tot);
    double m = 0.0;
    for (int t = threadIdx.x; t < S.ntile; t += TILE) m = fmax(m, S.part[(size_t)3 * S.ntile + t]);
    m = block_max(m, ldm);
    if (threadIdx.x == 0) {
        out[0] = tot[0];
        out[1] = tot[1];
        out[2] = tot[2];
        out[3] = m;
        out[4] = S.sst->energy;
        out[5] = (double)S.sst->status;
    }
}

} // namespace ctbop
