// k_md.h -- velocity-Verlet NVE integration (user atom order).
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
};

__global__ void __launch_bounds__(TILE) k_md_kick_drift(const Tile *tiles, Seg *segs, MdIO io)
{
    const Tile T = my_tile(tiles);
    const Seg &S = segs[T.seg];
    const int i = T.row0 + threadIdx.x;
    if (i >= S.n) return;
    if (io.fixed && io.fixed[i]) return;
    const double a = 0.5 * io.dt * ACC_UNIT / io.mass[S.type[i]];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double v = io.v[d * S.n + i] + a * io.F[d * S.n + i];
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
            ke += 0.5 * m * v * v / ACC_UNIT;
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

} // namespace ctbop
