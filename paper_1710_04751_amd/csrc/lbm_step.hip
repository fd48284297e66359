// gfx950 kernels of the cascaded double-distribution lattice Boltzmann
// update (arXiv:1710.04751) and the observables around it.
//
// Step kernel: one thread per cell, one pass per time step (A -> B).
//   * pull streaming (eq. 2b, 13b): population a of cell x is read from
//     x - e_a in the previous post-collision state; each value is read once
//     and written once, so the kernel moves (15 + q) values in and out per
//     cell and is bound by HBM bandwidth;
//   * row groups interleaved: each group of consecutive x-rows holds one
//     run per population, x fastest, so a wave reads 64 consecutive cells
//     of one population, shifted by at most one element (coalesced), and
//     the streams of one block lie within a few runs of ~32 KB;
//   * walls (Sec. 3): a link whose source lies outside the box takes the
//     opposite population of the cell itself (half-way bounce-back for the
//     flow; anti-bounce-back -g + 2 w T_wall across the two Dirichlet walls,
//     which take precedence on edges; bounce-back across the adiabatic ones);
//   * T = sum g (eq. 25), F = g beta (T - T0) z (Boussinesq), then the flow
//     collision and the scalar collision with the same step's velocity, all
//     in registers, then non-temporal stores of the post-collision state;
//   * blocks are numbered so that each of the 8 XCDs works on a contiguous
//     range of tiles: neighbouring tiles of a row share the partly-read
//     cache lines of the x-shifted populations in the same L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lbm_dispatch.hpp"
#include "lbm_step.hpp"

namespace lbm {

namespace kern {

// Block number -> tile number, so that XCD k (hardware places block b on XCD
// b mod 8) receives the contiguous tile range [start_k, start_k + count_k).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
    const uint32_t q = nb >> 3, r = nb & 7u, k = b & 7u;
    return k * q + (k < r ? k : r) + (b >> 3);
}

struct CellPos {
    int x, y, z, y0;  // y0: first row of the block's tile
    bool ok;
};

__device__ __forceinline__ CellPos tile_cell(const Geom& g) {
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t per_z = (uint32_t)g.tiles_x * (uint32_t)g.tiles_y;
    const uint32_t tz = t / per_z;
    const uint32_t rem = t - tz * per_z;
    const uint32_t ty = rem / (uint32_t)g.tiles_x;
    const uint32_t tx = rem - ty * (uint32_t)g.tiles_x;
    CellPos c;
    c.x = (int)(tx * blockDim.x + threadIdx.x);
    c.y = (int)(ty * blockDim.y + threadIdx.y);
    c.z = (int)tz;
    c.y0 = (int)(ty * blockDim.y);
    c.ok = c.x < g.nx && c.y < g.ny;
    return c;
}

// Single cavity: one thread per cell, blocks of bx * by cells of one plane.
template <typename R, typename S, int QT, bool HG>
__global__ void __launch_bounds__(1024)
k_step(const S* __restrict__ in, S* __restrict__ out, Geom g, KCoef<R> k) {
    const CellPos p = tile_cell(g);
    if (!p.ok) return;
    update_cell<R, S, QT, HG>(in, out, p.x, p.y, p.z, p.y0, g.nx, g.ny, g.nz, g.gs, k, k.seed);
}

template <typename R, typename S, int QT, bool HG>
hipError_t step_impl(const Geom& g, StateBuf in, StateBuf out, const Coefs& c, hipStream_t s) {
    const KCoef<R> k = make_kcoef<R>(c, QT);
    const dim3 block(g.bx, g.by, 1);
    const dim3 grid((unsigned)((int64_t)g.tiles_x * g.tiles_y * g.nz), 1, 1);
    hipLaunchKernelGGL((k_step<R, S, QT, HG>), grid, block, 0, s, (const S*)in.F, (S*)out.F, g,
                       k);
    return hipGetLastError();
}

}  // namespace kern
using namespace kern;

hipError_t launch_step(Prec p, int qt, bool general, const Geom& g, StateBuf in,
                       StateBuf out, const Coefs& c, hipStream_t s) {
    if (general) {
        LBM_DISPATCH_PQ(p, qt, return (step_impl<R, S, Q, true>(g, in, out, c, s)));
    } else {
        LBM_DISPATCH_PQ(p, qt, return (step_impl<R, S, Q, false>(g, in, out, c, s)));
    }
}

const char* step_kernel_name(Prec p, int qt, bool general) {
    static const char* names[3][2][2] = {
        {{"lbm::kern::k_step<double, double, 7, false>", "lbm::kern::k_step<double, double, 7, true>"},
         {"lbm::kern::k_step<double, double, 15, false>", "lbm::kern::k_step<double, double, 15, true>"}},
        {{"lbm::kern::k_step<float, float, 7, false>", "lbm::kern::k_step<float, float, 7, true>"},
         {"lbm::kern::k_step<float, float, 15, false>", "lbm::kern::k_step<float, float, 15, true>"}},
        {{"lbm::kern::k_step<float, _Float16, 7, false>", "lbm::kern::k_step<float, _Float16, 7, true>"},
         {"lbm::kern::k_step<float, _Float16, 15, false>", "lbm::kern::k_step<float, _Float16, 15, true>"}}};
    return names[(int)p][qt == 15][general ? 1 : 0];
}

}  // namespace lbm
