// gfx950 kernels of the cascaded double-distribution lattice Boltzmann
// update (arXiv:1710.04751) and the observables around it.
//
// Step kernel: one thread per cell, one pass per time step (A -> B).
//   * pull streaming (eq. 2b, 13b): population a of cell x is read from
//     x - e_a in the previous post-collision state; each value is read once
//     and written once, so the kernel moves (15 + q) values in and out per
//     cell and is bound by HBM bandwidth;
//   * SoA layout, x fastest: a wave reads 64 consecutive cells of one
//     population, shifted by at most one element, so loads are coalesced;
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
    int x, y, z;
    uint32_t cell;
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
    c.ok = c.x < g.nx && c.y < g.ny;
    c.cell = ((uint32_t)c.z * (uint32_t)g.ny + (uint32_t)c.y) * (uint32_t)g.nx + (uint32_t)c.x;
    return c;
}

// Single cavity: one thread per cell, blocks of bx * by cells of one plane.
template <typename R, typename S, int QT, bool HG>
__global__ void __launch_bounds__(1024)
k_step(const S* __restrict__ Fi, const S* __restrict__ Gi, S* __restrict__ Fo,
       S* __restrict__ Go, int64_t ps, Geom g, KCoef<R> k) {
    const CellPos p = tile_cell(g);
    if (!p.ok) return;
    update_cell<R, S, QT, HG>(Fi, Gi, Fo, Go, ps, p.cell, p.x, p.y, p.z, g.nx, g.ny, g.nz, k);
}

// ---------------------------------------------------------------------------
// Initialisation and state I/O
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint4* __restrict__ p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

template <typename R, typename S, int QT>
__global__ void k_init_macros(S* __restrict__ F, S* __restrict__ G, int64_t ps, int64_t ncell,
                              const float* ux, const float* uy, const float* uz, const float* T,
                              R cs2) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const R u = ux ? (R)ux[c] : R(0), v = uy ? (R)uy[c] : R(0), w = uz ? (R)uz[c] : R(0);
    const R t = T ? (R)T[c] : R(0);
    R d[15];
    flow_equilibrium<R>(R(0), u, v, w, d);
#pragma unroll
    for (int a = 0; a < 15; ++a) F[a * ps + c] = (S)d[a];
    R g[QT];
    if constexpr (QT == 7)
        thermal_equilibrium7<R>(t, u, v, w, cs2, g);
    else
        thermal_equilibrium15<R>(t, u, v, w, cs2, g);
#pragma unroll
    for (int a = 0; a < QT; ++a) G[a * ps + c] = (S)g[a];
}

// Macroscopic fields from the stored post-collision populations: the
// collision conserves rho and T and adds F to the momentum, so
// u = (sum f~ e - F/2) / rho.
template <typename R, typename S, int QT, typename O>
__global__ void k_macros(const S* __restrict__ F, const S* __restrict__ G, int64_t ps,
                         int64_t ncell, O* rho, O* ux, O* uy, O* uz, O* To, R gbeta, R T_ref) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    R d[15];
#pragma unroll
    for (int a = 0; a < 15; ++a) d[a] = Store<S>::template ld<R>(F + a * ps + c);
    R T = 0;
#pragma unroll
    for (int a = 0; a < QT; ++a) T += Store<S>::template ld<R>(G + a * ps + c);
    const Raw15<R> r = raw15(d);
    const R rh = R(1) + r.m0;
    const R Fz = gbeta * (T - T_ref);
    if (rho) rho[c] = (O)rh;
    if (ux) ux[c] = (O)(r.x / rh);
    if (uy) uy[c] = (O)(r.y / rh);
    if (uz) uz[c] = (O)((r.z - R(0.5) * Fz) / rh);
    if (To) To[c] = (O)T;
}

template <typename S, int QT>
__global__ void k_get_pops(const S* __restrict__ F, const S* __restrict__ G, int64_t ps,
                           int64_t ncell, double* Fo, double* Go) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    if (Fo)
#pragma unroll
        for (int a = 0; a < 15; ++a)
            Fo[a * ncell + c] = flow_weight(a) + Store<S>::template ld<double>(F + a * ps + c);
    if (Go)
#pragma unroll
        for (int a = 0; a < QT; ++a) Go[a * ncell + c] = Store<S>::template ld<double>(G + a * ps + c);
}

template <typename S, int QT>
__global__ void k_set_pops(S* __restrict__ F, S* __restrict__ G, int64_t ps, int64_t ncell,
                           const double* Fi, const double* Gi) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
#pragma unroll
    for (int a = 0; a < 15; ++a) F[a * ps + c] = (S)(Fi[a * ncell + c] - flow_weight(a));
#pragma unroll
    for (int a = 0; a < QT; ++a) G[a * ps + c] = (S)Gi[a * ncell + c];
}

template <typename S, int QT>
__global__ void k_gather_cells(const S* __restrict__ F, const S* __restrict__ G, int64_t ps,
                               const int64_t* cells, int64_t n, double* Fo, double* Go) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = cells[i];
    if (Fo)
#pragma unroll
        for (int a = 0; a < 15; ++a)
            Fo[i * 15 + a] = flow_weight(a) + Store<S>::template ld<double>(F + a * ps + c);
    if (Go)
#pragma unroll
        for (int a = 0; a < QT; ++a) Go[i * QT + a] = Store<S>::template ld<double>(G + a * ps + c);
}

// ---------------------------------------------------------------------------
// Nusselt number (FP64)
// ---------------------------------------------------------------------------
// Local wall heat flux from the links crossing the two Dirichlet walls:
// hot wall (x = -1/2): sum over links entering the fluid (e_x > 0) of
// 2 (w_a T_hot - G_opp(a)(0, y, z)); cold wall (x = nx - 1/2): sum over links
// leaving it (e_x > 0) of 2 (G_a(nx-1, y, z) - w_a T_cold).
template <typename S, int QT>
__global__ void k_nusselt_local(const S* __restrict__ G, int64_t ps, Geom g, double* nu_hot,
                                double* nu_cold, double T_hot, double T_cold, double wf,
                                double wc, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)g.ny * g.nz;
    if (i >= n) return;
    const int64_t row = i * g.nx;  // cell (0, y, z) with i = z*ny + y
    const int64_t hot = row, cold = row + g.nx - 1;
    auto ld = [&](int a, int64_t c) { return Store<S>::template ld<double>(G + a * ps + c); };
    double qh = 2.0 * (wf * T_hot - ld(2, hot));
    double qc = 2.0 * (ld(1, cold) - wf * T_cold);
    if (QT == 15) {
        qh += 2.0 * (4.0 * wc * T_hot - (ld(8, hot) + ld(10, hot) + ld(12, hot) + ld(14, hot)));
        qc += 2.0 * ((ld(7, cold) + ld(9, cold) + ld(11, cold) + ld(13, cold)) - 4.0 * wc * T_cold);
    }
    nu_hot[i] = qh * scale;
    nu_cold[i] = qc * scale;
}

// One block: face means, mid-line (y = L/2) means and the extremes of the
// hot-wall mid-line with their z positions.  result[0..7] = lbm_nu fields.
__global__ void __launch_bounds__(1024)
k_nusselt_reduce(const double* __restrict__ nh, const double* __restrict__ nc, int ny, int nz,
                 double* result) {
    __shared__ double s_h[1024], s_c[1024], s_mh[1024], s_mc[1024];
    __shared__ double s_max[1024], s_min[1024];
    __shared__ int s_imax[1024], s_imin[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int64_t n = (int64_t)ny * nz;
    double sh = 0, sc = 0;
    for (int64_t i = t; i < n; i += nt) {
        sh += nh[i];
        sc += nc[i];
    }
    double mh = 0, mc = 0, vmax = -INFINITY, vmin = INFINITY;
    int imax = 0, imin = 0;
    const int y0 = (ny % 2) ? ny / 2 : ny / 2 - 1, y1 = ny / 2;
    for (int z = t; z < nz; z += nt) {
        const double lh = 0.5 * (nh[(int64_t)z * ny + y0] + nh[(int64_t)z * ny + y1]);
        const double lc = 0.5 * (nc[(int64_t)z * ny + y0] + nc[(int64_t)z * ny + y1]);
        mh += lh;
        mc += lc;
        if (lh > vmax) vmax = lh, imax = z;
        if (lh < vmin) vmin = lh, imin = z;
    }
    s_h[t] = sh;
    s_c[t] = sc;
    s_mh[t] = mh;
    s_mc[t] = mc;
    s_max[t] = vmax;
    s_min[t] = vmin;
    s_imax[t] = imax;
    s_imin[t] = imin;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (t < w) {
            s_h[t] += s_h[t + w];
            s_c[t] += s_c[t + w];
            s_mh[t] += s_mh[t + w];
            s_mc[t] += s_mc[t + w];
            if (s_max[t + w] > s_max[t] || (s_max[t + w] == s_max[t] && s_imax[t + w] < s_imax[t]))
                s_max[t] = s_max[t + w], s_imax[t] = s_imax[t + w];
            if (s_min[t + w] < s_min[t] || (s_min[t + w] == s_min[t] && s_imin[t + w] < s_imin[t]))
                s_min[t] = s_min[t + w], s_imin[t] = s_imin[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        result[0] = s_h[0] / (double)n;
        result[1] = s_c[0] / (double)n;
        result[2] = s_mh[0] / (double)nz;
        result[3] = s_mc[0] / (double)nz;
        result[4] = s_max[0];
        result[5] = (s_imax[0] + 0.5) / (double)nz;
        result[6] = s_min[0];
        result[7] = (s_imin[0] + 0.5) / (double)nz;
    }
}

// ---------------------------------------------------------------------------
// Steady-state residual: max |T - T_snapshot| and a NaN/Inf flag
// ---------------------------------------------------------------------------
template <typename S, int QT, typename Snap>
__global__ void __launch_bounds__(256)
k_residual(const S* __restrict__ G, int64_t ps, int64_t ncell, Snap* __restrict__ snap,
           int compare, unsigned long long* max_bits, unsigned int* bad) {
    __shared__ double s_red[4];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dev = 0;
    if (c < ncell) {
        double T = 0;
#pragma unroll
        for (int a = 0; a < QT; ++a) T += Store<S>::template ld<double>(G + a * ps + c);
        const Snap Ts = (Snap)T;
        if (!isfinite(T)) atomicOr(bad, 1u);
        if (compare) dev = fabs((double)Ts - (double)snap[c]);
        snap[c] = Ts;
    }
    for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) s_red[wv] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_red[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, s_red[i]);
        if (m > 0) atomicMax(max_bits, (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

template <typename S>
struct PrecOf;

// ---------------------------------------------------------------------------
// Dispatch helpers
// ---------------------------------------------------------------------------
template <typename R, typename S, int QT, bool HG>
hipError_t step_impl(const Geom& g, int64_t ps, StateBuf in, StateBuf out, const Coefs& c,
                     hipStream_t s) {
    const KCoef<R> k = make_kcoef<R>(c, QT);
    const dim3 block(g.bx, g.by, 1);
    const dim3 grid((unsigned)((int64_t)g.tiles_x * g.tiles_y * g.nz), 1, 1);
    hipLaunchKernelGGL((k_step<R, S, QT, HG>), grid, block, 0, s, (const S*)in.F, (const S*)in.G,
                       (S*)out.F, (S*)out.G, ps, g, k);
    return hipGetLastError();
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace kern
using namespace kern;

int value_bytes(Prec p) { return p == Prec::FP64 ? 8 : (p == Prec::FP32 ? 4 : 2); }

#define LBM_DISPATCH_PQ(p, qt, ...)                                       \
    do {                                                                  \
        if (p == Prec::FP64 && qt == 7) {                                 \
            using R = double; using S = double; constexpr int Q = 7; __VA_ARGS__; \
        } else if (p == Prec::FP64 && qt == 15) {                         \
            using R = double; using S = double; constexpr int Q = 15; __VA_ARGS__; \
        } else if (p == Prec::FP32 && qt == 7) {                          \
            using R = float; using S = float; constexpr int Q = 7; __VA_ARGS__;  \
        } else if (p == Prec::FP32 && qt == 15) {                         \
            using R = float; using S = float; constexpr int Q = 15; __VA_ARGS__; \
        } else if (p == Prec::FP32_S16 && qt == 7) {                      \
            using R = float; using S = _Float16; constexpr int Q = 7; __VA_ARGS__; \
        } else if (p == Prec::FP32_S16 && qt == 15) {                     \
            using R = float; using S = _Float16; constexpr int Q = 15; __VA_ARGS__; \
        } else {                                                          \
            return hipErrorInvalidValue;                                  \
        }                                                                 \
    } while (0)

hipError_t launch_step(Prec p, int qt, bool general, const Geom& g, int64_t ps, StateBuf in,
                       StateBuf out, const Coefs& c, hipStream_t s) {
    if (general) {
        LBM_DISPATCH_PQ(p, qt, return (step_impl<R, S, Q, true>(g, ps, in, out, c, s)));
    } else {
        LBM_DISPATCH_PQ(p, qt, return (step_impl<R, S, Q, false>(g, ps, in, out, c, s)));
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

hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 65536);
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (uint4*)ptr, n16);
    return hipGetLastError();
}

hipError_t launch_init_macros(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st,
                              const float* ux, const float* uy, const float* uz, const float* T,
                              const Coefs& c, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        hipLaunchKernelGGL((k_init_macros<R, S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (S*)st.F, (S*)st.G, ps, ncell, ux, uy, uz, T, (R)c.cs2);
        return hipGetLastError();
    });
}

hipError_t launch_macros(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st, void* rho,
                         void* ux, void* uy, void* uz, void* T, bool fp64, const Coefs& c,
                         hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        if (fp64) {
            hipLaunchKernelGGL((k_macros<R, S, Q, double>), dim3(blocks_for(ncell, 256)), dim3(256),
                               0, s, (const S*)st.F, (const S*)st.G, ps, ncell, (double*)rho,
                               (double*)ux, (double*)uy, (double*)uz, (double*)T, (R)c.gbeta,
                               (R)c.T_ref);
        } else {
            hipLaunchKernelGGL((k_macros<R, S, Q, float>), dim3(blocks_for(ncell, 256)), dim3(256),
                               0, s, (const S*)st.F, (const S*)st.G, ps, ncell, (float*)rho,
                               (float*)ux, (float*)uy, (float*)uz, (float*)T, (R)c.gbeta,
                               (R)c.T_ref);
        }
        return hipGetLastError();
    });
}

hipError_t launch_nusselt(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st,
                          double* local_hot, double* local_cold, double* result,
                          const Coefs& c, hipStream_t s) {
    const int64_t n = (int64_t)g.ny * g.nz;
    const double wf = qt == 7 ? c.cs2 / 2 : (c.cs2 - c.cs2 * c.cs2) / 2;
    const double wc = qt == 7 ? 0.0 : c.cs2 * c.cs2 / 8;
    const double scale = (double)g.nx / (c.alpha * (c.T_hot - c.T_cold));
    LBM_DISPATCH_PQ(p, qt, {
        hipLaunchKernelGGL((k_nusselt_local<S, Q>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const S*)st.G, ps, g, local_hot, local_cold, c.T_hot, c.T_cold, wf, wc,
                           scale);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_nusselt_reduce, dim3(1), dim3(1024), 0, s, local_hot, local_cold, g.ny,
                           g.nz, result);
        return hipGetLastError();
    });
}

hipError_t launch_residual(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st, void* snapshot,
                           bool compare, unsigned long long* max_bits, unsigned int* bad_flag,
                           hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        using Snap = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
        hipLaunchKernelGGL((k_residual<S, Q, Snap>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (const S*)st.G, ps, ncell, (Snap*)snapshot, compare ? 1 : 0, max_bits,
                           bad_flag);
        return hipGetLastError();
    });
}

hipError_t launch_get_pops(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st, double* F,
                           double* G, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_get_pops<S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (const S*)st.F, (const S*)st.G, ps, ncell, F, G);
        return hipGetLastError();
    });
}

hipError_t launch_set_pops(Prec p, int qt, const Geom& g, int64_t ps, StateBuf st,
                           const double* F, const double* G, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_set_pops<S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (S*)st.F, (S*)st.G, ps, ncell, F, G);
        return hipGetLastError();
    });
}

hipError_t launch_gather_cells(Prec p, int qt, int64_t ncell, int64_t ps, StateBuf st,
                               const int64_t* cells, int64_t n, double* F, double* G,
                               hipStream_t s) {
    (void)ncell;
    if (n == 0) return hipSuccess;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_gather_cells<S, Q>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const S*)st.F, (const S*)st.G, ps, cells, n, F, G);
        return hipGetLastError();
    });
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 1u << 20);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

}  // namespace lbm
