// gfx950 kernels around the cascaded double-distribution lattice Boltzmann
// update (arXiv:1710.04751): initialisation, state I/O and the observables
// (macroscopic fields, wall Nusselt numbers, steady-state residual), and the
// plain copy used as the bandwidth reference.  The per-step update itself
// lives in lbm_step.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lbm_dispatch.hpp"
#include "lbm_step.hpp"

namespace lbm {

namespace kern {

// ---------------------------------------------------------------------------
// Initialisation and state I/O
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint4* __restrict__ p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

// Staggered sums of an initial state: sum (-1)^x ux, sum (-1)^y uy,
// sum (-1)^z uz and sum (-1)^z (T - T_ref) (FP64, added into sums[0..3]).
__global__ void __launch_bounds__(256) k_stagger_sums(const float* ux, const float* uy,
                                                      const float* uz, const float* T,
                                                      double T_ref, Geom g, double* sums) {
    __shared__ double red[4][256];
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < ncell) {
        const int x = (int)(c % g.nx);
        const int y = (int)((c / g.nx) % g.ny);
        const int z = (int)(c / ((int64_t)g.nx * g.ny));
        if (ux) a[0] = (x & 1) ? -(double)ux[c] : (double)ux[c];
        if (uy) a[1] = (y & 1) ? -(double)uy[c] : (double)uy[c];
        if (uz) a[2] = (z & 1) ? -(double)uz[c] : (double)uz[c];
        const double t = (T ? (double)T[c] : 0.0) - T_ref;
        a[3] = (z & 1) ? -t : t;
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) atomicAdd(&sums[k], red[k][0]);
}

// Equilibrium populations of (rho = 1, u, T), with the staggered part of
// the velocity set as a start from rest has it.  Pull streaming moves every
// population that carries x-momentum to a cell of the other x parity,
// bounce-back returns it with the sign of e_x reversed, and collision
// conserves momentum, so Qx = sum (-1)^x j_x only changes sign from step to
// step (likewise Qy); along z the collision adds S = sum (-1)^z F_z, so Qz
// alternates about S/2.  Rest has Qx = Qy = 0 and Qz at S/2 = 0; any other
// staggered momentum would persist as a period-2 oscillation.  So ux and uy
// lose their staggered sums and uz gets sum (-1)^z uz = S/2 (uniform
// (-1)^x, (-1)^y, (-1)^z corrections).
template <typename R, typename S, int QT>
__global__ void k_init_macros(S* __restrict__ F, S* __restrict__ G, PopLay pl, Geom geo,
                              const float* ux, const float* uy, const float* uz, const float* T,
                              const double* __restrict__ stag, double gbeta, R cs2, R src) {
    const int64_t ncell = (int64_t)geo.nx * geo.ny * geo.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int x = (int)(c % geo.nx);
    const int y = (int)((c / geo.nx) % geo.ny);
    const int z = (int)(c / ((int64_t)geo.nx * geo.ny));
    const double inv = 1.0 / (double)ncell;
    const double cx = stag[0] * inv, cy = stag[1] * inv;
    const double cz = (stag[2] - 0.5 * gbeta * stag[3]) * inv;
    const R u = ux ? (R)((double)ux[c] - ((x & 1) ? -cx : cx)) : R(0);
    const R v = uy ? (R)((double)uy[c] - ((y & 1) ? -cy : cy)) : R(0);
    const R w = (R)((uz ? (double)uz[c] : 0.0) - ((z & 1) ? -cz : cz));
    // scalar equilibrium at T - R/2, so that the first step sees T (eq. 25)
    const R t = (T ? (R)T[c] : R(0)) - R(0.5) * src;
    R d[15];
    flow_equilibrium<R>(R(0), u, v, w, d);
#pragma unroll
    for (int a = 0; a < 15; ++a) F[pop_at(pl, a, c)] = (S)d[a];
    R g[QT];
    if constexpr (QT == 7)
        thermal_equilibrium7<R>(t, u, v, w, cs2, g);
    else
        thermal_equilibrium15<R>(t, u, v, w, cs2, g);
#pragma unroll
    for (int a = 0; a < QT; ++a) G[pop_at(pl, a, c)] = (S)g[a];
}

// Rest state with a scalar source: flow at rest (deviations 0) and the
// scalar equilibrium at T = -R/2 with u = 0, so that the first step sees
// T = sum gbar + R/2 = 0 (eq. 25).
template <typename R, typename S, int QT>
__global__ void k_init_rest_source(S* __restrict__ F, S* __restrict__ G, PopLay pl,
                                   int64_t ncell, R cs2, R src) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
#pragma unroll
    for (int a = 0; a < 15; ++a) F[pop_at(pl, a, c)] = (S)0;
    R g[QT];
    if constexpr (QT == 7)
        thermal_equilibrium7<R>(R(-0.5) * src, R(0), R(0), R(0), cs2, g);
    else
        thermal_equilibrium15<R>(R(-0.5) * src, R(0), R(0), R(0), cs2, g);
#pragma unroll
    for (int a = 0; a < QT; ++a) G[pop_at(pl, a, c)] = (S)g[a];
}

// Macroscopic fields from the stored post-collision populations: the
// collision conserves rho, adds F to the momentum and R to the scalar sum,
// so u = (sum f~ e - F/2) / rho and T = sum g~ - R/2 (eq. 25).
template <typename R, typename S, int QT, typename O>
__global__ void k_macros(const S* __restrict__ F, const S* __restrict__ G, PopLay pl,
                         int64_t ncell, O* rho, O* ux, O* uy, O* uz, O* To, R gbeta, R T_ref,
                         R src) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    R d[15];
#pragma unroll
    for (int a = 0; a < 15; ++a) d[a] = Store<S>::template ld<R>(F + pop_at(pl, a, c));
    R T = 0;
#pragma unroll
    for (int a = 0; a < QT; ++a) T += Store<S>::template ld<R>(G + pop_at(pl, a, c));
    T -= R(0.5) * src;
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
__global__ void k_get_pops(const S* __restrict__ F, const S* __restrict__ G, PopLay pl,
                           int64_t ncell, double* Fo, double* Go) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    if (Fo)
#pragma unroll
        for (int a = 0; a < 15; ++a)
            Fo[a * ncell + c] = flow_weight(a) + Store<S>::template ld<double>(F + pop_at(pl, a, c));
    if (Go)
#pragma unroll
        for (int a = 0; a < QT; ++a) Go[a * ncell + c] = Store<S>::template ld<double>(G + pop_at(pl, a, c));
}

template <typename S, int QT>
__global__ void k_set_pops(S* __restrict__ F, S* __restrict__ G, PopLay pl, int64_t ncell,
                           const double* Fi, const double* Gi) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
#pragma unroll
    for (int a = 0; a < 15; ++a) F[pop_at(pl, a, c)] = (S)(Fi[a * ncell + c] - flow_weight(a));
#pragma unroll
    for (int a = 0; a < QT; ++a) G[pop_at(pl, a, c)] = (S)Gi[a * ncell + c];
}

template <typename S, int QT>
__global__ void k_gather_cells(const S* __restrict__ F, const S* __restrict__ G, PopLay pl,
                               const int64_t* cells, int64_t n, double* Fo, double* Go) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = cells[i];
    if (Fo)
#pragma unroll
        for (int a = 0; a < 15; ++a)
            Fo[i * 15 + a] = flow_weight(a) + Store<S>::template ld<double>(F + pop_at(pl, a, c));
    if (Go)
#pragma unroll
        for (int a = 0; a < QT; ++a) Go[i * QT + a] = Store<S>::template ld<double>(G + pop_at(pl, a, c));
}

// ---------------------------------------------------------------------------
// Nusselt number (FP64)
// ---------------------------------------------------------------------------
// Local wall heat flux from the links crossing the two Dirichlet walls:
// hot wall (x = -1/2): sum over links entering the fluid (e_x > 0) of
// 2 (w_a T_hot - G_opp(a)(0, y, z)); cold wall (x = nx - 1/2): sum over links
// leaving it (e_x > 0) of 2 (G_a(nx-1, y, z) - w_a T_cold).
template <typename S, int QT>
__global__ void k_nusselt_local(const S* __restrict__ G, PopLay pl, Geom g, double* nu_hot,
                                double* nu_cold, double T_hot, double T_cold, double wf,
                                double wc, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)g.ny * g.nz;
    if (i >= n) return;
    const int64_t row = i * g.nx;  // cell (0, y, z) with i = z*ny + y
    const int64_t hot = row, cold = row + g.nx - 1;
    auto ld = [&](int a, int64_t c) { return Store<S>::template ld<double>(G + pop_at(pl, a, c)); };
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
k_residual(const S* __restrict__ G, PopLay pl, int64_t ncell, Snap* __restrict__ snap,
           int compare, unsigned long long* max_bits, unsigned int* bad) {
    __shared__ double s_red[4];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dev = 0;
    if (c < ncell) {
        double T = 0;
#pragma unroll
        for (int a = 0; a < QT; ++a) T += Store<S>::template ld<double>(G + pop_at(pl, a, c));
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

}  // namespace kern
using namespace kern;

int value_bytes(Prec p) { return p == Prec::FP64 ? 8 : (p == Prec::FP32 ? 4 : 2); }

hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 65536);
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (uint4*)ptr, n16);
    return hipGetLastError();
}

hipError_t launch_init_rest(Prec p, int qt, const Geom& g, PopLay pl, void* state,
                            size_t state_bytes, StateBuf st, const Coefs& c, hipStream_t s) {
    hipError_t e = launch_fill_zero(state, state_bytes, s);
    if (e != hipSuccess || c.src == 0.0) return e;
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        hipLaunchKernelGGL((k_init_rest_source<R, S, Q>), dim3(blocks_for(ncell, 256)), dim3(256),
                           0, s, (S*)st.F, (S*)st.G, pl, ncell, (R)c.cs2, (R)c.src);
        return hipGetLastError();
    });
}

hipError_t launch_init_macros(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                              const float* ux, const float* uy, const float* uz, const float* T,
                              double* stag, const Coefs& c, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    hipError_t e = launch_fill_zero(stag, 32, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stagger_sums, dim3(blocks_for(ncell, 256)), dim3(256), 0, s, ux, uy, uz,
                       T, c.T_ref, g, stag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    LBM_DISPATCH_PQ(p, qt, {
        hipLaunchKernelGGL((k_init_macros<R, S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (S*)st.F, (S*)st.G, pl, g, ux, uy, uz, T, (const double*)stag,
                           c.gbeta, (R)c.cs2, (R)c.src);
        return hipGetLastError();
    });
}

hipError_t launch_macros(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, void* rho,
                         void* ux, void* uy, void* uz, void* T, bool fp64, const Coefs& c,
                         hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        if (fp64) {
            hipLaunchKernelGGL((k_macros<R, S, Q, double>), dim3(blocks_for(ncell, 256)), dim3(256),
                               0, s, (const S*)st.F, (const S*)st.G, pl, ncell, (double*)rho,
                               (double*)ux, (double*)uy, (double*)uz, (double*)T, (R)c.gbeta,
                               (R)c.T_ref, (R)c.src);
        } else {
            hipLaunchKernelGGL((k_macros<R, S, Q, float>), dim3(blocks_for(ncell, 256)), dim3(256),
                               0, s, (const S*)st.F, (const S*)st.G, pl, ncell, (float*)rho,
                               (float*)ux, (float*)uy, (float*)uz, (float*)T, (R)c.gbeta,
                               (R)c.T_ref, (R)c.src);
        }
        return hipGetLastError();
    });
}

hipError_t launch_nusselt(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                          double* local_hot, double* local_cold, double* result,
                          const Coefs& c, hipStream_t s) {
    const int64_t n = (int64_t)g.ny * g.nz;
    const double wf = qt == 7 ? c.cs2 / 2 : (c.cs2 - c.cs2 * c.cs2) / 2;
    const double wc = qt == 7 ? 0.0 : c.cs2 * c.cs2 / 8;
    const double scale = (double)g.nx / (c.alpha * (c.T_hot - c.T_cold));
    LBM_DISPATCH_PQ(p, qt, {
        hipLaunchKernelGGL((k_nusselt_local<S, Q>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const S*)st.G, pl, g, local_hot, local_cold, c.T_hot, c.T_cold, wf, wc,
                           scale);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_nusselt_reduce, dim3(1), dim3(1024), 0, s, local_hot, local_cold, g.ny,
                           g.nz, result);
        return hipGetLastError();
    });
}

hipError_t launch_residual(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, void* snapshot,
                           bool compare, unsigned long long* max_bits, unsigned int* bad_flag,
                           hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        using Snap = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
        hipLaunchKernelGGL((k_residual<S, Q, Snap>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (const S*)st.G, pl, ncell, (Snap*)snapshot, compare ? 1 : 0, max_bits,
                           bad_flag);
        return hipGetLastError();
    });
}

hipError_t launch_get_pops(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, double* F,
                           double* G, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_get_pops<S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (const S*)st.F, (const S*)st.G, pl, ncell, F, G);
        return hipGetLastError();
    });
}

hipError_t launch_set_pops(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                           const double* F, const double* G, hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_set_pops<S, Q>), dim3(blocks_for(ncell, 256)), dim3(256), 0, s,
                           (S*)st.F, (S*)st.G, pl, ncell, F, G);
        return hipGetLastError();
    });
}

hipError_t launch_gather_cells(Prec p, int qt, int64_t ncell, PopLay pl, StateBuf st,
                               const int64_t* cells, int64_t n, double* F, double* G,
                               hipStream_t s) {
    (void)ncell;
    if (n == 0) return hipSuccess;
    LBM_DISPATCH_PQ(p, qt, {
        (void)sizeof(R);
        hipLaunchKernelGGL((k_gather_cells<S, Q>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const S*)st.F, (const S*)st.G, pl, cells, n, F, G);
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
