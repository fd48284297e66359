// Observables of the cavity beyond the wall heat flux: velocity profiles on
// the symmetry plane, from which the peak velocities of Table 1 of
// arXiv:1710.04751 are taken.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lbm_step.hpp"

namespace lbm {

namespace kern {

// Velocity along x and z of one cell, FP64, from the stored post-collision
// state: the collision conserves rho and adds F to the momentum, so
// u = (sum f~ e - F/2) / rho with F = g beta (T - T0) z-hat (eq. 3).  With a
// source the stored scalar sum exceeds T by R/2 (eq. 25); the caller folds
// that into T_ref.
template <typename S, int QT>
__device__ void cell_velocity(const S* __restrict__ F, const S* __restrict__ G, PopLay pl,
                              int64_t c, double gbeta, double T_ref, double* ux, double* uz) {
    double d[15];
#pragma unroll
    for (int a = 0; a < 15; ++a) d[a] = Store<S>::template ld<double>(F + pop_at(pl, a, c));
    double T = 0;
#pragma unroll
    for (int a = 0; a < QT; ++a) T += Store<S>::template ld<double>(G + pop_at(pl, a, c));
    const Raw15<double> r = raw15(d);
    const double rh = 1.0 + r.m0;
    *ux = r.x / rh;
    *uz = (r.z - 0.5 * gbeta * (T - T_ref)) / rh;
}

// Centreline profiles on y = L/2: thread t < nz gives -u_x/u0 at height t on
// x = L/2, thread t < nx gives u_z/u0 at x = t on z = L/2; an even count of
// cells across a line averages the two middle cells.
template <typename S, int QT>
__global__ void k_centerlines(const S* __restrict__ F, const S* __restrict__ G, PopLay pl,
                              Geom g, double gbeta, double T_ref, double inv_u0, double* u_line,
                              double* w_line) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int y0 = (g.ny - 1) / 2, y1 = g.ny / 2;
    if (t < g.nz) {
        const int x0 = (g.nx - 1) / 2, x1 = g.nx / 2;
        double acc = 0;
        int n = 0;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                double ux, uz;
                cell_velocity<S, QT>(F, G, pl, ((int64_t)t * g.ny + y) * g.nx + x, gbeta, T_ref,
                                     &ux, &uz);
                acc -= ux;
                ++n;
            }
        u_line[t] = acc / n * inv_u0;
    }
    if (t < g.nx) {
        const int z0 = (g.nz - 1) / 2, z1 = g.nz / 2;
        double acc = 0;
        int n = 0;
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) {
                double ux, uz;
                cell_velocity<S, QT>(F, G, pl, ((int64_t)z * g.ny + y) * g.nx + t, gbeta, T_ref,
                                     &ux, &uz);
                acc += uz;
                ++n;
            }
        w_line[t] = acc / n * inv_u0;
    }
}

template <typename S, int QT>
hipError_t centerlines_impl(const Geom& g, PopLay pl, StateBuf st, double* u_line,
                            double* w_line, const Coefs& c, double u0, hipStream_t s) {
    const int n = std::max(g.nx, g.nz);
    hipLaunchKernelGGL((k_centerlines<S, QT>), dim3((n + 255) / 256), dim3(256), 0, s,
                       (const S*)st.F, (const S*)st.G, pl, g, c.gbeta, c.T_ref + 0.5 * c.src, 1.0 / u0, u_line,
                       w_line);
    return hipGetLastError();
}

// Projection of (ux, uy, uz, T) onto the symmetries of the cavity (Sec. 3):
// the mirror y -> ny-1-y (uy changes sign) and the half turn about the y
// axis through the centre, (x, z) -> (nx-1-x, nz-1-z) (ux, uz and T - T0
// change sign).  One thread per orbit of the four-element group: it reads
// the four images, averages them with their signs and writes all four back,
// so orbits never overlap and the update is in place.
__global__ void k_symmetrize(Geom g, float* ux, float* uy, float* uz, float* T, double T0) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int x = (int)(c % g.nx);
    const int y = (int)((c / g.nx) % g.ny);
    const int z = (int)(c / ((int64_t)g.nx * g.ny));
    const int xm = g.nx - 1 - x, ym = g.ny - 1 - y, zm = g.nz - 1 - z;
    if (y > ym || z > zm || (z == zm && x > xm)) return;  // not the orbit's representative
    const int64_t id = c;
    const int64_t mir = ((int64_t)z * g.ny + ym) * g.nx + x;
    const int64_t rot = ((int64_t)zm * g.ny + y) * g.nx + xm;
    const int64_t mr = ((int64_t)zm * g.ny + ym) * g.nx + xm;
    // sign of each field under (identity, mirror, rotation, mirror-rotation)
    if (ux) {
        const double a = 0.25 * ((double)ux[id] + ux[mir] - ux[rot] - ux[mr]);
        ux[id] = (float)a, ux[mir] = (float)a, ux[rot] = (float)-a, ux[mr] = (float)-a;
    }
    if (uy) {
        const double a = 0.25 * ((double)uy[id] - uy[mir] + uy[rot] - uy[mr]);
        uy[id] = (float)a, uy[mir] = (float)-a, uy[rot] = (float)a, uy[mr] = (float)-a;
    }
    if (uz) {
        const double a = 0.25 * ((double)uz[id] + uz[mir] - uz[rot] - uz[mr]);
        uz[id] = (float)a, uz[mir] = (float)a, uz[rot] = (float)-a, uz[mr] = (float)-a;
    }
    if (T) {
        const double a = 0.25 * (((double)T[id] - T0) + ((double)T[mir] - T0) -
                                 ((double)T[rot] - T0) - ((double)T[mr] - T0));
        T[id] = (float)(T0 + a), T[mir] = (float)(T0 + a);
        T[rot] = (float)(T0 - a), T[mr] = (float)(T0 - a);
    }
}

}  // namespace kern

hipError_t launch_symmetrize(const Geom& g, float* ux, float* uy, float* uz, float* T, double T0,
                             hipStream_t s) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(kern::k_symmetrize, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s,
                       g, ux, uy, uz, T, T0);
    return hipGetLastError();
}

hipError_t launch_centerlines(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                              double* u_line, double* w_line, const Coefs& c, double u0,
                              hipStream_t s) {
    using namespace kern;
    const bool q7 = qt == 7;
    switch (p) {
        case Prec::FP64:
            return q7 ? centerlines_impl<double, 7>(g, pl, st, u_line, w_line, c, u0, s)
                      : centerlines_impl<double, 15>(g, pl, st, u_line, w_line, c, u0, s);
        case Prec::FP32:
            return q7 ? centerlines_impl<float, 7>(g, pl, st, u_line, w_line, c, u0, s)
                      : centerlines_impl<float, 15>(g, pl, st, u_line, w_line, c, u0, s);
        case Prec::FP32_S16:
            return q7 ? centerlines_impl<_Float16, 7>(g, pl, st, u_line, w_line, c, u0, s)
                      : centerlines_impl<_Float16, 15>(g, pl, st, u_line, w_line, c, u0, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
