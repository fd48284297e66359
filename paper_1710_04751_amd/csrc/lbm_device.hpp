// Device-side lattice algebra for the cascaded central-moment collisions.
//
// Lattices (Sec. 2.2 eq. (5) and Appendix C of arXiv:1710.04751):
//   D3Q15: 0 rest, 1..6 faces (+x,-x,+y,-y,+z,-z), 7..14 corners
//          7 (+,+,+) 8 (-,+,+) 9 (+,-,+) 10 (-,-,+)
//          11 (+,+,-) 12 (-,+,-) 13 (+,-,-) 14 (-,-,-)
//   D3Q7:  0 rest, 1..6 faces.
//
// How the collisions are evaluated.  On D3Q15 the fifteen raw monomial
// moments {1, x, y, z, xy, xz, yz, xx, yy, zz, xyy, xxy, xxz, xyz, xxyy}
// determine the populations: the eight corners are the 2x2x2 Hadamard
// transform of {xxyy, xyy, xxy, xxz, xy, xz, yz, xyz}, each face pair is
// fixed by one first- and one second-order moment, and the rest population
// by mass.  A collision therefore is:
//   raw moments (Hadamard) -> central moments about u (binomial shift) ->
//   relaxation of each central moment toward its equilibrium (Appendix A for
//   the flow, Sec. 2.2 / Appendix C for the scalar) -> raw moments of the
//   result (shift back) -> populations (inverse Hadamard).
// This reaches the same post-collision state as the paper's cascaded kernels
// (the kernels are the closed form of exactly this relaxation), with about a
// quarter of the arithmetic.
//
// Flow populations are handled as deviations d = f - w from the rest state
// (rho = 1, u = 0; w = 2/9, 1/9, 1/72), so every constant of the rest state
// cancels analytically and rounding acts on O(Ma) numbers.  The scalar is
// handled directly (reference temperature 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

template <typename R>
struct FlowCoef {
    R omega;       // shear rates omega_4..omega_8
    R omega_bulk;  // trace rate omega_9
    R omega_hi;    // omega_10..omega_14
    R gbeta, T_ref;
    int fourth_maxwell;
};

template <typename R>
struct ThermCoef {
    R omega_T;    // first-order rates omega_1..omega_3 (eq. 23)
    R omega_hiT;  // rates of orders >= 2
    R cs2;        // c_sphi^2
    R src;        // uniform scalar source R per cell and step (eq. 4)
};

template <typename R>
__device__ __forceinline__ R fast_rcp(R x) {
    return R(1) / x;
}
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}

// Raw monomial moments of a D3Q15 population vector.
template <typename R>
struct Raw15 {
    R m0, x, y, z, xx, yy, zz, xy, xz, yz, xyy, xxy, xxz, xyz, xxyy;
};

template <typename R>
__device__ __forceinline__ Raw15<R> raw15(const R (&d)[15]) {
    // corners: Hadamard over x, then y, then z
    const R s_pp = d[7] + d[8], x_pp = d[7] - d[8];     // y+ z+
    const R s_mp = d[9] + d[10], x_mp = d[9] - d[10];   // y- z+
    const R s_pm = d[11] + d[12], x_pm = d[11] - d[12]; // y+ z-
    const R s_mm = d[13] + d[14], x_mm = d[13] - d[14]; // y- z-
    const R zp_s = s_pp + s_mp, zp_y = s_pp - s_mp, zp_x = x_pp + x_mp, zp_xy = x_pp - x_mp;
    const R zm_s = s_pm + s_mm, zm_y = s_pm - s_mm, zm_x = x_pm + x_mm, zm_xy = x_pm - x_mm;
    const R c0 = zp_s + zm_s, cz = zp_s - zm_s;
    const R cy = zp_y + zm_y, cyz = zp_y - zm_y;
    const R cx = zp_x + zm_x, cxz = zp_x - zm_x;
    const R cxy = zp_xy + zm_xy, cxyz = zp_xy - zm_xy;
    const R px = d[1] + d[2], py = d[3] + d[4], pz = d[5] + d[6];
    Raw15<R> r;
    r.m0 = d[0] + px + py + pz + c0;
    r.x = (d[1] - d[2]) + cx;
    r.y = (d[3] - d[4]) + cy;
    r.z = (d[5] - d[6]) + cz;
    r.xx = px + c0;
    r.yy = py + c0;
    r.zz = pz + c0;
    r.xy = cxy;
    r.xz = cxz;
    r.yz = cyz;
    r.xyy = cx;  // on D3Q15, x y^2 is nonzero only on corners
    r.xxy = cy;
    r.xxz = cz;
    r.xyz = cxyz;
    r.xxyy = c0;
    return r;
}

// Populations from the fifteen raw moments (inverse of raw15).
template <typename R>
__device__ __forceinline__ void pops15(const Raw15<R>& r, R (&d)[15]) {
    const R e = R(0.125);
    // corner (sx,sy,sz) = (xxyy + sx xyy + sy xxy + sz xxz + sx sy xy + sx sz xz
    //                      + sy sz yz + sx sy sz xyz) / 8
    const R Pp = (r.xxyy + r.xxz) * e, Pm = (r.xxyy - r.xxz) * e;
    const R Xp = (r.xyy + r.xz) * e, Xm = (r.xyy - r.xz) * e;
    const R Yp = (r.xxy + r.yz) * e, Ym = (r.xxy - r.yz) * e;
    const R XYp = (r.xy + r.xyz) * e, XYm = (r.xy - r.xyz) * e;
    const R Qpp = Pp + Yp, QXpp = Xp + XYp;  // y+ z+
    const R Qmp = Pp - Yp, QXmp = Xp - XYp;  // y- z+
    const R Qpm = Pm + Ym, QXpm = Xm + XYm;  // y+ z-
    const R Qmm = Pm - Ym, QXmm = Xm - XYm;  // y- z-
    d[7] = Qpp + QXpp;
    d[8] = Qpp - QXpp;
    d[9] = Qmp + QXmp;
    d[10] = Qmp - QXmp;
    d[11] = Qpm + QXpm;
    d[12] = Qpm - QXpm;
    d[13] = Qmm + QXmm;
    d[14] = Qmm - QXmm;
    const R h = R(0.5);
    const R ax = r.xx - r.xxyy, bx = r.x - r.xyy;
    const R ay = r.yy - r.xxyy, by = r.y - r.xxy;
    const R az = r.zz - r.xxyy, bz = r.z - r.xxz;
    d[1] = h * (ax + bx);
    d[2] = h * (ax - bx);
    d[3] = h * (ay + by);
    d[4] = h * (ay - by);
    d[5] = h * (az + bz);
    d[6] = h * (az - bz);
    d[0] = r.m0 - r.xx - r.yy - r.zz + R(2) * r.xxyy;
}

// Post-collision raw moments from post-collision central moments about u.
// Each raw monomial is the binomial expansion of ((e-u)+u)^m.
//   m0:     zeroth moment written to the result
//   mass:   zeroth moment as it multiplies powers of u
//   k1*:    first-order central moments
//   kxx..:  diagonal second-order central moments written to the result
//   kxxP..: diagonal second-order central moments as they multiply u
//   kxy..:  mixed second order; k3*: third order; kxxyy: fourth order.
// For the scalar m0 = mass and kxxP = kxx.  For the flow deviations the
// written values are deviations from the rest state while the products with
// u need the full values (rho, 1/3 + kxx); the rest state's own raw moments
// (1, 1/3, 1/9) cancel against the deviation of the result.
template <typename R>
__device__ __forceinline__ Raw15<R> shift_back15(R m0, R mass, R ux, R uy, R uz, R k1x, R k1y,
                                                 R k1z, R kxx, R kyy, R kzz, R kxxP, R kyyP,
                                                 R kxy, R kxz, R kyz, R kxyy, R kxxy, R kxxz,
                                                 R kxyz, R kxxyy) {
    Raw15<R> r;
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    r.m0 = m0;
    r.x = k1x + ux * mass;
    r.y = k1y + uy * mass;
    r.z = k1z + uz * mass;
    r.xx = kxx + ux * (R(2) * k1x + ux * mass);
    r.yy = kyy + uy * (R(2) * k1y + uy * mass);
    r.zz = kzz + uz * (R(2) * k1z + uz * mass);
    r.xy = kxy + ux * k1y + uy * k1x + uxy * mass;
    r.xz = kxz + ux * k1z + uz * k1x + ux * uz * mass;
    r.yz = kyz + uy * k1z + uz * k1y + uy * uz * mass;
    r.xyy = kxyy + R(2) * uy * kxy + uyy * k1x + ux * kyyP + R(2) * uxy * k1y + uxy * uy * mass;
    r.xxy = kxxy + R(2) * ux * kxy + uxx * k1y + uy * kxxP + R(2) * uxy * k1x + uxx * uy * mass;
    r.xxz = kxxz + R(2) * ux * kxz + uxx * k1z + uz * kxxP + R(2) * ux * uz * k1x + uxx * uz * mass;
    r.xyz = kxyz + ux * kyz + uy * kxz + uz * kxy + uxy * k1z + ux * uz * k1y + uy * uz * k1x +
            uxy * uz * mass;
    r.xxyy = kxxyy + R(2) * uy * kxxy + R(2) * ux * kxyy + uyy * kxxP + uxx * kyyP +
             R(4) * uxy * kxy + R(2) * uxy * uy * k1x + R(2) * uxy * ux * k1y + uxy * uxy * mass;
    return r;
}

// ---------------------------------------------------------------------------
// Flow collision, eq. (2a) with the kernel of Appendix A.
// d: pre-collision deviations fbar - w in, post-collision deviations out.
// Fz: Boussinesq force (only z).  Returns the velocity of eq. (3).
//
// Source: central moments (0; F; 0...) (no second- or higher-order central
// moments), so eta = fbar + S has the central moments of fbar except at
// first order, where it carries F/2; orders 0 and 1 are invariants.
// Second order relaxes with omega (deviatoric) and omega_bulk (trace) toward
// rho/3 on the diagonal; third order with omega_hi toward 0; xxyy with
// omega_hi toward kxx~ kyy~ / rho (or rho/9 when fourth_maxwell).
// HG = false specialises omega_hi == 1.
// ---------------------------------------------------------------------------
template <typename R, bool HG>
__device__ __forceinline__ void collide_flow(R (&d)[15], R Fz, const FlowCoef<R>& c, R& ux,
                                             R& uy, R& uz) {
    const Raw15<R> r = raw15(d);
    const R rho_d = r.m0;  // rho - 1
    const R rho = R(1) + rho_d;
    const R inv = fast_rcp(rho);
    const R hz = R(0.5) * Fz;
    const R Jz = r.z + hz;  // rho uz
    ux = r.x * inv;
    uy = r.y * inv;
    uz = Jz * inv;
    const R third = R(1) / R(3);

    // second-order central moments of fbar (deviations from 1/3 on the
    // diagonal), using sum fbar e = (rho ux, rho uy, rho uz - Fz/2)
    const R kxx0 = r.xx - ux * r.x;
    const R kyy0 = r.yy - uy * r.y;
    const R kzz0 = r.zz - uz * (r.z - hz);
    const R kxy0 = r.xy - ux * r.y;
    const R kxz0 = r.xz - uz * r.x + ux * hz;
    const R kyz0 = r.yz - uz * r.y + uy * hz;

    // relaxation: functionals xx-yy, xx+yy-2zz (omega), trace (omega_bulk)
    const R om1 = R(1) - c.omega;
    const R A = om1 * (kxx0 - kyy0);
    const R B = om1 * (kxx0 + kyy0 - R(2) * kzz0);
    const R C0 = kxx0 + kyy0 + kzz0;
    const R C = C0 + c.omega_bulk * (rho_d - C0);
    const R sixth = R(1) / R(6);
    const R kxx = (R(3) * A + B + R(2) * C) * sixth;
    const R kyy = (R(-3) * A + B + R(2) * C) * sixth;
    const R kzz = (C - B) * third;
    const R kxy = om1 * kxy0, kxz = om1 * kxz0, kyz = om1 * kyz0;

    // fourth-order equilibrium (deviation from 1/9)
    R e4;
    if (c.fourth_maxwell)
        e4 = rho_d * (R(1) / R(9));
    else
        e4 = ((kxx + kyy) * third + kxx * kyy - rho_d * (R(1) / R(9))) * inv;

    R k3xyy = 0, k3xxy = 0, k3xxz = 0, k3xyz = 0, k4 = e4;
    if constexpr (HG) {
        // pre-collision third- and fourth-order central moments of fbar
        const R a = ux, b = uy, cc = uz, rx = r.x, ry = r.y, rz = r.z;
        const R rxx = third + r.xx, ryy = third + r.yy;
        const R m3xyy = r.xyy - R(2) * b * r.xy + b * b * rx - a * ryy + R(2) * a * b * ry - a * b * b * rho;
        const R m3xxy = r.xxy - R(2) * a * r.xy + a * a * ry - b * rxx + R(2) * a * b * rx - a * a * b * rho;
        const R m3xxz = r.xxz - R(2) * a * r.xz + a * a * rz - cc * rxx + R(2) * a * cc * rx - a * a * cc * rho;
        const R m3xyz = r.xyz - a * r.yz - b * r.xz - cc * r.xy + a * b * rz + a * cc * ry + b * cc * rx -
                        a * b * cc * rho;
        const R m4 = r.xxyy - R(2) * b * r.xxy + b * b * rxx - R(2) * a * r.xyy + R(4) * a * b * r.xy -
                     R(2) * a * b * b * rx + a * a * ryy - R(2) * a * a * b * ry + a * a * b * b * rho;
        // (r.xxyy is already the deviation from the rest value 1/9)
        const R oh1 = R(1) - c.omega_hi;
        k3xyy = oh1 * m3xyy;
        k3xxy = oh1 * m3xxy;
        k3xxz = oh1 * m3xxz;
        k3xyz = oh1 * m3xyz;
        k4 = m4 + c.omega_hi * (e4 - m4);
    }

    // back to raw moments: first-order central moments (0, 0, Fz/2), zeroth
    // moment rho; written as deviations from the rest state
    const Raw15<R> q = shift_back15<R>(rho_d, rho, ux, uy, uz, R(0), R(0), hz, kxx, kyy, kzz,
                                       third + kxx, third + kyy, kxy, kxz, kyz, k3xyy, k3xxy,
                                       k3xxz, k3xyz, k4);
    pops15(q, d);
}

// ---------------------------------------------------------------------------
// Scalar collision, D3Q15 (Sec. 2.2, eq. (13a)).
// g holds gbar = g - S/2 (eq. 13); the kernel relaxes the central moments of
// eta = gbar + S (eq. 21), S the source populations.  The zeroth central
// moment is kept; first order relaxes with omega_T toward 0; orders >= 2
// with omega_hiT toward cs2 phi (diagonal), 0 (mixed, third), cs2^2 phi
// (xxyy) (eq. 15), phi = sum gbar + R/2 (eq. 25).
// HG = false specialises omega_hiT == 1 and R == 0.
// ---------------------------------------------------------------------------
template <typename R, bool HG>
__device__ __forceinline__ void collide_thermal15(R (&g)[15], R ux, R uy, R uz,
                                                  const ThermCoef<R>& c) {
    Raw15<R> r = raw15(g);
    R phi = r.m0;
    if constexpr (HG) {
        // lattice raw moments of S = K^-1 m^s (eq. 19 as printed; its cubic
        // projections alias on D3Q15, whence the (u.u - 1)/2 of the
        // third-order sums and the 1/3 of xxyy)
        const R s = c.src;
        const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
        const R h3 = R(0.5) * (uxx + uyy + uzz - R(1)) * s;
        phi = r.m0 + R(0.5) * s;
        r.m0 += s;
        r.x += ux * s;
        r.y += uy * s;
        r.z += uz * s;
        r.xx += uxx * s;
        r.yy += uyy * s;
        r.zz += uzz * s;
        r.xy += ux * uy * s;
        r.xz += ux * uz * s;
        r.yz += uy * uz * s;
        r.xyy += ux * h3;
        r.xxy += uy * h3;
        r.xxz += uz * h3;
        r.xyz += ux * uy * uz * s;
        r.xxyy += (uxx * uyy + uxx * uzz + uyy * uzz) * s * (R(1) / R(3));
    }
    const R T = r.m0;  // zeroth moment of eta: the mass of the shifts
    const R o1 = R(1) - c.omega_T;
    const R k1x = o1 * (r.x - ux * T), k1y = o1 * (r.y - uy * T), k1z = o1 * (r.z - uz * T);
    const R cT = c.cs2 * phi;
    R kxx = cT, kyy = cT, kzz = cT, kxy = 0, kxz = 0, kyz = 0;
    R k3xyy = 0, k3xxy = 0, k3xxz = 0, k3xyz = 0, k4 = c.cs2 * cT;
    if constexpr (HG) {
        const R a = ux, b = uy, cc = uz, rx = r.x, ry = r.y, rz = r.z;
        const R mxx = r.xx - R(2) * a * rx + a * a * T;
        const R myy = r.yy - R(2) * b * ry + b * b * T;
        const R mzz = r.zz - R(2) * cc * rz + cc * cc * T;
        const R mxy = r.xy - a * ry - b * rx + a * b * T;
        const R mxz = r.xz - a * rz - cc * rx + a * cc * T;
        const R myz = r.yz - b * rz - cc * ry + b * cc * T;
        const R m3xyy = r.xyy - R(2) * b * r.xy + b * b * rx - a * r.yy + R(2) * a * b * ry - a * b * b * T;
        const R m3xxy = r.xxy - R(2) * a * r.xy + a * a * ry - b * r.xx + R(2) * a * b * rx - a * a * b * T;
        const R m3xxz = r.xxz - R(2) * a * r.xz + a * a * rz - cc * r.xx + R(2) * a * cc * rx - a * a * cc * T;
        const R m3xyz = r.xyz - a * r.yz - b * r.xz - cc * r.xy + a * b * rz + a * cc * ry + b * cc * rx -
                        a * b * cc * T;
        const R m4 = r.xxyy - R(2) * b * r.xxy + b * b * r.xx - R(2) * a * r.xyy + R(4) * a * b * r.xy -
                     R(2) * a * b * b * rx + a * a * r.yy - R(2) * a * a * b * ry + a * a * b * b * T;
        const R w = c.omega_hiT, w1 = R(1) - w;
        kxx = mxx + w * (cT - mxx);
        kyy = myy + w * (cT - myy);
        kzz = mzz + w * (cT - mzz);
        kxy = w1 * mxy;
        kxz = w1 * mxz;
        kyz = w1 * myz;
        k3xyy = w1 * m3xyy;
        k3xxy = w1 * m3xxy;
        k3xxz = w1 * m3xxz;
        k3xyz = w1 * m3xyz;
        k4 = m4 + w * (c.cs2 * cT - m4);
    }
    const Raw15<R> t = shift_back15<R>(T, T, ux, uy, uz, k1x, k1y, k1z, kxx, kyy, kzz, kxx, kyy,
                                       kxy, kxz, kyz, k3xyy, k3xxy, k3xxz, k3xyz, k4);
    pops15(t, g);
}

// ---------------------------------------------------------------------------
// Scalar collision, D3Q7 (Appendix C, eq. (13a)), gbar and eta = gbar + S
// as for D3Q15.  Moments 1, x, y, z, xx-yy, xx+yy-2zz, xx+yy+zz; the three
// second-order functionals share omega_hiT, so the diagonal central moments
// relax individually toward cs2 phi.  The source's raw moments on D3Q7 are
// (R; u R; u_i^2 R) exactly.  HG = false specialises omega_hiT == 1, R == 0.
// ---------------------------------------------------------------------------
template <typename R, bool HG>
__device__ __forceinline__ void collide_thermal7(R (&g)[7], R ux, R uy, R uz,
                                                 const ThermCoef<R>& c) {
    R px = g[1] + g[2], py = g[3] + g[4], pz = g[5] + g[6];
    R jx = g[1] - g[2], jy = g[3] - g[4], jz = g[5] - g[6];
    R T = g[0] + px + py + pz;
    R phi = T;
    if constexpr (HG) {
        const R s = c.src;
        phi = T + R(0.5) * s;
        T += s;
        jx += ux * s;
        jy += uy * s;
        jz += uz * s;
        px += ux * ux * s;
        py += uy * uy * s;
        pz += uz * uz * s;
    }
    const R o1 = R(1) - c.omega_T;
    const R kx = o1 * (jx - ux * T), ky = o1 * (jy - uy * T), kz = o1 * (jz - uz * T);
    const R cT = c.cs2 * phi;
    R kxx = cT, kyy = cT, kzz = cT;
    if constexpr (HG) {
        const R w = c.omega_hiT;
        const R mxx = px - R(2) * ux * jx + ux * ux * T;
        const R myy = py - R(2) * uy * jy + uy * uy * T;
        const R mzz = pz - R(2) * uz * jz + uz * uz * T;
        kxx = mxx + w * (cT - mxx);
        kyy = myy + w * (cT - myy);
        kzz = mzz + w * (cT - mzz);
    }
    const R rx = kx + ux * T, ry = ky + uy * T, rz = kz + uz * T;
    const R rxx = kxx + ux * (R(2) * kx + ux * T);
    const R ryy = kyy + uy * (R(2) * ky + uy * T);
    const R rzz = kzz + uz * (R(2) * kz + uz * T);
    const R h = R(0.5);
    g[1] = h * (rxx + rx);
    g[2] = h * (rxx - rx);
    g[3] = h * (ryy + ry);
    g[4] = h * (ryy - ry);
    g[5] = h * (rzz + rz);
    g[6] = h * (rzz - rz);
    g[0] = T - rxx - ryy - rzz;
}

// Flow equilibrium deviations at (rho = 1 + rho_d, u): central moments
// (rho; 0; rho/3 diagonal; 0; rho/9).
template <typename R>
__device__ __forceinline__ void flow_equilibrium(R rho_d, R ux, R uy, R uz, R (&d)[15]) {
    const R third = R(1) / R(3), ninth = R(1) / R(9);
    const R rho = R(1) + rho_d, k = rho_d * third;
    const Raw15<R> q = shift_back15<R>(rho_d, rho, ux, uy, uz, R(0), R(0), R(0), k, k, k,
                                       rho * third, rho * third, R(0), R(0), R(0), R(0), R(0),
                                       R(0), R(0), rho_d * ninth);
    pops15(q, d);
}

// Scalar equilibrium at (T, u), eq. (15).
template <typename R>
__device__ __forceinline__ void thermal_equilibrium15(R T, R ux, R uy, R uz, R cs2, R (&g)[15]) {
    const R cT = cs2 * T;
    const Raw15<R> t = shift_back15<R>(T, T, ux, uy, uz, R(0), R(0), R(0), cT, cT, cT, cT, cT, R(0),
                                       R(0), R(0), R(0), R(0), R(0), R(0), cs2 * cT);
    pops15(t, g);
}

template <typename R>
__device__ __forceinline__ void thermal_equilibrium7(R T, R ux, R uy, R uz, R cs2, R (&g)[7]) {
    const R cT = cs2 * T, h = R(0.5);
    const R rx = ux * T, ry = uy * T, rz = uz * T;
    const R rxx = cT + ux * rx, ryy = cT + uy * ry, rzz = cT + uz * rz;
    g[1] = h * (rxx + rx);
    g[2] = h * (rxx - rx);
    g[3] = h * (ryy + ry);
    g[4] = h * (ryy - ry);
    g[5] = h * (rzz + rz);
    g[6] = h * (rzz - rz);
    g[0] = T - rxx - ryy - rzz;
}

}  // namespace lbm
