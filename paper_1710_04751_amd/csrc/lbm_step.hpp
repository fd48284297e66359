// Shared device code of the fused step: lattice tables, range-checked
// population access and the per-cell stream-collide update.  Included by
// the single-cavity kernels (lbm_kernels.hip) and the batched kernels
// (lbm_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_index.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace kern {


using idx::EX15;
using idx::EY15;
using idx::EZ15;
using idx::OPP15;
using idx::EX7;
using idx::EY7;
using idx::EZ7;
using idx::OPP7;

// Rest-state flow weights (D3Q15, c_s^2 = 1/3).
__device__ __forceinline__ double flow_weight(int a) {
    return a == 0 ? 2.0 / 9.0 : (a <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
}

template <typename S>
struct Store;
template <>
struct Store<double> {
    template <typename R>
    __device__ static R ld(const double* p) { return (R)*p; }
    __device__ static void st(double* p, double v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<float> {
    template <typename R>
    __device__ static R ld(const float* p) { return (R)*p; }
    __device__ static void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<_Float16> {
    template <typename R>
    __device__ static R ld(const _Float16* p) { return (R)(float)*p; }
    __device__ static void st(_Float16* p, float v) {
        __builtin_nontemporal_store((_Float16)v, p);  // round to nearest even
    }
};

// Stochastic rounding to FP16 with the gfx950 conversion instruction: v goes
// to the FP16 neighbour below or above it in magnitude, the upper one with
// probability equal to v's distance from the lower one in ulps, so the
// rounding is unbiased.  The instruction takes its random bits from the high
// 16 bits of rnd and resolves the probability to 2^-13 of an ulp (the 13
// FP32 mantissa bits below an FP16 normal's last place): for inputs of
// either sign, normal and subnormal in FP16, the share of round-ups over all
// 2^16 values of the high half equals that distance truncated to 13 bits.
__device__ __forceinline__ _Float16 half_stochastic(float v, uint32_t rnd) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 o = {0, 0};
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, v, rnd, false);
    return o[0];
}

// 32-bit integer mix (the "lowbias32" finaliser of C. Wellons' hash
// prospector): the seed of stochastic rounding's random stream, keyed by
// step and cell.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Position of population a of cell c = (z*ny + y)*nx + x in a state
// (c < 2^31; the flow base for a < 15, the scalar base for scalar a).
__host__ __device__ __forceinline__ int64_t pop_at(PopLay L, int a, int64_t c) {
    const uint32_t row = (uint32_t)c / (uint32_t)L.nx;
    const uint32_t x = (uint32_t)c - row * (uint32_t)L.nx;
    const uint32_t grp = row >> L.gs, sub = row & ((1u << L.gs) - 1u);
    return ((((int64_t)grp * L.rq + a) << L.gs) + sub) * L.nx + x;
}

// Range-checked population access.  Every load and store of the step kernel
// goes through a raw buffer resource over a window of the state that starts
// at a row of the block's own tile or before it and ends at or before the
// state's end: the hardware returns 0 for a load and drops a store outside
// it, so no index, however computed, can touch memory beyond the state.
// Offsets are 32-bit byte offsets from the window's (scalar) base.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
constexpr int kNonTemporal = 2;  // cache policy of the stores: non-temporal

template <typename S>
struct Buf;
template <>
struct Buf<float> {
    template <typename R>
    __device__ static R ld(__amdgpu_buffer_rsrc_t r, uint32_t i) {
        return (R)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0));
    }
    __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t i, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, i * 4u, 0,
                                              kNonTemporal);
    }
};
template <>
struct Buf<double> {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    template <typename R>
    __device__ static R ld(__amdgpu_buffer_rsrc_t r, uint32_t i) {
        return (R)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
    }
    __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t i, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, i * 8u, 0, kNonTemporal);
    }
};
template <>
struct Buf<_Float16> {
    template <typename R>
    __device__ static R ld(__amdgpu_buffer_rsrc_t r, uint32_t i) {
        return (R)(float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, i * 2u, 0, 0));
    }
    __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t i, float v) {
        // round to nearest even
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r,
                                              i * 2u, 0, kNonTemporal);
    }
};

template <typename R>
struct KCoef {
    FlowCoef<R> f;
    ThermCoef<R> t;
    R T_hot, T_cold;
    R w_face, w_corner;  // rest weights of the scalar (anti-bounce-back)
    int32_t sr;          // FP16 storage: stochastic rounding
    uint32_t seed;       // step index
    int32_t spec;        // scalar on the adiabatic faces: specular reflection
};

template <typename R>
KCoef<R> make_kcoef(const Coefs& c, int qt) {
    KCoef<R> k;
    k.f.omega = (R)c.omega;
    k.f.omega_bulk = (R)c.omega_bulk;
    k.f.omega_hi = (R)c.omega_hi;
    k.f.gbeta = (R)c.gbeta;
    k.f.T_ref = (R)c.T_ref;
    k.f.fourth_maxwell = c.fourth_maxwell;
    k.t.omega_T = (R)c.omega_T;
    k.t.omega_hiT = (R)c.omega_hiT;
    k.t.cs2 = (R)c.cs2;
    k.t.src = (R)c.src;
    k.sr = c.sr;
    k.seed = c.seed;
    k.spec = c.spec;
    k.T_hot = (R)c.T_hot;
    k.T_cold = (R)c.T_cold;
    if (qt == 7) {
        k.w_face = (R)(c.cs2 / 2);
        k.w_corner = 0;
    } else {
        k.w_face = (R)((c.cs2 - c.cs2 * c.cs2) / 2);
        k.w_corner = (R)(c.cs2 * c.cs2 / 8);
    }
    return k;
}

// ---------------------------------------------------------------------------
// Fused stream-collide update of one cell (shared by the single-cavity and
// the batched kernels, so both compute bit-identical results)
// ---------------------------------------------------------------------------
// seed: the step index keying stochastic rounding (FP16 storage with k.sr).
template <typename R, typename S, int QT, bool HG>
__device__ __forceinline__ void update_cell(const S* __restrict__ in, S* __restrict__ out, int x,
                                            int y, int z, int y0, int nxi, int nyi, int nzi,
                                            int gs, const KCoef<R>& k, uint32_t seed) {
    constexpr int RQ = 15 + QT;
    // The block's window starts at the group of row (z-1, y0-1) and runs to
    // the end of the state; y0 and z are uniform over the block, so the base
    // is a scalar.  Every offset below is relative to it (lbm_index.hpp).
    const idx::Window w = idx::window_of(z, y0, nxi, nyi, nzi, gs, RQ, (int)sizeof(S));
    const __amdgpu_buffer_rsrc_t ri = pop_rsrc(in + (size_t)w.g0 * w.glen, w.bytes);
    const __amdgpu_buffer_rsrc_t ro = pop_rsrc(out + (size_t)w.g0 * w.glen, w.bytes);
    const idx::CellAt c = idx::cell_at(w, x, y, z, nxi, nyi, nzi);
    R d[15];
#pragma unroll
    for (int a = 0; a < 15; ++a) d[a] = Buf<S>::template ld<R>(ri, idx::flow_load(w, c, a));
    R gq[QT];
    // Scalar gather: anti-bounce-back across the Dirichlet walls (this rule
    // wins on edges), bounce-back or -- with specular reflection, D3Q15
    // only (on D3Q7 the two coincide) -- the mirrored population across the
    // adiabatic faces.  The choice is uniform over the launch.
    auto gather_scalar = [&](auto spec_tag) {
        constexpr bool SPEC = decltype(spec_tag)::value;
#pragma unroll
        for (int a = 0; a < QT; ++a) {
            const idx::ScalarLoad l = idx::scalar_load<QT, SPEC>(w, c, a);
            R v = Buf<S>::template ld<R>(ri, l.off);
            if (l.dirichlet) {
                const int ex = QT == 7 ? EX7[a] : EX15[a];
                const int ey = QT == 7 ? EY7[a] : EY15[a];
                const int ez = QT == 7 ? EZ7[a] : EZ15[a];
                const R wa = (ey == 0 && ez == 0) ? k.w_face : k.w_corner;
                const R tw = ex > 0 ? k.T_hot : k.T_cold;  // source beyond x = -1/2 or nx - 1/2
                v = R(2) * wa * tw - v;
            }
            gq[a] = v;
        }
    };
    if (QT == 15 && k.spec)
        gather_scalar(std::true_type{});
    else
        gather_scalar(std::false_type{});

    R T = 0;
#pragma unroll
    for (int a = 0; a < QT; ++a) T += gq[a];
    if constexpr (HG) T += R(0.5) * k.t.src;  // eq. (25) with the source
    const R Fz = k.f.gbeta * (T - k.f.T_ref);
    R ux, uy, uz;
    collide_flow<R, HG>(d, Fz, k.f, ux, uy, uz);
    if constexpr (QT == 7)
        collide_thermal7<R, HG>(gq, ux, uy, uz, k.t);
    else
        collide_thermal15<R, HG>(gq, ux, uy, uz, k.t);

    if constexpr (std::is_same<S, _Float16>::value) {
        if (k.sr) {
            // The cell's random stream: a hash of (step, cell) seeds a
            // xorshift32 generator (shifts 13, 17, 5; state never 0); each
            // 32-bit word gives the 16 random bits of two stores.
            const uint32_t cell = ((uint32_t)z * w.ny + (uint32_t)y) * w.nx + (uint32_t)x;
            uint32_t xs = mix32(seed * 0x9e3779b9u ^ cell);
            xs = xs ? xs : 0x9e3779b9u;
            uint32_t rnd[(15 + QT + 1) / 2];
#pragma unroll
            for (int j = 0; j < (15 + QT + 1) / 2; ++j) {
                xs ^= xs << 13;
                xs ^= xs >> 17;
                xs ^= xs << 5;
                rnd[j] = xs;
            }
            // value 2j takes the high half of word j, value 2j + 1 the low half
#pragma unroll
            for (int a = 0; a < 15; ++a)
                Buf<S>::st(ro, idx::store_at(w, c, a),
                           (float)half_stochastic(d[a], rnd[a >> 1] << (16 * (a & 1))));
#pragma unroll
            for (int a = 0; a < QT; ++a)
                Buf<S>::st(ro, idx::store_at(w, c, 15 + a),
                           (float)half_stochastic(gq[a], rnd[(a + 15) >> 1] << (16 * ((a + 15) & 1))));
            return;
        }
    }
#pragma unroll
    for (int a = 0; a < 15; ++a) Buf<S>::st(ro, idx::store_at(w, c, a), d[a]);
#pragma unroll
    for (int a = 0; a < QT; ++a) Buf<S>::st(ro, idx::store_at(w, c, 15 + a), gq[a]);
}

}  // namespace kern
}  // namespace lbm
