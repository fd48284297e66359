// Compile-time dispatch over (storage precision, scalar lattice) shared by
// the kernel launchers.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.hpp"

namespace lbm {

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

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

}  // namespace lbm
