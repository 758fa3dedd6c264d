// Transform shapes built into the library and the launch-shape helpers shared
// by the filter kernels (one-work-group-per-tile and persistent forms).
#pragma once
#include "mf_internal.hpp"

namespace mf {

constexpr int clamp_threads(int x) { return x < 64 ? 64 : (x > 1024 ? 1024 : x); }

inline bool want(mf_precision prec, bool f64) { return (prec == MF_FP64) == f64; }

// Pass 1 keeps the occupancy its LDS allows for the wide FP32 tiles (8 waves
// per SIMD: four 512-thread or two 1024-thread work-groups per CU, 64 VGPRs)
// and for the FP64 256-thread tiles (4 waves, 128 VGPRs): it is bound by its
// stores, which need many waves in flight.
template <typename T, int NT>
constexpr int pass1_min_waves() {
    return sizeof(T) == 4 ? (NT >= 512 ? 8 : 1) : (NT == 256 ? 4 : 1);
}

// Every (precision, N1, N2, C, B, R2, XS) instantiated (R2: largest radix of
// the pass-2 stages, 16 or 8; it sets the pass-2 threads B N2 / R2.  XS: 1 the
// pass-2 stages exchange real and imaginary parts separately, in half the
// LDS; 2 the same with bank-conflict-free layouts).  The first entry for each
// N and precision is its default plan.
#define MF_SHAPES(X)                                                                                              \
    X(float, 32, 32, 16, 32, 16, 0) X(float, 32, 64, 16, 32, 16, 0) X(float, 64, 64, 16, 64, 16, 0)                 \
    X(float, 64, 128, 16, 32, 16, 0) X(float, 128, 128, 16, 32, 16, 0) X(float, 128, 256, 16, 16, 16, 0)            \
    X(float, 256, 256, 16, 16, 16, 0) X(float, 256, 512, 16, 8, 16, 0) X(float, 512, 512, 16, 8, 16, 0)             \
    X(float, 512, 1024, 16, 4, 16, 0) X(float, 256, 4096, 32, 1, 16, 2) X(float, 256, 4096, 16, 1, 16, 1)           \
    X(float, 256, 4096, 16, 1, 16, 0)                                                                              \
    X(float, 1024, 2048, 16, 2, 16, 0) X(float, 1024, 4096, 16, 1, 16, 2) X(float, 1024, 4096, 16, 1, 16, 1)        \
    X(float, 1024, 4096, 16, 1, 16, 0)                                                                             \
    X(float, 1024, 4096, 8, 1, 16, 0) X(float, 1024, 4096, 8, 1, 16, 1)                                           \
    X(float, 1024, 1024, 8, 4, 16, 0) X(float, 1024, 1024, 16, 8, 16, 0) X(float, 1024, 1024, 16, 4, 16, 0)         \
    X(float, 512, 2048, 16, 2, 16, 0) X(float, 2048, 512, 8, 8, 16, 0) X(float, 2048, 2048, 8, 2, 16, 0)            \
    X(float, 512, 8192, 16, 1, 16, 0) X(float, 256, 4096, 16, 1, 8, 0)                                             \
    X(float, 1024, 4096, 8, 1, 8, 0) X(float, 256, 4096, 32, 1, 16, 1) X(float, 256, 4096, 16, 1, 16, 2)          \
    X(double, 32, 32, 8, 32, 16, 0) X(double, 32, 64, 8, 32, 16, 0) X(double, 64, 64, 8, 64, 16, 0)                 \
    X(double, 64, 128, 8, 32, 16, 0) X(double, 128, 128, 8, 32, 16, 0) X(double, 128, 256, 8, 16, 16, 0)            \
    X(double, 256, 256, 8, 16, 16, 0) X(double, 256, 512, 8, 8, 16, 0) X(double, 512, 512, 8, 8, 16, 0)             \
    X(double, 512, 1024, 8, 4, 16, 0) X(double, 256, 4096, 16, 1, 16, 1) X(double, 256, 4096, 8, 1, 16, 1)         \
    X(double, 512, 2048, 8, 2, 16, 0)                                                                              \
    X(double, 1024, 2048, 4, 2, 16, 0)                                                                             \
    X(double, 2048, 2048, 2, 2, 16, 0) X(double, 1024, 1024, 8, 4, 16, 0) X(double, 1024, 1024, 4, 4, 16, 0)        \
    X(double, 1024, 1024, 4, 2, 16, 0) X(double, 512, 2048, 8, 2, 8, 0) X(double, 256, 4096, 8, 1, 16, 0)         \
    X(double, 256, 4096, 16, 1, 16, 2)

}  // namespace mf
