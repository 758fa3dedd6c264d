// Device building blocks shared by the libmf kernels: complex arithmetic,
// constant-size inverse DFTs held in registers, and the stationary-phase
// template rotor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mf.h"

namespace mf {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
// two-element vector of T (one 8- or 16-byte access), for the non-temporal loads and stores
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

// Raw buffer loads: a base and byte range in scalar registers (a gfx9 buffer
// descriptor with a 32-bit data format and no stride), a per-lane byte offset
// and a wave-uniform byte offset, so unrolled loads at constant distances from
// one lane offset need no per-load address arithmetic.  Reads outside the range
// return zero.
constexpr int kBufferWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufferWord3);
}
// AUX: the instruction's cache-policy bits (0: default, kBufferNT: non-temporal)
constexpr int kBufferNT = 2;
template <typename T, int AUX = 0>
__device__ __forceinline__ cx<T> buffer_load_cx(__amdgpu_buffer_rsrc_t rs, unsigned int lane_off, int uniform_off) {
    if constexpr (sizeof(T) == 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, uniform_off, AUX);
        return {__uint_as_float(v[0]), __uint_as_float(v[1])};
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, uniform_off, AUX);
        return {__hiloint2double((int)v[1], (int)v[0]), __hiloint2double((int)v[3], (int)v[2])};
    }
}

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by +i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------
// Inverse DFT of R points in registers: v_u <- sum_r v_r e^{+2 pi i u r / R}.
// Radix-2 decimation in time down to a hand-written 4-point kernel; the
// twiddles are compile-time roots of unity (R <= 16).
// ---------------------------------------------------------------------------
struct Roots16 {
    // cos and sin of 2 pi u / 16, u = 0..7
    static constexpr double c[8] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674};
    static constexpr double s[8] = {0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
                                    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977};
};

// multiply by e^{+2 pi i u / R} with compile-time u, R
template <int U, int R, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
    constexpr int q = (U * 16 / R) % 16;  // index in 16th roots
    if constexpr (q == 0) {
        return a;
    } else if constexpr (q == 4) {
        return mul_i(a);
    } else if constexpr (q == 8) {
        return cx<T>{-a.x, -a.y};
    } else if constexpr (q == 12) {
        return cx<T>{a.y, -a.x};
    } else if constexpr (q == 2 || q == 6 || q == 10 || q == 14) {
        // (+-1 +- i)/sqrt(2) multiples: 2 multiplies
        constexpr T h = T(0.70710678118654752);
        constexpr T cr = (q == 2 || q == 14) ? h : -h;
        constexpr T sr = (q == 2 || q == 6) ? h : -h;
        return cx<T>{(a.x * cr) - (a.y * sr), (a.x * sr) + (a.y * cr)};
    } else {
        constexpr T cr = q < 8 ? T(Roots16::c[q]) : T(Roots16::c[q - 8]) * T(-1);
        constexpr T sr = q < 8 ? T(Roots16::s[q]) : T(Roots16::s[q - 8]) * T(-1);
        return cx<T>{a.x * cr - a.y * sr, a.x * sr + a.y * cr};
    }
}

template <int R, typename T>
struct IDft;

template <typename T>
struct IDft<1, T> {
    __device__ __forceinline__ static void run(cx<T>*) {}
};

template <typename T>
struct IDft<2, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <typename T>
struct IDft<4, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
        cx<T> s13 = v[1] + v[3], d13 = mul_i(v[1] - v[3]);
        v[0] = s02 + s13;
        v[2] = s02 - s13;
        v[1] = d02 + d13;
        v[3] = d02 - d13;
    }
};

// Butterfly (e + w a, e - w a) with w = (+-1 +- i)/sqrt(2) (16th-root index q
// = 2, 6, 10, 14): w a = h (sx, sy) with sx, sy signed sums of a.x and a.y, so
// each output component is one add and one fused multiply-add.
template <int Q, typename T>
__device__ __forceinline__ void butterfly_diag(cx<T> e, cx<T> a, cx<T>& lo, cx<T>& hi) {
    constexpr T h = T(0.70710678118654752);
    T sx, sy;
    if constexpr (Q == 2) {
        sx = a.x - a.y;
        sy = a.x + a.y;
    } else if constexpr (Q == 6) {
        sx = -(a.x + a.y);
        sy = a.x - a.y;
    } else if constexpr (Q == 10) {
        sx = a.y - a.x;
        sy = -(a.x + a.y);
    } else {
        sx = a.x + a.y;
        sy = a.y - a.x;
    }
    lo = cx<T>{fma(sx, h, e.x), fma(sy, h, e.y)};
    hi = cx<T>{fma(sx, -h, e.x), fma(sy, -h, e.y)};
}

// Butterfly (e + w a, e - w a) with w = e^{2 pi i q / 16}, q odd and q < 8:
// w a = k (y.x, y.y) with k the larger of |cos|, |sin| (signed) and y formed by
// two fused multiply-adds with the ratio of the smaller to the larger
// (tan or cot of pi/8 in magnitude), so each output component is one more
// fused multiply-add: 6 operations instead of 8.
template <int Q, typename T>
__device__ __forceinline__ void butterfly_odd(cx<T> e, cx<T> a, cx<T>& lo, cx<T>& hi) {
    static_assert(Q == 1 || Q == 3 || Q == 5 || Q == 7, "odd sixteenth roots in the upper half plane");
    constexpr T t8 = T(0.41421356237309505);  // tan(pi/8)
    constexpr T c8 = T(0.92387953251128674);  // cos(pi/8)
    T yx, yy, k;
    if constexpr (Q == 1) {  // cos = c8, sin = t8 c8: w a = c8 (a.x - t8 a.y, a.y + t8 a.x)
        yx = fma(-t8, a.y, a.x);
        yy = fma(t8, a.x, a.y);
        k = c8;
    } else if constexpr (Q == 3) {  // cos = t8 c8, sin = c8: w a = c8 (t8 a.x - a.y, a.x + t8 a.y)
        yx = fma(t8, a.x, -a.y);
        yy = fma(t8, a.y, a.x);
        k = c8;
    } else if constexpr (Q == 5) {  // cos = -t8 c8, sin = c8: w a = c8 (-t8 a.x - a.y, a.x - t8 a.y)
        yx = fma(-t8, a.x, -a.y);
        yy = fma(-t8, a.y, a.x);
        k = c8;
    } else {  // Q == 7: cos = -c8, sin = t8 c8: w a = c8 (-a.x - t8 a.y, t8 a.x - a.y)
        yx = fma(-t8, a.y, -a.x);
        yy = fma(t8, a.x, -a.y);
        k = c8;
    }
    lo = cx<T>{fma(yx, k, e.x), fma(yy, k, e.y)};
    hi = cx<T>{fma(yx, -k, e.x), fma(yy, -k, e.y)};
}

template <int R, typename T>
struct IDft {
    template <int U>
    __device__ __forceinline__ static void combine(cx<T>* v, cx<T>* e, cx<T>* o) {
        if constexpr (U < R / 2) {
            constexpr int q = (U * 16 / R) % 16;
            if constexpr (q == 2 || q == 6 || q == 10 || q == 14) {
                butterfly_diag<q, T>(e[U], o[U], v[U], v[U + R / 2]);
            } else if constexpr (q == 1 || q == 3 || q == 5 || q == 7) {
                butterfly_odd<q, T>(e[U], o[U], v[U], v[U + R / 2]);
            } else {
                cx<T> t = rot<U, R>(o[U]);
                v[U] = e[U] + t;
                v[U + R / 2] = e[U] - t;
            }
            combine<U + 1>(v, e, o);
        }
    }
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
            e[r] = v[2 * r];
            o[r] = v[2 * r + 1];
        }
        IDft<R / 2, T>::run(e);
        IDft<R / 2, T>::run(o);
        combine<0>(v, e, o);
    }
};

// Radix of stage s for an L-point transform: maxr (16 or 8) while at least
// maxr remains, then the remainder.
__host__ __device__ constexpr int radix_at(int L, int s, int maxr = 16) {
    int rem = L;
    for (int i = 0; i < s; ++i) rem /= (rem >= maxr ? maxr : rem);
    return rem >= maxr ? maxr : rem;
}
__host__ __device__ constexpr int num_stages(int L, int maxr = 16) {
    int n = 0;
    for (int rem = L; rem > 1; rem /= (rem >= maxr ? maxr : rem)) ++n;
    return n;
}
__host__ __device__ constexpr int span_before(int L, int s, int maxr = 16) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= radix_at(L, i, maxr);
    return ns;
}
__host__ __device__ constexpr int ilog2(long long x) {
    int r = 0;
    while ((1LL << r) < x) ++r;
    return r;
}

// ---------------------------------------------------------------------------
// Wave-wide reductions of a 32-bit value (all 64 lanes active): four DPP
// steps reduce each row of 16 lanes (swap neighbours, swap pairs, mirror the
// half-row, mirror the row), then the four row results are read into scalar
// registers.  The result is wave-uniform.
// ---------------------------------------------------------------------------
template <typename Op>
__device__ __forceinline__ unsigned int wave_reduce_u32(unsigned int v, Op op) {
    v = op(v, (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v = op(v, (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    v = op(v, (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
    v = op(v, (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xf, 0xf, false));  // row_mirror
    const unsigned int r0 = (unsigned int)__builtin_amdgcn_readlane((int)v, 0);
    const unsigned int r1 = (unsigned int)__builtin_amdgcn_readlane((int)v, 16);
    const unsigned int r2 = (unsigned int)__builtin_amdgcn_readlane((int)v, 32);
    const unsigned int r3 = (unsigned int)__builtin_amdgcn_readlane((int)v, 48);
    return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v) {
    return wave_reduce_u32(v, [](unsigned int a, unsigned int b) { return a > b ? a : b; });
}
__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v) {
    return wave_reduce_u32(v, [](unsigned int a, unsigned int b) { return a + b; });
}

// ---------------------------------------------------------------------------
// Roots of unity e^{+2 pi i m / M} from an exact dyadic argument frac = m / M.
// FP32: the argument is reduced exactly to [-1/2, 1/2] cycles and handed to
// the hardware sine and cosine, which take revolutions (max abs error ~1.3e-7
// on that range, measured against FP64).  FP64: sincospi.
// ---------------------------------------------------------------------------
__device__ __forceinline__ cx<float> root_of_unity(float frac) {
    const float x = frac - rintf(frac);
    return {__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x)};
}
__device__ __forceinline__ cx<double> root_of_unity(double frac) {
    double s, c;
    sincospi(2.0 * frac, &s, &c);
    return {c, s};
}

// ---------------------------------------------------------------------------
// Stationary-phase template rotor e^{+i Psi_k} for bin k.
//   Psi_k / 2 pi = b1 u + b2 u^2 + b3 u^3 + b5 u^5 + c0,  u = k^(-1/3)
// In the FP64-phase modes u is refined to ~1e-13 (below), the polynomial is
// evaluated in FP64 and reduced exactly to [-1/2, 1/2] cycles (subtracting
// the nearest integer is exact), and only the reduced fraction is rounded to
// the FFT precision before sin/cos.
// ---------------------------------------------------------------------------
// u = k^{-1/3}: hardware FP32 estimate (relative error ~1e-6), then two
// Newton steps on g(u) = u^-3 - k, u <- u + u (1 - k u^3) / 3, the first in
// FP32 and the second in FP64.  Each step squares the relative error (e -> 2e^2),
// so the FP64 result is accurate to ~1e-13, i.e. ~1e-9 cycles of a phase of
// 10^3 cycles.
__device__ __forceinline__ double inv_cbrt_f64(double kd) {
    const float kf = (float)kd;
    float uf = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(kf) * (-1.0f / 3.0f));
    uf = fmaf(uf * fmaf(-kf, uf * uf * uf, 1.0f), 1.0f / 3.0f, uf);
    const double u = (double)uf;
    const double r = fma(-kd, u * u * u, 1.0);
    return fma(u * r, 1.0 / 3.0, u);
}

// Higher-accuracy variant (two FP64 Newton steps, full double precision) for
// the gradient kernel, whose phase reaches ~10^6 cycles when t_c is large.
__device__ __forceinline__ double inv_cbrt_f64_full(double kd) {
    double u = inv_cbrt_f64(kd);
    const double r = fma(-kd, u * u * u, 1.0);
    return fma(u * r, 1.0 / 3.0, u);
}

struct PhaseCoef {
    double b1, b2, b3, b5, c0;
};

// Bank templates (t_c = 0): Psi/2pi = b1 u + b2 u^2 + b3 u^3 + b5 u^5 + c0.
__device__ __forceinline__ double spa_cycles_f64(const PhaseCoef& p, double kd) {
    const double u = inv_cbrt_f64(kd);
    const double uu = u * u;
    return fma(u, fma(u, fma(u, fma(uu, p.b5, p.b3), p.b2), p.b1), p.c0);
}

// e^{2 pi i x} for a reduced fraction |x| <= 1/2 with the hardware sine and
// cosine, which take their argument in revolutions (max abs error ~1.3e-7 on
// this range, measured against FP64).
__device__ __forceinline__ cx<float> rotor_rev(float x) {
    return {__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x)};
}

// FP64 phase, rotor in precision T
template <typename T>
__device__ __forceinline__ cx<T> spa_rotor_ph64(const PhaseCoef& p, double kd) {
    double ph = spa_cycles_f64(p, kd);
    ph -= rint(ph);
    if constexpr (sizeof(T) == 4) {
        return rotor_rev((float)ph);
    } else {
        return root_of_unity(ph);
    }
}

// FP32 phase throughout (precision study): u, polynomial and reduction in FP32.
__device__ __forceinline__ cx<float> spa_rotor_ph32(const PhaseCoef& p, float kf) {
    float u = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(kf) * (-1.0f / 3.0f));
    // one FP32 Newton step brings the hardware estimate to ~1 ulp
    float u3 = u * u * u;
    u = fmaf(u * fmaf(-kf, u3, 1.0f), 1.0f / 3.0f, u);
    float uu = u * u;
    float poly = u * fmaf(u, fmaf(u, fmaf(uu, (float)p.b5, (float)p.b3), (float)p.b2), (float)p.b1);
    float ph = poly + (float)p.c0;
    ph -= rintf(ph);
    return rotor_rev(ph);
}

__device__ __forceinline__ PhaseCoef load_coef(const mf_bank_entry& e) {
    return PhaseCoef{e.b1, e.b2, e.b3, e.b5, e.c0};
}

}  // namespace mf
