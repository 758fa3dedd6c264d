// Matched-filter hot path on gfx950: Eq. (1) and Eq. (3) of arXiv:0906.4175
// evaluated per (template, segment) unit as a two-pass inverse DFT.
//
// With N = N1 * N2, bins k = N2 k1 + k2 and times j = j1 + N1 j2,
//   z_j = sum_k2 e^{2 pi i j2 k2 / N2} [ e^{2 pi i j1 k2 / N}
//                                        sum_k1 q_{N2 k1 + k2} e^{2 pi i j1 k1 / N1} ].
// Pass 1 (one work-group per C adjacent columns k2 of one unit) generates the
// stationary-phase rotor e^{+i Psi_k} of the template in registers, forms
// q_k = e^{+i Psi_k} w_k (w_k = 4 df f_k^{-7/6} s_k / S_k, the template
// amplitude folded into the data weight), runs the N1-point column transforms
// in registers and LDS and writes the intermediate once.  Columns only carry
// data for k1 < N1/2 (negative frequencies are zero) and inside [k_lo, k_hi].
// Pass 2 (one work-group per B rows j1) reads each row once, applies the
// four-step factor e^{2 pi i j1 k2 / N} inside its stage twiddles, runs the
// N2-point row transforms and never writes z: it squares |z_j|, counts
// threshold crossings and reduces the maximum with the lowest index.
// Both passes are Stockham auto-sort transforms (radix 16 stages, remainder
// last) whose butterflies live in registers, with LDS between stages.
#include <hip/hip_runtime.h>

#include "filter_shapes.hpp"
#include "filter_tiles.hpp"

namespace mf {

template <size_t A, size_t B>
struct MaxSz {
    static constexpr size_t value = A > B ? A : B;
};

template <typename T, int PH, int MODE, int N1, int N2, int C, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass1_min_waves<T, NT>())))
k_pass1(FilterArgs a) {
    using P = Pass1<T, PH, MODE, N1, N2, C, NT>;
    __shared__ __align__(16) char smem[P::SMEM];
    P::run(a, smem, blockIdx.x, blockIdx.y);
}

template <typename T, bool RAW, int N1, int N2, int B, int NT, int R2, int XS>
__global__ void __launch_bounds__(NT) k_pass2(FilterArgs a) {
    using P = Pass2<T, RAW, N1, N2, B, NT, R2, XS>;
    __shared__ __align__(16) char smem[P::SMEM];
    P::run(a, smem, blockIdx.x, blockIdx.y);
}

// Pipelined step: pass 1 of batch b (a1) and pass 2 of batch b-1 (a2) in one
// launch.  The two roles touch disjoint intermediates and disjoint units, and
// their work-groups are interleaved so that every CU mixes the store-bound
// pass 1 with the arithmetic-bound pass 2.
template <typename T, int PH, int N1, int N2, int C, int B, int NT, int XS>
__global__ void __launch_bounds__(NT) k_step(FilterArgs a1, FilterArgs a2) {
    using P1 = Pass1<T, PH, P1_PRODUCT, N1, N2, C, NT>;
    using P2 = Pass2<T, false, N1, N2, B, NT, 16, XS>;
    __shared__ __align__(16) char smem[MaxSz<P1::SMEM, P2::SMEM>::value];
    constexpr int W1 = N2 / C;  // pass-1 tiles per unit
    constexpr int W2 = N1 / B;  // pass-2 tiles per unit
    const int64_t t1 = a1.units * W1, t2 = a2.units * W2;
    const int64_t m = t1 < t2 ? t1 : t2;
    const int64_t b = blockIdx.x;
    bool first;
    int64_t idx;
    if (b < 2 * m) {
        first = (b & 1) == 0;
        idx = b >> 1;
    } else {
        first = t1 > t2;
        idx = b - m;
    }
    if (first) {
        P1::run(a1, smem, (int)(idx % W1), idx / W1);
    } else {
        P2::run(a2, smem, (int)(idx % W2), idx / W2);
    }
}

// ---------------------------------------------------------------------------
// Finalize: unit peaks -> mf_peak[t][s]
// ---------------------------------------------------------------------------
__global__ void k_finalize32(const unsigned long long* keys, const unsigned int* counts, const mf_bank_entry* bank,
                             int64_t n_tmpl, int64_t n_seg, int64_t n_units, mf_peak* peaks) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    const int64_t t = u % n_tmpl, s = u / n_tmpl;
    const unsigned long long key = keys[u];
    const float zz = __uint_as_float((unsigned int)(key >> 32));
    const unsigned int j = 0xffffffffu - (unsigned int)(key & 0xffffffffull);
    mf_peak p;
    p.rho = sqrt((double)zz) / bank[t].sigma;
    p.j = (int32_t)j;
    p.n_above = (int32_t)counts[u];
    peaks[t * n_seg + s] = p;
}

// One 64-thread work-group per unit: strided scan of the partials, then a
// shuffle reduction (same order-independent comparison as in pass 2).
__global__ void __launch_bounds__(64) k_finalize64(const Partial64* part, int n_part, const mf_bank_entry* bank,
                                                   int64_t n_tmpl, int64_t n_seg, int64_t unit0, mf_peak* peaks) {
    const int64_t u = unit0 + blockIdx.x;
    const int64_t t = u % n_tmpl, s = u / n_tmpl;
    double bzz = -1.0;
    int bj = 0x7fffffff;
    long long cnt = 0;
    for (int i = threadIdx.x; i < n_part; i += 64) {
        const Partial64 p = part[u * n_part + i];
        cnt += p.cnt;
        if (better64(p.zz, p.j, bzz, bj)) {
            bzz = p.zz;
            bj = p.j;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        const double ozz = __shfl_xor(bzz, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (better64(ozz, oj, bzz, bj)) {
            bzz = ozz;
            bj = oj;
        }
    }
    if (threadIdx.x == 0) {
        mf_peak o;
        o.rho = sqrt(bzz) / bank[t].sigma;
        o.j = bj;
        o.n_above = (int32_t)cnt;
        peaks[t * n_seg + s] = o;
    }
}

// ---------------------------------------------------------------------------
// Host side: instantiated shapes, plans and launchers
// ---------------------------------------------------------------------------
size_t cx_bytes(mf_precision prec) { return prec == MF_FP64 ? 16 : 8; }



static void fill(Plan& p, int n1, int n2, int c1, int b2, int r2, int xs) {
    p.n1 = n1;
    p.n2 = n2;
    p.c1 = c1;
    p.b2 = b2;
    p.nt1 = clamp_threads(c1 * n1 / 16);
    p.nt2 = clamp_threads(b2 * n2 / r2);
    p.log2n = ilog2((long long)n1 * n2);
    p.fused = p.nt1 == p.nt2;
    p.xs = xs;
}

int plan_candidates(int log2n, mf_precision prec, Plan* out, int cap) {
    int n = 0;
#define MF_CAND(T, N1, N2, C, B, R2, XS)                                                                \
    if (want(prec, std::is_same<T, double>::value) && ilog2((long long)N1 * N2) == log2n) {            \
        Plan q{};                                                                                      \
        fill(q, N1, N2, C, B, R2, XS);                                                                 \
        q.units = 0;                                                                                   \
        q.prune1 = true; /* bitwise the same results, never slower */                                  \
        for (int f = 0; f < (q.nt1 == q.nt2 && R2 == 16 ? 2 : 1); ++f) {                               \
            for (int pr = 0; pr < (pre0_fits(q) && f == 0 ? 2 : 1); ++pr) {                            \
                for (int ps = 0; ps < (f == 0 ? 2 : 1); ++ps) {                                        \
                    q.fused = f == 1;                                                                  \
                    q.pre0 = pr == 1;                                                                  \
                    q.persist = ps == 1;                                                               \
                    if (out && n < cap) out[n] = q;                                                    \
                    ++n;                                                                               \
                }                                                                                      \
            }                                                                                          \
        }                                                                                              \
    }
    MF_SHAPES(MF_CAND)
#undef MF_CAND
    return n;
}

bool plan_supported(const Plan& q, mf_precision prec) {
#define MF_MATCH(T, N1, N2, C, B, R2, XS)                                                                  \
    if (want(prec, std::is_same<T, double>::value) && q.n1 == N1 && q.n2 == N2 && q.c1 == C && q.b2 == B && \
        q.nt2 == clamp_threads(B * N2 / R2) && q.xs == XS)                                                   \
        return true;
    MF_SHAPES(MF_MATCH)
#undef MF_MATCH
    return false;
}

Plan default_plan(int log2n, mf_precision prec) {
    Plan p{};
    p.log2n = -1;
    bool found = false;
#define MF_FIRST(T, N1, N2, C, B, R2, XS)                                                                         \
    if (!found && want(prec, std::is_same<T, double>::value) && ilog2((long long)N1 * N2) == log2n) {           \
        fill(p, N1, N2, C, B, R2, XS);                                                                            \
        found = true;                                                                                             \
    }
    MF_SHAPES(MF_FIRST)
#undef MF_FIRST
    if (!found) return p;
    // About 8 GiB of intermediates per batch (of the 288 GB of HBM): every
    // pass boundary drains and refills the GPU, so few long launches win.
    // Measured on MI355X (N = 2^20, FP32): 128 units 275k, 512 units 293k
    // units/s; (N = 2^22, 1024x4096, C = 8): 32 units 51k, 128 units 56k.  Separate pass-1 /
    // pass-2 launches measured faster than the pipelined step at large
    // batches, so the step is off by default.
    const size_t bytes_per_unit = ((size_t)1 << log2n) * cx_bytes(prec);
    size_t u = ((size_t)8 << 30) / bytes_per_unit;
    p.units = (int)(u < 1 ? 1 : (u > 4096 ? 4096 : u));
    p.fused = false;
    // Pass 1 skips the stage-0 transform of narrow bands (bitwise the same
    // result).  Measured on MI355X (32768 uneven templates x 4 segments, FP32):
    // pass 1 1.495 -> 1.486 ms per 1024-unit launch; it is bound by its writes.
    p.prune1 = true;
    // Pass 1 applies the row factor of pass 2's first stage (one complex
    // product per element moves from the VALU-bound pass 2 to the store-bound
    // pass 1; in FP32 the product is the same, so the results are bitwise
    // equal).  Measured on MI355X, 32768 uneven templates x 4 segments: pass 2
    // 1.680 -> 1.617 ms per 1024-unit launch (FP32), 2.093 -> 2.054 ms per
    // 512 units (FP64), pass 1 unchanged; 1024 templates x 1 segment:
    // 299k-305k -> 308k-310k units/s.
    p.pre0 = pre0_fits(p);
    // Persistent pass 1 with the heaviest units first, for the FP32 256x4096
    // shape with 32 columns per tile.  Measured on MI355X (A/B, alternating):
    // 32768 x 4 bank pass 1 1.529 -> 1.514 ms per 1024 units (337.8k -> 339.2k
    // units/s), 1024 x 1 unchanged within noise (323k vs 324k); FP64 pass 1
    // 1.51 -> 1.65 ms (its persistent form spills), so FP64 keeps one
    // work-group per tile.
    p.persist = prec != MF_FP64 && p.n1 == 256 && p.n2 == 4096 && p.c1 == 32;
    return p;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FilterLayout filter_layout(const Plan& p, mf_precision prec, int64_t n, int64_t n_tmpl, int64_t n_seg) {
    FilterLayout L{};
    const int64_t n_units = n_tmpl * n_seg;
    const int64_t upb = n_units < p.units ? n_units : p.units;
    L.units_per_batch = upb < 1 ? 1 : upb;
    size_t off = 0;
    L.off_w = off;
    off = align256(off + (size_t)n_seg * (size_t)(n / 2 + 1) * cx_bytes(prec));
    L.off_inter = off;
    // the pipelined step keeps two batches of intermediates (written / being read)
    L.inter_bytes = (size_t)L.units_per_batch * (size_t)n * cx_bytes(prec);
    off = align256(off + (p.fused ? 2 : 1) * L.inter_bytes);
    L.off_keys = off;
    if (prec != MF_FP64) off = align256(off + (size_t)n_units * 8);
    L.off_counts = off;
    if (prec != MF_FP64) off = align256(off + (size_t)n_units * 4);
    L.off_part = off;
    if (prec == MF_FP64) off = align256(off + (size_t)n_units * (size_t)(p.n1 / p.b2) * sizeof(Partial64));
    L.off_tw2 = off;
    if (pass2_uses_tw2(prec, p.n2, p.b2, p.nt2))
        off = align256(off + (size_t)(kTw2Radix - 1) * kTw2Span * cx_bytes(prec));
    // persistent pass 1: work order [units per batch] i32, then the queue counter
    L.off_lpt = off;
    L.off_lpt_ctr = p.persist ? align256(off + (size_t)L.units_per_batch * 4) : off;
    if (p.persist) off = L.off_lpt_ctr + 256;
    L.total = off;
    return L;
}

template <typename T, int PH, int MODE, int N1, int N2, int C>
static hipError_t run_pass1(const FilterArgs& a, hipStream_t s) {
    static_assert(N2 % C == 0 && C <= N2, "pass-1 columns per work-group must tile N2");
    constexpr int NT = clamp_threads(C * N1 / 16);
    dim3 grid(N2 / C, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass1<T, PH, MODE, N1, N2, C, NT>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, bool RAW, int N1, int N2, int B, int R2, int XS>
static hipError_t run_pass2(const FilterArgs& a, hipStream_t s) {
    static_assert(N1 % B == 0 && B <= N1, "pass-2 rows per work-group must tile N1");
    constexpr int NT = clamp_threads(B * N2 / R2);
    dim3 grid(N1 / B, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass2<T, RAW, N1, N2, B, NT, R2, XS>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass1(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s) {
#define MF_P1(T, N1, N2, C, B, R2, XS)                                                                          \
    if (want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C && p.b2 == B) {    \
        if (raw) return run_pass1<T, 0, P1_RAW, N1, N2, C>(a, s);                                              \
        if (a.pre0_r0 > 0) {                                                                                   \
            if (std::is_same<T, float>::value && prec == MF_FP32)                                              \
                return run_pass1<float, 1, P1_PRODUCT_PRE, N1, N2, C>(a, s);                                   \
            return run_pass1<T, 0, P1_PRODUCT_PRE, N1, N2, C>(a, s);                                           \
        }                                                                                                      \
        if (std::is_same<T, float>::value && prec == MF_FP32)                                                  \
            return run_pass1<float, 1, P1_PRODUCT, N1, N2, C>(a, s);                                           \
        return run_pass1<T, 0, P1_PRODUCT, N1, N2, C>(a, s);                                                   \
    }
    MF_SHAPES(MF_P1)
#undef MF_P1
    return hipErrorInvalidValue;
}

hipError_t launch_pass2(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s) {
#define MF_P2(T, N1, N2, C, B, R2, XS)                                                                       \
    if (want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C && p.b2 == B && \
        p.nt2 == clamp_threads(B * N2 / R2) && p.xs == XS)                                                   \
        return raw ? run_pass2<T, true, N1, N2, B, R2, XS>(a, s) : run_pass2<T, false, N1, N2, B, R2, XS>(a, s);
    MF_SHAPES(MF_P2)
#undef MF_P2
    return hipErrorInvalidValue;
}

template <typename T, int PH, int N1, int N2, int C, int B, int XS>
static hipError_t run_step(const FilterArgs& a1, const FilterArgs& a2, hipStream_t s) {
    constexpr int NT1 = clamp_threads(C * N1 / 16), NT2 = clamp_threads(B * N2 / 16);
    if constexpr (NT1 == NT2) {
        const int64_t blocks = a1.units * (N2 / C) + a2.units * (N1 / B);
        if (blocks <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_step<T, PH, N1, N2, C, B, NT1, XS>), dim3((unsigned)blocks), dim3(NT1), 0, s, a1, a2);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const Plan& p, mf_precision prec, const FilterArgs& a1, const FilterArgs& a2, hipStream_t s) {
#define MF_ST(T, N1, N2, C, B, R2, XS)                                                                         \
    if (want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C && p.b2 == B &&   \
        R2 == 16 && p.xs == XS) {                                                                             \
        if (std::is_same<T, float>::value && prec == MF_FP32)                                                  \
            return run_step<float, 1, N1, N2, C, B, XS>(a1, a2, s);                                            \
        return run_step<T, 0, N1, N2, C, B, XS>(a1, a2, s);                                                    \
    }
    MF_SHAPES(MF_ST)
#undef MF_ST
    return hipErrorInvalidValue;
}

// tw2[(r - 1) * span + k] = e^{2 pi i k r / (span R)}, each from its exactly
// reduced argument
template <typename T>
__global__ void k_tw2_fill(cx<T>* tw2) {
    constexpr int M = kTw2Span * kTw2Radix;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (kTw2Radix - 1) * kTw2Span) return;
    const int r = q / kTw2Span + 1, k = q % kTw2Span;
    tw2[q] = root_of_unity((T)((k * r) & (M - 1)) / (T)M);
}

hipError_t launch_tw2_fill(mf_precision prec, void* tw2, hipStream_t s) {
    constexpr int total = (kTw2Radix - 1) * kTw2Span;
    if (prec == MF_FP64)
        hipLaunchKernelGGL(k_tw2_fill<double>, dim3((total + 255) / 256), dim3(256), 0, s, (cx<double>*)tw2);
    else
        hipLaunchKernelGGL(k_tw2_fill<float>, dim3((total + 255) / 256), dim3(256), 0, s, (cx<float>*)tw2);
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan& p, mf_precision prec, const FilterArgs& a, mf_peak* peaks, hipStream_t s) {
    if (prec == MF_FP64) {
        hipLaunchKernelGGL(k_finalize64, dim3((unsigned)a.n_units), dim3(64), 0, s, (const Partial64*)a.partials,
                           p.n1 / p.b2, a.bank, a.n_tmpl, a.n_seg, (int64_t)0, peaks);
    } else {
        const int threads = 256;
        const unsigned blocks = (unsigned)((a.n_units + threads - 1) / threads);
        hipLaunchKernelGGL(k_finalize32, dim3(blocks), dim3(threads), 0, s, a.keys, a.counts, a.bank, a.n_tmpl,
                           a.n_seg, a.n_units, peaks);
    }
    return hipGetLastError();
}

}  // namespace mf
