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
// in registers and LDS, applies the four-step twiddle and writes the
// intermediate once.  Columns only carry data for k1 < N1/2 (negative
// frequencies are zero) and inside [k_lo, k_hi].
// Pass 2 (one work-group per B rows j1) reads each row once, runs the
// N2-point row transforms and never writes z: it squares |z_j|, counts
// threshold crossings and reduces the maximum with the lowest index.
// Both passes are Stockham auto-sort transforms (radix 16 stages, remainder
// last) whose butterflies live in registers, with LDS between stages.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct Partial64 {
    double zz;
    int32_t j;
    int32_t cnt;
};

// Per-(log2 N, precision) shape of the two passes.
template <int LOG2N, typename T>
struct Cfg {
    static constexpr int N1 = 1 << (LOG2N / 2);
    static constexpr int N2 = 1 << (LOG2N - LOG2N / 2);
    static constexpr int BUF1 = std::is_same<T, float>::value ? 16384 : 4096;  // LDS elements, pass 1
    static constexpr int C0 = BUF1 / N1;
    static constexpr int CMAX = std::is_same<T, float>::value ? 16 : 8;
    static constexpr int C = C0 < CMAX ? (C0 < 1 ? 1 : C0) : CMAX;
    static constexpr int NT1R = C * N1 / 16;
    static constexpr int NT1 = NT1R < 64 ? 64 : (NT1R > 1024 ? 1024 : NT1R);
    static constexpr int B0 = 4096 / N2;
    static constexpr int B = B0 > N1 ? N1 : (B0 < 1 ? 1 : B0);
    static constexpr int NT2R = B * N2 / 16;
    static constexpr int NT2 = NT2R < 64 ? 64 : (NT2R > 1024 ? 1024 : NT2R);
};

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
// PH: 0 = FP64 phase, 1 = FP32 phase.  RAW: input is a full N-point spectrum
// (diagnostic inverse DFT) instead of the template x weight product.
template <typename T, int PH, bool RAW, int N1, int N2, int C, int NT>
__global__ void __launch_bounds__(NT) k_pass1(FilterArgs a) {
    constexpr int64_t N = (int64_t)N1 * N2;
    constexpr int NS = num_stages(N1);
    constexpr int LOG2N2 = ilog2(N2);
    __shared__ cx<T> buf[N1 * C];
    __shared__ cx<T> t1[N1];  // e^{+2 pi i m / N1}
    __shared__ cx<T> t2[N2];  // e^{+2 pi i m / N}

    const int tid = threadIdx.x;
    const int k2_0 = blockIdx.x * C;
    const int64_t ul = blockIdx.y;
    const int64_t u = a.unit0 + ul;

    for (int m = tid; m < N1; m += NT) t1[m] = root_of_unity((T)m / (T)N1);
    for (int m = tid; m < N2; m += NT) t2[m] = root_of_unity((T)m / (T)N);

    PhaseCoef coef{};
    int64_t klo = 0, khi = -1;
    const cx<T>* w = nullptr;
    const cx<T>* qin = nullptr;
    if constexpr (RAW) {
        qin = (const cx<T>*)a.raw_in + u * N;
    } else {
        const int64_t t = u % a.n_tmpl;
        const int64_t s = u / a.n_tmpl;
        const mf_bank_entry e = a.bank[t];
        coef = load_coef(e);
        klo = e.k_lo;
        khi = e.k_hi;
        w = (const cx<T>*)a.wgt + s * (N / 2 + 1);
        if (blockIdx.x == 0 && tid == 0 && a.keys != nullptr) {
            a.keys[u] = 0ull;
            a.counts[u] = 0u;
        }
    }
    __syncthreads();

    cx<T>* inter = (cx<T>*)a.inter + ul * N;

    static_for<0, NS>([&](auto S_) {
        constexpr int s = decltype(S_)::value;
        constexpr int R = radix_at(N1, s);
        constexpr int NSPAN = span_before(N1, s);
        constexpr int NBF = C * N1 / R;
        constexpr int BPT = (NBF + NT - 1) / NT;
        cx<T> v[BPT][R];
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int bf = tid + i * NT;
            if (NBF % NT == 0 || bf < NBF) {
                const int c = bf % C;
                const int j = bf / C;
                if constexpr (s == 0) {
                    const int64_t k2 = k2_0 + c;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t k1 = j + r * (N1 / R);
                        if constexpr (RAW) {
                            v[i][r] = qin[k1 * N2 + k2];
                        } else {
                            v[i][r] = cx<T>{T(0), T(0)};
                            if (r < R / 2) {  // k1 < N1/2: non-negative frequencies only
                                const int64_t k = k1 * N2 + k2;
                                if (k >= klo && k <= khi) {
                                    cx<T> rotor;
                                    if constexpr (PH == 0) {
                                        rotor = spa_rotor_ph64<T>(coef, (double)k);
                                    } else {
                                        rotor = spa_rotor_ph32(coef, (float)k);
                                    }
                                    v[i][r] = cmul(rotor, w[k]);
                                }
                            }
                        }
                    }
                } else {
                    const int k = j % NSPAN;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * (N1 / R)) * C + c];
#pragma unroll
                    for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], t1[(r * k) * (N1 / (NSPAN * R))]);
                }
                IDft<R, T>::run(v[i]);
            }
        }
        if constexpr (s == NS - 1) {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = tid + i * NT;
                if (NBF % NT == 0 || bf < NBF) {
                    const int c = bf % C;
                    const int j = bf / C;
                    const int k2 = k2_0 + c;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int j1 = j + r * NSPAN;
                        const int m = j1 * k2;  // < N <= 2^22
                        const cx<T> tw = cmul(t1[m >> LOG2N2], t2[m & (N2 - 1)]);
                        inter[(int64_t)j1 * N2 + k2] = cmul(v[i][r], tw);
                    }
                }
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = tid + i * NT;
                if (NBF % NT == 0 || bf < NBF) {
                    const int c = bf % C;
                    const int j = bf / C;
                    const int idxD = (j / NSPAN) * NSPAN * R + (j % NSPAN);
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[(idxD + r * NSPAN) * C + c] = v[i][r];
                }
            }
            __syncthreads();
        }
    });
}

// ---------------------------------------------------------------------------
// Pass 2
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pad16(int k) { return k + (k >> 4); }

__device__ __forceinline__ bool better64(double zz, int j, double bzz, int bj) {
    const bool an = zz != zz, bn = bzz != bzz;
    if (an != bn) return an;
    if (an) return j < bj;
    return zz > bzz || (zz == bzz && j < bj);
}

template <typename T, bool RAW, int N1, int N2, int B, int NT>
__global__ void __launch_bounds__(NT) k_pass2(FilterArgs a) {
    constexpr int64_t N = (int64_t)N1 * N2;
    constexpr int NS = num_stages(N2);
    constexpr int PN2 = N2 + N2 / 16;
    constexpr int NWAVE = NT / 64;
    constexpr bool F64 = std::is_same<T, double>::value;
    __shared__ cx<T> buf[B * PN2];
    __shared__ cx<T> tw2[N2];  // e^{+2 pi i m / N2}
    __shared__ unsigned long long red_key[NWAVE];
    __shared__ double red_zz[NWAVE];
    __shared__ int red_j[NWAVE];
    __shared__ unsigned int red_cnt[NWAVE];

    const int tid = threadIdx.x;
    const int rb = blockIdx.x;
    const int64_t ul = blockIdx.y;
    const int64_t u = a.unit0 + ul;
    const cx<T>* inter = (const cx<T>*)a.inter + ul * N;

    for (int m = tid; m < N2; m += NT) tw2[m] = root_of_unity((T)m / (T)N2);

    // peak-search state
    T thr2 = T(0);
    double sigma = 1.0;
    float inv_sigma_f = 1.0f;
    int slot = -1;
    if constexpr (!RAW) {
        const int64_t t = u % a.n_tmpl;
        const mf_bank_entry e = a.bank[t];
        sigma = e.sigma;
        inv_sigma_f = e.inv_sigma;
        const double th = a.rho_threshold * sigma;
        thr2 = (T)(th * th);
        const int64_t pub = t * a.n_seg + u / a.n_tmpl;  // public unit id t * n_seg + s
        for (int i = 0; i < a.n_series; ++i)
            if (a.series_units[i] == pub) slot = i;
    }
    unsigned long long best_key = 0ull;
    double best_zz = -1.0;
    int best_j = 0x7fffffff;
    unsigned int cnt = 0u;
    __syncthreads();

    static_for<0, NS>([&](auto S_) {
        constexpr int s = decltype(S_)::value;
        constexpr int R = radix_at(N2, s);
        constexpr int NSPAN = span_before(N2, s);
        constexpr int NBF = B * N2 / R;
        constexpr int BPT = (NBF + NT - 1) / NT;
        constexpr int PER_ROW = N2 / R;
        cx<T> v[BPT][R];
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int bf = tid + i * NT;
            if (NBF % NT == 0 || bf < NBF) {
                const int j = bf % PER_ROW;
                const int b = bf / PER_ROW;
                if constexpr (s == 0) {
                    const int64_t j1 = (int64_t)rb * B + b;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i][r] = inter[j1 * N2 + j + r * PER_ROW];
                } else {
                    const int k = j % NSPAN;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i][r] = buf[b * PN2 + pad16(j + r * PER_ROW)];
#pragma unroll
                    for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw2[(r * k) * (N2 / (NSPAN * R))]);
                }
                IDft<R, T>::run(v[i]);
            }
        }
        if constexpr (s == NS - 1) {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = tid + i * NT;
                if (NBF % NT == 0 || bf < NBF) {
                    const int j = bf % PER_ROW;
                    const int b = bf / PER_ROW;
                    const int j1 = rb * B + b;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int j2 = j + r * NSPAN;
                        const int jg = j1 + N1 * j2;
                        if constexpr (RAW) {
                            ((cx<T>*)a.raw_out)[u * N + jg] = v[i][r];
                        } else {
                            const T zz = norm2(v[i][r]);
                            if (slot >= 0) {
                                if constexpr (F64) {
                                    ((double*)a.rho)[(int64_t)slot * N + jg] = sqrt(zz) / sigma;
                                } else {
                                    ((float*)a.rho)[(int64_t)slot * N + jg] = sqrtf(zz) * inv_sigma_f;
                                }
                            }
                            if (jg >= a.j_begin && jg < a.j_end) {
                                cnt += (zz >= thr2) ? 1u : 0u;
                                if constexpr (F64) {
                                    if (better64(zz, jg, best_zz, best_j)) {
                                        best_zz = zz;
                                        best_j = jg;
                                    }
                                } else {
                                    const unsigned long long key =
                                        ((unsigned long long)__float_as_uint(zz) << 32) |
                                        (unsigned long long)(0xffffffffu - (unsigned int)jg);
                                    best_key = key > best_key ? key : best_key;
                                }
                            }
                        }
                    }
                }
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = tid + i * NT;
                if (NBF % NT == 0 || bf < NBF) {
                    const int j = bf % PER_ROW;
                    const int b = bf / PER_ROW;
                    const int idxD = (j / NSPAN) * NSPAN * R + (j % NSPAN);
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[b * PN2 + pad16(idxD + r * NSPAN)] = v[i][r];
                }
            }
            __syncthreads();
        }
    });

    if constexpr (!RAW) {
        // work-group reduction: wave shuffles, then one LDS slot per wave
        const int lane = tid & 63;
        const int wave = tid >> 6;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off, 64);
            if constexpr (F64) {
                const double ozz = __shfl_xor(best_zz, off, 64);
                const int oj = __shfl_xor(best_j, off, 64);
                if (better64(ozz, oj, best_zz, best_j)) {
                    best_zz = ozz;
                    best_j = oj;
                }
            } else {
                const unsigned long long o = __shfl_xor(best_key, off, 64);
                best_key = o > best_key ? o : best_key;
            }
        }
        if (lane == 0) {
            red_cnt[wave] = cnt;
            red_key[wave] = best_key;
            red_zz[wave] = best_zz;
            red_j[wave] = best_j;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < NWAVE; ++w) {
                cnt += red_cnt[w];
                if constexpr (F64) {
                    if (better64(red_zz[w], red_j[w], best_zz, best_j)) {
                        best_zz = red_zz[w];
                        best_j = red_j[w];
                    }
                } else {
                    best_key = red_key[w] > best_key ? red_key[w] : best_key;
                }
            }
            if constexpr (F64) {
                Partial64* part = (Partial64*)a.partials + ul * (N1 / B) + rb;
                *part = Partial64{best_zz, best_j, (int32_t)cnt};
            } else {
                atomicMax(a.keys + u, best_key);
                if (cnt) atomicAdd(a.counts + u, cnt);
            }
        }
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

__global__ void k_finalize64(const Partial64* part, int n_part, const mf_bank_entry* bank, int64_t n_tmpl,
                             int64_t n_seg, int64_t unit0, int64_t units, mf_peak* peaks) {
    const int64_t ul = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ul >= units) return;
    const int64_t u = unit0 + ul;
    const int64_t t = u % n_tmpl, s = u / n_tmpl;
    double bzz = -1.0;
    int bj = 0x7fffffff;
    long long cnt = 0;
    for (int i = 0; i < n_part; ++i) {
        const Partial64 p = part[ul * n_part + i];
        cnt += p.cnt;
        if (better64(p.zz, p.j, bzz, bj)) {
            bzz = p.zz;
            bj = p.j;
        }
    }
    mf_peak o;
    o.rho = sqrt(bzz) / bank[t].sigma;
    o.j = bj;
    o.n_above = (int32_t)cnt;
    peaks[t * n_seg + s] = o;
}

// ---------------------------------------------------------------------------
// Host side: plans and launchers
// ---------------------------------------------------------------------------
size_t cx_bytes(mf_precision prec) { return prec == MF_FP64 ? 16 : 8; }

template <int LOG2N, typename T>
static void fill_plan(Plan& p) {
    using K = Cfg<LOG2N, T>;
    p.log2n = LOG2N;
    p.n1 = K::N1;
    p.n2 = K::N2;
    p.c1 = K::C;
    p.nt1 = K::NT1;
    p.b2 = K::B;
    p.nt2 = K::NT2;
}

#define MF_FOR_EACH_LOG2N(X) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22)

Plan default_plan(int log2n, mf_precision prec) {
    Plan p{};
    switch (log2n) {
#define MF_CASE(L)                                   \
    case L:                                          \
        if (prec == MF_FP64)                         \
            fill_plan<L, double>(p);                 \
        else                                         \
            fill_plan<L, float>(p);                  \
        break;
        MF_FOR_EACH_LOG2N(MF_CASE)
#undef MF_CASE
        default:
            p.log2n = -1;
            return p;
    }
    // keep about 64 MiB of intermediates in flight (fits the 256 MiB last-level cache)
    const size_t bytes_per_unit = ((size_t)1 << log2n) * cx_bytes(prec);
    size_t u = ((size_t)64 << 20) / bytes_per_unit;
    p.units = (int)(u < 1 ? 1 : (u > 4096 ? 4096 : u));
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
    off = align256(off + (size_t)L.units_per_batch * (size_t)n * cx_bytes(prec));
    L.off_keys = off;
    if (prec != MF_FP64) off = align256(off + (size_t)n_units * 8);
    L.off_counts = off;
    if (prec != MF_FP64) off = align256(off + (size_t)n_units * 4);
    L.off_part = off;
    if (prec == MF_FP64) off = align256(off + (size_t)L.units_per_batch * (size_t)(p.n1 / p.b2) * sizeof(Partial64));
    L.total = off;
    return L;
}

template <int LOG2N, typename T, int PH, bool RAW>
static hipError_t run_pass1(const FilterArgs& a, hipStream_t s) {
    using K = Cfg<LOG2N, T>;
    dim3 grid(K::N2 / K::C, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass1<T, PH, RAW, K::N1, K::N2, K::C, K::NT1>), grid, dim3(K::NT1), 0, s, a);
    return hipGetLastError();
}

template <int LOG2N, typename T, bool RAW>
static hipError_t run_pass2(const FilterArgs& a, hipStream_t s) {
    using K = Cfg<LOG2N, T>;
    dim3 grid(K::N1 / K::B, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass2<T, RAW, K::N1, K::N2, K::B, K::NT2>), grid, dim3(K::NT2), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass1(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s) {
    switch (p.log2n) {
#define MF_CASE(L)                                                                  \
    case L:                                                                         \
        if (prec == MF_FP64)                                                        \
            return raw ? run_pass1<L, double, 0, true>(a, s) : run_pass1<L, double, 0, false>(a, s); \
        if (raw) return run_pass1<L, float, 0, true>(a, s);                          \
        return prec == MF_FP32 ? run_pass1<L, float, 1, false>(a, s) : run_pass1<L, float, 0, false>(a, s);
        MF_FOR_EACH_LOG2N(MF_CASE)
#undef MF_CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_pass2(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s) {
    switch (p.log2n) {
#define MF_CASE(L)                                                                                 \
    case L:                                                                                        \
        if (prec == MF_FP64) return raw ? run_pass2<L, double, true>(a, s) : run_pass2<L, double, false>(a, s); \
        return raw ? run_pass2<L, float, true>(a, s) : run_pass2<L, float, false>(a, s);
        MF_FOR_EACH_LOG2N(MF_CASE)
#undef MF_CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const Plan& p, mf_precision prec, const FilterArgs& a, mf_peak* peaks, hipStream_t s) {
    if (prec == MF_FP64) {
        const int threads = 64;
        const unsigned blocks = (unsigned)((a.units + threads - 1) / threads);
        hipLaunchKernelGGL(k_finalize64, dim3(blocks), dim3(threads), 0, s, (const Partial64*)a.partials,
                           p.n1 / p.b2, a.bank, a.n_tmpl, a.n_seg, a.unit0, a.units, peaks);
    } else {
        const int threads = 256;
        const unsigned blocks = (unsigned)((a.n_units + threads - 1) / threads);
        hipLaunchKernelGGL(k_finalize32, dim3(blocks), dim3(threads), 0, s, a.keys, a.counts, a.bank, a.n_tmpl,
                           a.n_seg, a.n_units, peaks);
    }
    return hipGetLastError();
}

}  // namespace mf
