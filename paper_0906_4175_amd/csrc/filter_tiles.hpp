// Tile building blocks of the two-pass inverse DFT shared by the matched
// filter (Eq. (1), Eq. (3)) and its chi^2 band variant (Eq. (5)) of
// arXiv:0906.4175: stage twiddle tables, the pass-1 column tile and the
// pass-2 row tile.  See k_filter.hip for the decomposition.
#pragma once

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

// Weight of the input-index digit that stage s of an L-point Stockham
// transform consumes: L / (span * radix).
__host__ __device__ constexpr int digit_weight(int L, int s, int maxr = 16) {
    return L / (span_before(L, s, maxr) * radix_at(L, s, maxr));
}

// Stage twiddle tables, one contiguous table per stage s >= 1:
// e^{+2 pi i k / (span_s R_s)} for k < span_s, so that the lanes of a
// butterfly row read consecutive entries.
__host__ __device__ constexpr int tw_offset(int L, int s, int maxr = 16) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += span_before(L, i, maxr);
    return off;
}
__host__ __device__ constexpr int tw_total(int L, int maxr = 16) { return tw_offset(L, num_stages(L, maxr), maxr) + 1; }

template <typename T, int L, int MAXR = 16>
__device__ __forceinline__ void fill_stage_twiddles(cx<T>* tw, int tid, int nt) {
    static_for<1, num_stages(L, MAXR)>([&](auto S_) {
        constexpr int s = decltype(S_)::value;
        constexpr int SPAN = span_before(L, s, MAXR);
        constexpr int OFF = tw_offset(L, s, MAXR);
        constexpr T INV_M = (T)1 / (T)(SPAN * radix_at(L, s, MAXR));  // a power of two: exact
        for (int k = tid; k < SPAN; k += nt) tw[OFF + k] = root_of_unity((T)k * INV_M);
    });
}

// p[r] = w^r for r = 0..R-1 by a binary tree of products (depth log2 r).
template <int R, typename T>
__device__ __forceinline__ void powers(cx<T> w, cx<T>* p) {
    p[0] = cx<T>{T(1), T(0)};
    if constexpr (R > 1) p[1] = w;
#pragma unroll
    for (int r = 2; r < R; ++r) p[r] = cmul(p[r / 2], p[r - r / 2]);
}

__host__ __device__ constexpr int pad16(int k) { return k + (k >> 4); }
__host__ __device__ constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

// Event keys: larger key = larger |z|^2, then lower index.  FP32 keeps the
// float bits and the sample index; FP64 keeps |z|^2 to 36 mantissa bits and
// the index inside the window (windows of at most 2^16 samples).
__device__ __forceinline__ unsigned long long event_key32(float zz, unsigned int j) {
    return ((unsigned long long)__float_as_uint(zz) << 32) | (unsigned long long)(0xffffffffu - j);
}
__device__ __forceinline__ unsigned long long event_key64(double zz, unsigned int j_in_window) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(zz) & ~0xffffull;
    return b | (unsigned long long)(0xffffu - j_in_window);
}

__device__ __forceinline__ bool better64(double zz, int j, double bzz, int bj) {
    const bool an = zz != zz, bn = bzz != bzz;
    if (an != bn) return an;
    if (an) return j < bj;
    return zz > bzz || (zz == bzz && j < bj);
}

// Template and segment of unit u = s n_tmpl + t with one division.  The
// operands are wave-uniform, so the 64-bit division runs on the scalar unit
// (a 32-bit one would go through the vector unit's float reciprocal).
__device__ __forceinline__ void unit_split(int64_t u, int64_t n_tmpl, int64_t& t, int64_t& s) {
    s = u / n_tmpl;
    t = u - s * n_tmpl;
}

// digit_weight(L, st) for a run-time stage index st < num_stages(L) (a chain
// of selects between compile-time constants instead of a loop).
template <int L, int MAXR>
__device__ __forceinline__ int digit_weight_rt(int st) {
    int w = 0;
    static_for<0, num_stages(L, MAXR)>([&](auto S_) {
        if (st == decltype(S_)::value) w = digit_weight(L, decltype(S_)::value, MAXR);
    });
    return w;
}

// ---------------------------------------------------------------------------
// Pass 1 tile: C adjacent columns k2 of one unit.
// PH: 0 = FP64 phase, 1 = FP32 phase.  MODE: P1_PRODUCT transforms the
// template x weight product; P1_RAW a full N-point spectrum (diagnostic
// inverse DFT); P1_BAND transforms only the product's part inside one chi^2
// band and stores the other bands' parts in their slots (below).
// Output: Y[j1][k2] = sum_k1 q[N2 k1 + k2] e^{2 pi i j1 k1 / N1}.
// ---------------------------------------------------------------------------
// P1_PRODUCT_PRE is P1_PRODUCT that also applies the row factor of pass 2's
// first stage to its output (FilterArgs::pre0_r0); a separate instantiation,
// so the plain product keeps its register budget.
//
// chi^2 band mode: every non-empty band l but the transformed one keeps its
// product in a slot, a copy of the bins [s_l, s_l + n_l N2) with s_l = e_l
// rounded down to a multiple of kSlotAlign and n_l = ceil((e_{l+1} - s_l) / N2),
// zero outside the band.  The band table of a template holds the edges
// e_0..e_p, the transformed band's index and the slot starts (prefix sums of
// n_l N2, p + 1 entries); a unit's slots take at most band_slot_stride
// complex values.
enum Pass1Mode { P1_PRODUCT = 0, P1_RAW = 1, P1_BAND = 2, P1_PRODUCT_PRE = 3 };

constexpr int kSlotAlign = 16;
constexpr int kMaxBands = 64;
__host__ __device__ constexpr int band_tab_stride(int p) { return 2 * p + 3; }
// sum_l n_l N2 <= sum_l (e_{l+1} - e_l + kSlotAlign - 1 + N2 - 1) <= n/2 + p (N2 + kSlotAlign)
__host__ __device__ constexpr int64_t band_slot_stride(int64_t n, int n2, int p) {
    return n / 2 + (int64_t)p * (n2 + kSlotAlign);
}

template <typename T, int PH, int MODE, int N1, int N2, int C, int NT>
struct Pass1 {
    static constexpr bool RAW = MODE == P1_RAW;
    static constexpr int64_t N = (int64_t)N1 * N2;
    static constexpr int NS = num_stages(N1);
    static constexpr int TW = tw_total(N1);
    // FP32: stage 1 reads its factors w^(k r), k < 16, r < R1, from a full
    // table (the same for every column) instead of forming powers per
    // butterfly (FP64 keeps the powers: its roots cost more than the products)
    static constexpr bool USE_T1 = NS >= 2 && sizeof(T) == 4;
    static constexpr int R1 = NS >= 2 ? radix_at(N1, 1) : 1;
    static constexpr int T1 = USE_T1 ? 16 * R1 : 0;
    // XS: the stages exchange real parts, then imaginary parts, through N1 C
    // scalars (half the LDS); every thread holds EPT = C N1 / NT values at every
    // stage, so the next stage's inputs are read into one array of that size.
    static constexpr bool all_full() {
        for (int s = 0; s < NS; ++s)
            if ((C * N1 / radix_at(N1, s)) % NT != 0) return false;
        return true;
    }
    static constexpr bool XS = NS > 1 && all_full();
    static constexpr int EPT = C * N1 / NT;
    // Narrow bands (product rows k1 < N1/16 only: k_hi < N2 N1 / 16, templates
    // heavier than about 17 M_sun at N1 = 256): every stage-0 butterfly has a
    // single non-zero input, so its 16 outputs all equal that input and stage 1
    // reads the products directly (no stage-0 transform, one LDS value per row).
    static constexpr bool PRODUCT = MODE == P1_PRODUCT || MODE == P1_PRODUCT_PRE;
    static constexpr bool NARROW_OK = PRODUCT && XS && NS == 2 && radix_at(N1, 0) == 16 &&
                                      radix_at(N1, 1) == 16 && C * N1 / 16 == NT;
    static constexpr size_t BUF_BYTES = (size_t)N1 * C * (XS ? sizeof(T) : sizeof(cx<T>));
    // PRE (product mode, FilterArgs::pre0_r0 > 0): the factor pass 2's first
    // stage would apply to this tile's columns, one per output row j1
    static constexpr int PRE = MODE == P1_PRODUCT_PRE ? N1 : 0;
    // P1_BAND: the template's band edges and slot starts
    static constexpr int BANDI = MODE == P1_BAND ? 2 * (kMaxBands + 1) : 0;
    static constexpr size_t SMEM = BUF_BYTES + (size_t)(TW + T1 + PRE) * sizeof(cx<T>) + (size_t)BANDI * sizeof(int);

    __device__ static void run(const FilterArgs& a, char* smem, int tile, int64_t ul) {
        cx<T>* buf = (cx<T>*)smem;
        T* fbuf = (T*)smem;
        cx<T>* tw = (cx<T>*)(smem + BUF_BYTES);
        cx<T>* t1 = tw + TW;  // [k][r]
        cx<T>* tpre = t1 + T1;  // PRE: [j1]
        [[maybe_unused]] int* bedge = (int*)(tpre + PRE);  // P1_BAND: e_0..e_p
        [[maybe_unused]] int* bslot = bedge + kMaxBands + 1;  // P1_BAND: slot starts
        [[maybe_unused]] cx<T> carry[XS ? EPT : 1];
        const int tid = threadIdx.x;
        const int k2_0 = tile * C;
        const int64_t u = a.unit0 + ul;

        PhaseCoef coef{};
        // bins of the non-negative half: k < N/2 <= 2^21, 32-bit arithmetic
        int klo = 0, khi = -1;
        const cx<T>* w = nullptr;
        const cx<T>* qin = nullptr;
        int blo = 0, bhi = 0;      // P1_BAND: the transformed band [blo, bhi)
        cx<T>* slots = nullptr;    // P1_BAND: this unit's band slots
        [[maybe_unused]] const int nb = a.p_bands;
        if constexpr (RAW) {
            qin = (const cx<T>*)a.raw_in + u * N;
        } else {
            int64_t t, s;
            unit_split(u, a.n_tmpl, t, s);
            const mf_bank_entry e = a.bank[t];
            coef = load_coef(e);
            klo = e.k_lo;
            khi = e.k_hi;
            w = (const cx<T>*)a.wgt + s * (N / 2 + 1);
            if constexpr (MODE == P1_BAND) {
                const int32_t* tab = a.band_tab + t * band_tab_stride(nb);
                const int wb = tab[nb + 1];
                blo = tab[wb];
                bhi = tab[wb + 1];
                slots = (cx<T>*)a.qbuf + ul * band_slot_stride(N, N2, nb);
                for (int q = tid; q <= nb; q += NT) {
                    bedge[q] = tab[q];
                    bslot[q] = tab[nb + 2 + q];
                }
                __syncthreads();
                // the slot bins outside their band: the head [s_l, e_l) lies in row
                // e_l / N2, the tail [e_{l+1}, s_l + n_l N2) (shorter than N2) in rows
                // e_{l+1} / N2 and the next; this tile writes the zeros of its columns
                for (int q = tid; q < nb * 3 * C; q += NT) {
                    const int l = q / (3 * C), d = (q / C) % 3, c = q % C;
                    const int sb0 = bslot[l], len = bslot[l + 1] - sb0;
                    const int e0 = bedge[l], e1 = bedge[l + 1];
                    const int sl = e0 & ~(kSlotAlign - 1);
                    const int row = d == 0 ? e0 / N2 : e1 / N2 + d - 1;
                    const int k = row * N2 + k2_0 + c;
                    const bool pad = d == 0 ? (k >= sl && k < e0) : (k >= e1 && k < sl + len);
                    if (len > 0 && pad) slots[sb0 + (k - sl)] = cx<T>{T(0), T(0)};
                }
            }
            if (tile == 0 && tid == 0 && a.keys != nullptr) {
                a.keys[u] = 0ull;
                a.counts[u] = 0u;
            }
        }
        cx<T>* inter = (cx<T>*)a.inter + ul * N;
        [[maybe_unused]] const bool narrow = NARROW_OK && a.prune1 != 0 && khi < (N1 / 16) * N2;
        // PRE: row j1 of this tile's columns k2 (all in one block of N2/R0, so
        // rr = floor(k2 / (N2/R0)) is the tile's) takes e^{2 pi i j1 rr / (N1 R0)}
        [[maybe_unused]] constexpr bool pre = PRE > 0;
        auto fill_pre = [&]() {
            if constexpr (PRE > 0) {
                if (pre) {
                    const int r0 = a.pre0_r0;
                    const int rr = k2_0 / (N2 / r0);
                    const int mask = N1 * r0 - 1;  // N1 R0 is a power of two
                    const T inv = (T)1 / (T)(N1 * r0);
                    for (int q = tid; q < N1; q += NT) tpre[q] = root_of_unity((T)((q * rr) & mask) * inv);
                }
            }
        };

        static_for<0, NS>([&](auto S_) {
            constexpr int s = decltype(S_)::value;
            constexpr int R = radix_at(N1, s);
            constexpr int NSPAN = span_before(N1, s);
            constexpr int NBF = C * N1 / R;
            constexpr int BPT = (NBF + NT - 1) / NT;
            if constexpr (s == 0 && NARROW_OK) {
                if (narrow) {  // uniform over the work-group
                    // thread (row k1 = j, column c): the product of its bin, or zero
                    const int c = tid % C, j = tid / C;
                    const int k = j * N2 + k2_0 + c;
                    cx<T> x{T(0), T(0)};
                    const cx<T> wk = w[(k >= klo && k <= khi) ? k : 0];
                    if (k >= klo && k <= khi) {
                        cx<T> rotor;
                        if constexpr (PH == 0) {
                            rotor = spa_rotor_ph64<T>(coef, (double)k);
                        } else {
                            rotor = spa_rotor_ph32(coef, (float)k);
                        }
                        x = cmul(rotor, wk);
                    }
                    fill_stage_twiddles<T, N1>(tw, tid, NT);
                    constexpr T INV_M1 = (T)1 / (T)(16 * R1);
                    for (int q = tid; q < T1; q += NT) {
                        const int kk = q / R1, r = q % R1;
                        t1[q] = root_of_unity((T)((kk * r) & (16 * R1 - 1)) * INV_M1);
                    }
                    fill_pre();
                    // stage-1 input r of every butterfly of column c is the product of row r
#pragma unroll
                    for (int part = 0; part < 2; ++part) {
                        __syncthreads();
                        fbuf[j * C + c] = part ? x.y : x.x;
                        __syncthreads();
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            if (part) carry[r].y = fbuf[r * C + c];
                            else carry[r].x = fbuf[r * C + c];
                        }
                    }
                    return;
                }
            }
            cx<T> v[BPT][R];
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = tid + i * NT;
                if (NBF % NT == 0 || bf < NBF) {
                    const int c = bf % C;
                    const int j = bf / C;
                    if constexpr (s == 0) {
                        const int64_t k2 = k2_0 + c;
                        // every weight load of the butterfly is issued before the
                        // first rotor (bins outside [k_lo, k_hi] load bin 0 and are
                        // discarded), so a wave waits for memory once
                        cx<T> wk[RAW ? 1 : R / 2];
                        if constexpr (!RAW) {
#pragma unroll
                            for (int r = 0; r < R / 2; ++r) {
                                const int k = (j + r * (N1 / R)) * N2 + (int)k2;
                                wk[r] = w[(k >= klo && k <= khi) ? k : 0];
                            }
                        }
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int64_t k1 = j + r * (N1 / R);
                            if constexpr (RAW) {
                                v[i][r] = qin[k1 * N2 + k2];
                            } else {
                                v[i][r] = cx<T>{T(0), T(0)};
                                if (r < R / 2) {  // k1 < N1/2: non-negative frequencies only
                                    const int k = (int)k1 * N2 + (int)k2;
                                    if (k >= klo && k <= khi) {
                                        cx<T> rotor;
                                        if constexpr (PH == 0) {
                                            rotor = spa_rotor_ph64<T>(coef, (double)k);
                                        } else {
                                            rotor = spa_rotor_ph32(coef, (float)k);
                                        }
                                        v[i][r] = cmul(rotor, wk[r]);
                                    }
                                    if constexpr (MODE == P1_BAND) {
                                        if (k < blo || k >= bhi) {
                                            if (k >= bedge[0] && k < bedge[nb]) {
                                                // the band of k: e_l <= k < e_{l+1} (bisection, e_0 <= k < e_p)
                                                int lo = 0, hi = nb;
                                                while (hi - lo > 1) {
                                                    const int mid = (lo + hi) >> 1;
                                                    if (bedge[mid] <= k) lo = mid; else hi = mid;
                                                }
                                                slots[bslot[lo] + (k - (bedge[lo] & ~(kSlotAlign - 1)))] = v[i][r];
                                            }
                                            v[i][r] = cx<T>{T(0), T(0)};
                                        }
                                    }
                                }
                            }
                        }
                    } else {
                        const int k = j % NSPAN;
                        if constexpr (XS) {
#pragma unroll
                            for (int r = 0; r < R; ++r) v[i][r] = carry[i * R + r];
                        } else {
                            const cx<T>* src = buf + j * C + c;
#pragma unroll
                            for (int r = 0; r < R; ++r) v[i][r] = src[r * (N1 / R) * C];
                        }
                        cx<T> p[R];
                        if constexpr (s == 1 && USE_T1) {
                            static_assert(NSPAN == 16 && R == R1, "stage-1 table shape");
#pragma unroll
                            for (int r = 1; r < R; ++r) p[r] = t1[k * R + r];
                        } else {
                            powers<R>(tw[tw_offset(N1, s) + k], p);
                        }
#pragma unroll
                        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], p[r]);
                    }
                    IDft<R, T>::run(v[i]);
                }
            }
            if constexpr (s == 0) {
                fill_stage_twiddles<T, N1>(tw, tid, NT);
                // each factor from its exactly reduced argument (k r mod 16 R1) / (16 R1)
                constexpr T INV_M1 = (T)1 / (T)(16 * R1);  // a power of two: exact
                for (int q = tid; q < T1; q += NT) {
                    const int k = q / R1, r = q % R1;
                    t1[q] = root_of_unity((T)((k * r) & (16 * R1 - 1)) * INV_M1);
                }
                fill_pre();
            }
            if constexpr (s == NS - 1) {
#pragma unroll
                for (int i = 0; i < BPT; ++i) {
                    const int bf = tid + i * NT;
                    if (NBF % NT == 0 || bf < NBF) {
                        const int c = bf % C;
                        const int j = bf / C;
                        cx<T>* dst = inter + (int64_t)j * N2 + k2_0 + c;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            cx<T> y = v[i][r];
                            if constexpr (PRE > 0) {
                                if (pre) y = cmul(y, tpre[j + r * NSPAN]);  // output r is row j1 = j + r NSPAN
                            }
                            if constexpr (MODE == P1_BAND) {
                                // band mode: pass 2 reads the batch back from the last-level cache
                                dst[(int64_t)r * NSPAN * N2] = y;
                            } else {
                                // non-temporal: the batch (8 GiB) is read back only by pass 2.  With
                                // the non-temporal pass-2 loads, measured on MI355X: 32768 x 4 bank
                                // 332k -> 338k units/s, 1024 x 1 308k -> 318k.
                                __builtin_nontemporal_store(vec2<T>{y.x, y.y}, (vec2<T>*)&dst[(int64_t)r * NSPAN * N2]);
                            }
                        }
                    }
                }
            } else if constexpr (XS) {
                constexpr int RN = radix_at(N1, s + 1);
                constexpr int BPTN = C * N1 / RN / NT;
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < BPT; ++i) {
                        const int bf = tid + i * NT;
                        const int c = bf % C;
                        const int j = bf / C;
                        const int idxD = (j / NSPAN) * NSPAN * R + (j % NSPAN);
                        T* dst = fbuf + idxD * C + c;
#pragma unroll
                        for (int r = 0; r < R; ++r) dst[r * NSPAN * C] = part ? v[i][r].y : v[i][r].x;
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < BPTN; ++i) {
                        const int bf = tid + i * NT;
                        const int c = bf % C;
                        const int j = bf / C;
                        const T* src = fbuf + j * C + c;
#pragma unroll
                        for (int r = 0; r < RN; ++r) {
                            if (part) carry[i * RN + r].y = src[r * (N1 / RN) * C];
                            else carry[i * RN + r].x = src[r * (N1 / RN) * C];
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
                        cx<T>* dst = buf + idxD * C + c;
#pragma unroll
                        for (int r = 0; r < R; ++r) dst[r * NSPAN * C] = v[i][r];
                    }
                }
                __syncthreads();
            }
        });
    }
};

// ---------------------------------------------------------------------------
// Bank-conflict-free exchange layouts of a 4096-point row transformed by three
// radix-16 stages with one butterfly (16 values) per thread.  With x = 256 h +
// 16 m + l, a wave writes x = 16 j + r after stage 0 and 256 (j >> 4) + 16 r +
// (j & 15) after stage 1 (r fixed per instruction, j over the lanes), and reads
// x = j + 256 r before stages 1 and 2.  No padding serves the first write and
// the reads together, so the first exchange stores x at x ^ m ^ ((h & 3) << 4)
// (an XOR swizzle: l ^ m and the low bits of m ^ h differ across the 64 lanes
// of every access); the second pads 16 slots per 256 (x + 16 h), whose offsets
// stay immediates.  Every access touches distinct banks for 64 banks of one
// lane each and for 32 banks per half-wave (so also for 8-byte elements).
// The buffer needs 4336 slots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cf_wr0(int j) {  // slot of x = 16 j; x = 16 j + r is at cf_wr0(j) ^ r
    return (16 * j) ^ (j & 15) ^ (((j >> 4) & 3) << 4);
}
__device__ __forceinline__ int cf_rd0(int j, int r) {  // slot of x = j + 256 r, j < 256 (first layout)
    return 256 * r + ((j ^ (j >> 4)) ^ ((r & 3) << 4));
}
__device__ __forceinline__ int cf_wr1(int j, int r) {  // slot of x = 256 (j >> 4) + 16 r + (j & 15)
    return 272 * (j >> 4) + (j & 15) + 16 * r;
}
__device__ __forceinline__ int cf_rd1(int j, int r) { return j + 272 * r; }  // x = j + 256 r (second layout)
constexpr int kCfSlots = 4336;

// ---------------------------------------------------------------------------
// Pass 2 tile: B rows j1 of one unit.
// Row j1: z[j1 + N1 j2] = sum_k2 (Y[j1][k2] t^k2) e^{2 pi i j2 k2 / N2}, t = e^{2 pi i j1 / N}.
// The four-step factor t^k2 is folded into the stage twiddles: writing k2 in
// the mixed radix of the stages, stage s multiplies its input r by
// (w_s t^{weight_s})^r with weight_s = N2 / (span_s R_s), so no separate
// twiddle pass is needed and the result is exact (not only up to a phase).
// The last stage squares |z| and reduces (max |z|^2, lowest index, count).
// ---------------------------------------------------------------------------
template <typename T, bool RAW, int N1, int N2, int B, int NT, int MAXR = 16, int XS = 0>
struct Pass2 {
    static constexpr int64_t N = (int64_t)N1 * N2;
    static constexpr int NS = num_stages(N2, MAXR);
    static constexpr int PN2 = pad16(N2);
    static constexpr int NWAVE = NT / 64;
    static constexpr int TW = tw_total(N2, MAXR);
    static constexpr bool F64 = std::is_same<T, double>::value;
    static constexpr int R0 = radix_at(N2, 0, MAXR);
    // XS >= 1: exchange the real parts, then the imaginary parts, through a
    // buffer of B * PN2 scalars (half the LDS, so more work-groups per CU,
    // for two more barriers per exchange); needs the same radix at every stage.
    // XS == 2 (4096-point rows of three radix-16 stages, one row per
    // work-group): bank-conflict-free layouts instead of the padding (below).
    static constexpr bool SPLIT = XS >= 1;
    static constexpr bool CF = XS == 2;
    static_assert(!SPLIT || (N2 == ipow_c(MAXR, NS) && NS > 1), "split exchange needs one radix at every stage");
    static_assert(!CF || (N2 == 4096 && MAXR == 16 && B == 1 && NT == 256 && PN2 >= kCfSlots),
                  "conflict-free layouts: 4096-point rows");
    // FP32 peak search over the full series when every thread holds exactly
    // one last-stage butterfly: each thread keeps its largest |z|^2 bits, the
    // work-group takes the maximum, and only threads that hold it look for
    // its lowest index (instead of every thread building a 64-bit key).
    static constexpr int RL = radix_at(N2, NS - 1, MAXR);
    static constexpr int SPAN_L = span_before(N2, NS - 1, MAXR);
    static constexpr bool DEFER = !F64 && !RAW && B * N2 / RL == NT;
    // TAB2 (FP64, 4096-point rows, three radix-16 stages, one row per
    // work-group): stage 0 applies the whole four-step factor
    // t^{k2} = t^j t^{256 r}, so the factors of stages 1 and 2, w^(k r), no
    // longer depend on the row and come from tables (stage 1: 15 x 16 entries
    // in LDS; stage 2: 15 x 256 entries in the workspace, filled once per call)
    // instead of products of powers.  In FP32 the table loads measured slower
    // than the products they replace.
    static constexpr bool TAB2 =
        F64 && !RAW && N2 == kTw2Span * kTw2Radix && MAXR == 16 && B == 1 && NT == 256 && NS == 3;
    static constexpr int TWL = TAB2 ? 15 * 16 : TW;
    // F1 (FP32 and the other non-TAB2 shapes of at least two stages, one
    // table entry per thread): stage 1 reads its factors (w_1 t^{weight_1})^r
    // from a per-row table [B][R1 - 1][span_1] of exactly reduced roots,
    // filled once per work-group during stage 0, instead of a product tree of
    // powers per butterfly (15 table reads for 14 complex products and one
    // twiddle product).
    static constexpr int R1 = NS >= 2 ? radix_at(N2, 1, MAXR) : 1;
    static constexpr int SPAN1 = NS >= 2 ? span_before(N2, 1, MAXR) : 0;
    static constexpr bool F1 = !TAB2 && NS >= 2 && B * (R1 - 1) * SPAN1 <= NT;
    static constexpr int NF1 = F1 ? B * (R1 - 1) * SPAN1 : 0;
    static constexpr size_t BUF_BYTES = (size_t)B * PN2 * (SPLIT ? sizeof(T) : sizeof(cx<T>));
    static constexpr size_t SMEM = BUF_BYTES + (size_t)(TWL + B * NS + B * R0 + NF1) * sizeof(cx<T>) +
                                   (size_t)NWAVE * (8 + 8 + 4 + 4);
    static_assert(B * NS <= NT, "one thread per (row, stage) factor");

    // LDS element offset of padded index x + r * step when x's padding is known
    template <int STEP>
    __device__ static __forceinline__ int off(int x, int r) {
        if constexpr (STEP % 16 == 0) {
            return pad16(x) + r * pad16(STEP);
        } else {
            return pad16(x + r * STEP);
        }
    }

    __device__ static void run(const FilterArgs& a, char* smem, int rb, int64_t ul) {
        cx<T>* buf = (cx<T>*)smem;
        T* fbuf = (T*)smem;  // SPLIT: [B][PN2] scalars
        cx<T>* tw = (cx<T>*)(smem + BUF_BYTES);  // TAB2: [r - 1][k] stage-1 factors
        cx<T>* trow = tw + TWL;  // [B][NS]: t^{weight_s} per row
        cx<T>* pow0 = trow + B * NS;  // [B][R0]: (t^{weight_0})^r, the stage-0 factors of each row
        cx<T>* f1 = pow0 + B * R0;    // F1: [B][R1 - 1][span_1] stage-1 factors
        unsigned long long* red_key = (unsigned long long*)(f1 + NF1);
        double* red_zz = (double*)(red_key + NWAVE);
        int* red_j = (int*)(red_zz + NWAVE);
        unsigned int* red_cnt = (unsigned int*)(red_j + NWAVE);

        const int tid = threadIdx.x;
        const int64_t u = a.unit0 + ul;
        const cx<T>* inter = (const cx<T>*)a.inter + ul * N;
        const __amdgpu_buffer_rsrc_t irs = buffer_rsrc(inter, (int)(N * (int64_t)sizeof(cx<T>)));

        if (!TAB2 && tid < B * NS) {
            const int b = tid / NS, st = tid % NS;
            const int m = (rb * B + b) * digit_weight_rt<N2, MAXR>(st);  // < N <= 2^22
            trow[b * NS + st] = root_of_unity((T)m / (T)N);
        }
        for (int q = tid; q < B * R0; q += NT) {
            // each power from its exactly reduced argument (no product chain)
            const int b = q / R0, r = q % R0;
            const int m = ((rb * B + b) * digit_weight(N2, 0, MAXR) * r) & (int)(N - 1);  // < N1 N2 <= 2^22
            pow0[q] = root_of_unity((T)m / (T)N);
        }

        T thr2 = T(0);
        bool count_on = false;
        const bool full_window = a.j_begin == 0 && a.j_end == N;
        double sigma = 1.0;
        float inv_sigma_f = 1.0f;
        int slot = -1;
        if constexpr (!RAW) {
            int64_t t, sg;
            unit_split(u, a.n_tmpl, t, sg);
            const mf_bank_entry e = a.bank[t];
            sigma = e.sigma;
            inv_sigma_f = e.inv_sigma;
            const double th = a.rho_threshold * sigma;
            thr2 = (T)(th * th);
            count_on = a.rho_threshold < INFINITY;
            const int64_t pub = t * a.n_seg + sg;  // public unit id t * n_seg + s
            for (int i = 0; i < a.n_series; ++i)
                if (a.series_units[i] == pub) slot = i;
        }
        unsigned long long best_key = 0ull;
        double best_zz = -1.0;
        int best_j = 0x7fffffff;
        unsigned int cnt = 0u;
        // DEFER: the thread's last-stage |z|^2, their maximum bits and the
        // sample index of output r = 0 (output r is at djg + r N1 SPAN_L)
        [[maybe_unused]] T dzz[DEFER ? RL : 1];
        [[maybe_unused]] unsigned int dmax = 0u;
        [[maybe_unused]] int djg = 0;
        __syncthreads();

        // SPLIT: the next stage's inputs, read during the exchange
        constexpr int CBPT = (B * N2 / R0 + NT - 1) / NT;
        cx<T> carry[SPLIT ? CBPT : 1][SPLIT ? R0 : 1];

        static_for<0, NS>([&](auto S_) {
            constexpr int s = decltype(S_)::value;
            constexpr int R = radix_at(N2, s, MAXR);
            constexpr int NSPAN = span_before(N2, s, MAXR);
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
                        // buffer loads from the unit's base (a unit is at most 2^22 complex
                        // values): one lane offset, the distances between the inputs r in
                        // scalar registers.  Non-temporal: each row is read once, and its
                        // lines are not kept (measured with the non-temporal pass-1 stores)
                        const unsigned int o0 = (unsigned int)(((rb * B + b) * N2 + j) * (int)sizeof(cx<T>));
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            v[i][r] = buffer_load_cx<T, kBufferNT>(irs, o0, r * PER_ROW * (int)sizeof(cx<T>));
                        if constexpr (TAB2) {
                            // input r is k2 = j + PER_ROW r: t^{k2} = t^j (t^{PER_ROW})^r
                            // (pass 1 already applied (t^{PER_ROW})^r when a.pre0_r0 is set)
                            const int64_t m = ((int64_t)(rb * B + b) * j) & (N - 1);
                            const cx<T> tj = root_of_unity((T)m / (T)N);
                            if (a.pre0_r0 > 0) {
#pragma unroll
                                for (int r = 0; r < R; ++r) v[i][r] = cmul(v[i][r], tj);
                            } else {
                                v[i][0] = cmul(v[i][0], tj);
#pragma unroll
                                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], cmul(pow0[b * R0 + r], tj));
                            }
                        } else if (a.pre0_r0 == 0) {
                            // stage 0 has no stage twiddle: its factors are the row's table
                            // (pass 1 applied them when a.pre0_r0 is set)
#pragma unroll
                            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], pow0[b * R0 + r]);
                        }
                    } else {
                        const int k = j % NSPAN;
                        if constexpr (SPLIT) {
#pragma unroll
                            for (int r = 0; r < R; ++r) v[i][r] = carry[i][r];
                        } else {
                            const cx<T>* src = buf + b * PN2;
#pragma unroll
                            for (int r = 0; r < R; ++r) v[i][r] = src[off<PER_ROW>(j, r)];
                        }
                        cx<T> p[R];
                        if constexpr (TAB2 && s == 1) {
#pragma unroll
                            for (int r = 1; r < R; ++r) p[r] = tw[(r - 1) * NSPAN + k];
                        } else if constexpr (TAB2 && s == 2) {
                            const cx<T>* t2 = (const cx<T>*)a.tw2;
#pragma unroll
                            for (int r = 1; r < R; ++r) p[r] = t2[(r - 1) * NSPAN + k];
                        } else if constexpr (F1 && s == 1) {
                            const cx<T>* f = f1 + b * (R1 - 1) * SPAN1 + k;
#pragma unroll
                            for (int r = 1; r < R; ++r) p[r] = f[(r - 1) * SPAN1];
                        } else {
                            powers<R>(cmul(tw[tw_offset(N2, s, MAXR) + k], trow[b * NS + s]), p);
                        }
#pragma unroll
                        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], p[r]);
                    }
                    IDft<R, T>::run(v[i]);
                }
            }
            if constexpr (s == 0) {
                if constexpr (TAB2) {
                    // stage-1 factors e^{2 pi i k r / 256}, k < 16, from exactly reduced arguments
                    for (int q = tid; q < 15 * 16; q += NT) {
                        const int r = q / 16 + 1, k = q % 16;
                        tw[q] = root_of_unity((T)((k * r) & 255) / (T)256);
                    }
                } else {
                    fill_stage_twiddles<T, N2, MAXR>(tw, tid, NT);
                }
                if constexpr (F1) {
                    // entry (b, r, k): exponent r dw_1 (k N1 + j1) mod N, the stage-1 factor
                    // (w_1^k t^{dw_1})^r of input r at span position k of row j1 = rb B + b
                    if (tid < NF1) {
                        const int b = tid / ((R1 - 1) * SPAN1), rk = tid % ((R1 - 1) * SPAN1);
                        const int r = rk / SPAN1 + 1, k = rk % SPAN1;
                        constexpr int DW1 = digit_weight(N2, 1, MAXR);
                        const int m = (int)(((unsigned int)r * (unsigned int)(DW1 * (k * N1 + rb * B + b))) &
                                            (unsigned int)(N - 1));
                        f1[tid] = root_of_unity((T)m / (T)N);
                    }
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
                        // output r of this butterfly is time sample j1 + N1 (j + r NSPAN): increasing in r
                        if constexpr (RAW) {
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                ((cx<T>*)a.raw_out)[u * N + j1 + (int64_t)N1 * (j + r * NSPAN)] = v[i][r];
                        } else {
                            T zz[R];
#pragma unroll
                            for (int r = 0; r < R; ++r) zz[r] = norm2(v[i][r]);
                            if (slot >= 0) {
#pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    const int64_t jg = j1 + (int64_t)N1 * (j + r * NSPAN);
                                    if constexpr (F64) {
                                        ((double*)a.rho)[(int64_t)slot * N + jg] = sqrt(zz[r]) / sigma;
                                    } else {
                                        ((float*)a.rho)[(int64_t)slot * N + jg] = sqrtf(zz[r]) * inv_sigma_f;
                                    }
                                }
                            }
                            if (full_window) {
                                // FP32: integer max of the non-negative float bits (NaN
                                // bits exceed +inf, so a NaN propagates)
                                unsigned int mb = 0u;
                                if constexpr (!F64) {
                                    mb = __float_as_uint(zz[0]);
#pragma unroll
                                    for (int r = 1; r < R; ++r) mb = max(mb, __float_as_uint(zz[r]));
                                }
                                if (count_on) {
                                    // FP32: almost no butterfly reaches the threshold, so
                                    // its largest |z|^2 is tested first
                                    if (F64 || mb >= __float_as_uint((float)thr2)) {
#pragma unroll
                                        for (int r = 0; r < R; ++r) cnt += (zz[r] >= thr2) ? 1u : 0u;
                                    }
                                }
                                if (a.ev_keys != nullptr) {
                                    // events: rare samples at or above the threshold update their window
                                    unsigned long long* ek = a.ev_keys + u * (N >> a.ev_log2w);
#pragma unroll
                                    for (int r = 0; r < R; ++r) {
                                        if (zz[r] >= thr2) {
                                            const unsigned int jg = (unsigned int)(j1 + N1 * (j + r * NSPAN));
                                            const unsigned long long key =
                                                F64 ? event_key64((double)zz[r], jg & ((1u << a.ev_log2w) - 1u))
                                                    : event_key32((float)zz[r], jg);
                                            atomicMax(ek + (jg >> a.ev_log2w), key);
                                        }
                                    }
                                }
                                if constexpr (F64) {
#pragma unroll
                                    for (int r = 0; r < R; ++r) {
                                        const int jg = j1 + N1 * (j + r * NSPAN);
                                        if (better64(zz[r], jg, best_zz, best_j)) {
                                            best_zz = zz[r];
                                            best_j = jg;
                                        }
                                    }
                                } else if constexpr (DEFER) {
                                    dmax = mb;
                                    djg = j1 + N1 * j;
#pragma unroll
                                    for (int r = 0; r < R; ++r) dzz[r] = zz[r];
                                } else {
                                    // the lowest r that attains the maximum
                                    int rmin = R - 1;
#pragma unroll
                                    for (int r = R - 2; r >= 0; --r) rmin = __float_as_uint(zz[r]) == mb ? r : rmin;
                                    const unsigned int jg = (unsigned int)(j1 + N1 * (j + rmin * NSPAN));
                                    const unsigned long long key =
                                        ((unsigned long long)mb << 32) | (unsigned long long)(0xffffffffu - jg);
                                    best_key = key > best_key ? key : best_key;
                                }
                            } else {
#pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    const int jg = j1 + N1 * (j + r * NSPAN);
                                    if (jg >= a.j_begin && jg < a.j_end) {
                                        if (count_on) cnt += (zz[r] >= thr2) ? 1u : 0u;
                                        if constexpr (F64) {
                                            if (better64(zz[r], jg, best_zz, best_j)) {
                                                best_zz = zz[r];
                                                best_j = jg;
                                            }
                                        } else {
                                            const unsigned long long key =
                                                ((unsigned long long)__float_as_uint(zz[r]) << 32) |
                                                (unsigned long long)(0xffffffffu - (unsigned int)jg);
                                            best_key = key > best_key ? key : best_key;
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
            } else if constexpr (SPLIT) {
                // same positions as below, one component at a time; the next
                // stage has the same radix, so the same (j, b) per thread
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < BPT; ++i) {
                        const int bf = tid + i * NT;
                        if (NBF % NT == 0 || bf < NBF) {
                            const int j = bf % PER_ROW;
                            const int b = bf / PER_ROW;
                            const int idxD = (j / NSPAN) * NSPAN * R + (j % NSPAN);
                            T* dst = fbuf + b * PN2;
                            if constexpr (CF && s == 0) {
                                // byte offsets: (w0 ^ r) * 4 = (w0 * 4) ^ (r * 4), one xor per store
                                unsigned int a0 = (unsigned int)cf_wr0(j) * (unsigned int)sizeof(T);
                                asm volatile("" : "+v"(a0));  // keep the xor on the scaled offset
                                char* d = (char*)dst;
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    *(T*)(d + (a0 ^ (unsigned int)(r * sizeof(T)))) = part ? v[i][r].y : v[i][r].x;
                            } else if constexpr (CF) {
#pragma unroll
                                for (int r = 0; r < R; ++r) dst[cf_wr1(j, r)] = part ? v[i][r].y : v[i][r].x;
                            } else {
#pragma unroll
                                for (int r = 0; r < R; ++r) dst[off<NSPAN>(idxD, r)] = part ? v[i][r].y : v[i][r].x;
                            }
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < BPT; ++i) {
                        const int bf = tid + i * NT;
                        if (NBF % NT == 0 || bf < NBF) {
                            const int j = bf % PER_ROW;
                            const int b = bf / PER_ROW;
                            const T* src = fbuf + b * PN2;
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                int at;
                                if constexpr (CF && s == 0) {
                                    at = cf_rd0(j, r);
                                } else if constexpr (CF) {
                                    at = cf_rd1(j, r);
                                } else {
                                    at = off<PER_ROW>(j, r);
                                }
                                if (part) carry[i][r].y = src[at];
                                else carry[i][r].x = src[at];
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
                        cx<T>* dst = buf + b * PN2;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            if constexpr (NSPAN == 1 && R == 16) {
                                dst[pad16(idxD) + r] = v[i][r];  // idxD = 16 j: r stays inside the 16-block
                            } else {
                                dst[off<NSPAN>(idxD, r)] = v[i][r];
                            }
                        }
                    }
                }
                __syncthreads();
            }
        });

        if constexpr (DEFER) {
            if (full_window) {
                const int lane = tid & 63;
                const int wave = tid >> 6;
                const unsigned int m = wave_max_u32(dmax);
                // threshold counts are rare in noise: reduce them only if a lane has one
                if (__builtin_amdgcn_ballot_w64(cnt != 0u) != 0ull) cnt = wave_sum_u32(cnt);
                unsigned int* red_max = (unsigned int*)red_j;
                if (lane == 0) {
                    red_cnt[wave] = cnt;
                    red_max[wave] = m;
                }
                if (tid == 0) red_key[0] = 0ull;
                __syncthreads();
                unsigned int bmax = red_max[0];
#pragma unroll
                for (int wv = 1; wv < NWAVE; ++wv) bmax = max(bmax, red_max[wv]);
                if (dmax == bmax) {
                    // rare: the lowest r of this thread that attains the maximum
                    int rmin = RL - 1;
#pragma unroll
                    for (int r = RL - 2; r >= 0; --r) rmin = __float_as_uint(dzz[r]) == bmax ? r : rmin;
                    const unsigned int jg = (unsigned int)(djg + N1 * rmin * SPAN_L);
                    atomicMax(red_key, ((unsigned long long)bmax << 32) | (unsigned long long)(0xffffffffu - jg));
                }
                __syncthreads();
                if (tid == 0) {
                    unsigned int total = 0u;
#pragma unroll
                    for (int wv = 0; wv < NWAVE; ++wv) total += red_cnt[wv];
                    atomicMax(a.keys + u, red_key[0]);
                    if (total) atomicAdd(a.counts + u, total);
                }
                return;
            }
        }
        if constexpr (!RAW) {
            // work-group reduction: wave shuffles, then one LDS slot per wave
            const int lane = tid & 63;
            const int wave = tid >> 6;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                cnt += __shfl_xor(cnt, o, 64);
                if constexpr (F64) {
                    const double ozz = __shfl_xor(best_zz, o, 64);
                    const int oj = __shfl_xor(best_j, o, 64);
                    if (better64(ozz, oj, best_zz, best_j)) {
                        best_zz = ozz;
                        best_j = oj;
                    }
                } else {
                    const unsigned long long ov = __shfl_xor(best_key, o, 64);
                    best_key = ov > best_key ? ov : best_key;
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
                for (int wv = 1; wv < NWAVE; ++wv) {
                    cnt += red_cnt[wv];
                    if constexpr (F64) {
                        if (better64(red_zz[wv], red_j[wv], best_zz, best_j)) {
                            best_zz = red_zz[wv];
                            best_j = red_j[wv];
                        }
                    } else {
                        best_key = red_key[wv] > best_key ? red_key[wv] : best_key;
                    }
                }
                if constexpr (F64) {
                    // partials of every unit of the call: [n_units][N1 / B]
                    Partial64* part = (Partial64*)a.partials + u * (N1 / B) + rb;
                    *part = Partial64{best_zz, best_j, (int32_t)cnt};
                } else {
                    atomicMax(a.keys + u, best_key);
                    if (cnt) atomicAdd(a.counts + u, cnt);
                }
            }
        }
    }
};

}  // namespace mf
