// chi^2 time-frequency veto of arXiv:0906.4175, Eq. (5) (Sec. 1.2), over the
// whole series: for every time sample j of every (template, segment) unit,
//   chi^2(j) = p / sigma^2 sum_l |z_l(j) - z(j)/p|^2
//            = (p sum_l |z_l(j)|^2 - |z(j)|^2) / sigma^2 ,   z = sum_l z_l,
// where z_l is Eq. (1) restricted to band l of p bands with equal shares of
// sigma^2 (Eq. (4)).  The paper runs one inverse FFT per band and a separate
// accumulation kernel; here the p band transforms share the two-pass inverse
// DFT of the matched filter (bins k = N2 k1 + k2, times j = j1 + N1 j2):
//
//  * The bands are contiguous in k and, except the widest, span only a few
//    thousand bins.  Pass 1 transforms only the widest band (its column
//    transform goes to the intermediate as in the plain filter) and copies
//    the template x weight product q of every other band l into a slot: the
//    n_l rows of N2 bins from s_l (e_l rounded down to a multiple of 16),
//    zero outside the band.
//  * Pass 2 rebuilds row j1 of every other band from its slot,
//    Y_l[j1][k2] = sum_m q[s_l + m N2 + k2] e^{2 pi i j1 m / N1} (mostly a
//    single row, so no products), runs the p row transforms, accumulates
//    z = sum_l e^{2 pi i s_l j / N} (transform of slot l) and sum_l |z_l|^2 in
//    registers and reduces |z|^2 (peak, threshold count, series) together
//    with chi^2.
//
// Per unit this moves the slots (written once, re-read from cache), one
// intermediate and the weights instead of p intermediates.
#include "filter_tiles.hpp"

#ifndef MF_BAND_WAVES
#define MF_BAND_WAVES 3
#endif

namespace mf {

// Peak record of one pass-2 work-group in band mode: max |z|^2 (lowest index
// on ties), chi^2 at that sample, threshold count.
struct PartialChi {
    double zz;
    double chi2;
    int32_t j;
    int32_t cnt;
};

// Band table of one template: e_0 = k_lo < e_1 <= ... <= e_p = k_hi + 1 with
// e_l = min{k : P[k-1] - P[k_lo-1] >= l/p (P[k_hi] - P[k_lo-1])} (a bin
// belongs to the band in which the sigma^2 sum before it falls), then the
// index of the band with the most slot rows n_l (the one pass 1 transforms),
// then the slot starts sum_{l' < l} n_l' N2 (n_l = 0 for it and for empty bands).
__global__ void __launch_bounds__(64) k_band_table(int64_t n, int n2, const mf_bank_entry* bank, const double* P,
                                                   int p, int32_t* tab) {
    __shared__ int64_t edge[kMaxBands + 1];
    const int tid = threadIdx.x;
    const int64_t t = blockIdx.x;
    const mf_bank_entry e = bank[t];
    const int64_t klo = e.k_lo, khi = e.k_hi;
    int32_t* row = tab + t * band_tab_stride(p);
    const bool valid = klo >= 1 && khi >= klo && khi <= n / 2 - 1;
    if (!valid) {
        // empty bands and slots: every bin stays untouched and the unit outputs zero
        for (int l = tid; l <= p; l += 64) {
            row[l] = 1;
            row[p + 2 + l] = 0;
        }
        if (tid == 0) row[p + 1] = 0;
        return;
    }
    if (tid == 0) {
        edge[0] = klo;
        edge[p] = khi + 1;
    }
    if (tid >= 1 && tid < p) {
        const double base = P[klo - 1];
        const double target = (double)tid / (double)p * (P[khi] - base);
        int64_t lo = klo + 1, hi = khi + 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (P[mid - 1] - base >= target) hi = mid; else lo = mid + 1;
        }
        edge[tid] = lo;
    }
    __syncthreads();
    for (int l = tid; l <= p; l += 64) row[l] = (int32_t)edge[l];
    if (tid == 0) {
        auto slot_rows = [&](int l) -> int64_t {
            const int64_t sl = edge[l] & ~(int64_t)(kSlotAlign - 1);
            return edge[l + 1] > edge[l] ? (edge[l + 1] - sl + n2 - 1) / n2 : 0;
        };
        int wide = 0;
        int64_t best = -1;
        for (int l = 0; l < p; ++l) {
            const int64_t rows = slot_rows(l);
            if (rows > best) {
                best = rows;
                wide = l;
            }
        }
        row[p + 1] = wide;
        int64_t acc = 0;
        for (int l = 0; l < p; ++l) {
            row[p + 2 + l] = (int32_t)acc;
            if (l != wide) acc += slot_rows(l) * n2;
        }
        row[2 * p + 2] = (int32_t)acc;
    }
}

// ---------------------------------------------------------------------------
// Pass 2 tile in band mode: B rows j1 of one unit, all p bands.
// ---------------------------------------------------------------------------
template <typename T, int N1, int N2, int B, int NT, int MAXR = 16>
struct Pass2Band {
    static constexpr int64_t N = (int64_t)N1 * N2;
    static constexpr int NS = num_stages(N2, MAXR);
    static constexpr int PN2 = pad16(N2);
    static constexpr int NWAVE = NT / 64;
    static constexpr int TW = tw_total(N2, MAXR);
    static constexpr int HALF = N1 / 2;
    static constexpr int RL = radix_at(N2, NS - 1, MAXR);
    static constexpr int NSPANL = span_before(N2, NS - 1, MAXR);
    static constexpr int PER_ROWL = N2 / RL;
    static constexpr int NBFL = B * N2 / RL;
    static constexpr int BPTL = (NBFL + NT - 1) / NT;
    static constexpr bool F64 = std::is_same<T, double>::value;
    // The stage factors do not depend on the band, so stages 0 and 1 read
    // theirs from per-row tables filled once: [B][R0] and [B][R1][span_1]
    // (r-major, so lanes with consecutive k read consecutive entries).
    // (Shapes with many rows per work-group keep the powers where a table
    // would crowd LDS.)
    static constexpr int R0 = radix_at(N2, 0, MAXR);
    static constexpr int R1 = NS >= 2 ? radix_at(N2, 1, MAXR) : 1;
    static constexpr int SP1 = NS >= 2 ? span_before(N2, 1, MAXR) : 0;
    static constexpr bool USE_F0 = B * R0 * sizeof(cx<T>) <= 4096;
    static constexpr bool USE_F1 = NS >= 2 && B * R1 * SP1 * sizeof(cx<T>) <= 8192;
    static constexpr int NF0 = USE_F0 ? B * R0 : 0;
    static constexpr int NF1 = USE_F1 ? B * R1 * SP1 : 0;
    static constexpr int TAB = NF0 + NF1;
    static constexpr size_t SMEM =
        (size_t)(B * PN2 + TW + B * NS + B * HALF + TAB) * sizeof(cx<T>) + (size_t)NWAVE * (8 + 8 + 4 + 4);
    static_assert(B * NS <= NT, "one thread per (row, stage) factor");
    // 4096-point rows, three radix-16 stages, one row per work-group: the
    // exchanges use the bank-conflict-free layouts of the plain pass 2 (on
    // complex values, where a half-wave must touch 32 distinct 8-byte slots).
    static constexpr bool CF = N2 == 4096 && MAXR == 16 && B == 1 && NT == 256;
    static_assert(kSlotAlign % RL == 0, "slot starts make the band factor uniform over a butterfly");
    static_assert(!CF || PN2 >= kCfSlots, "conflict-free layout slots");

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
        cx<T>* tw = buf + B * PN2;
        cx<T>* trow = tw + TW;   // [B][NS]: t^{weight_s} per row
        cx<T>* om = trow + B * NS;  // [B][N1/2]: e^{2 pi i j1 k1 / N1}
        cx<T>* f0 = om + B * HALF;  // [B][R0]: stage-0 factors
        cx<T>* f1 = f0 + NF0;       // [B][R1][SP1]: stage-1 factors
        double* red_zz = (double*)(f1 + NF1);
        double* red_chi = red_zz + NWAVE;
        int* red_j = (int*)(red_chi + NWAVE);
        unsigned int* red_cnt = (unsigned int*)(red_j + NWAVE);

        const int tid = threadIdx.x;
        const int64_t u = a.unit0 + ul;
        const int64_t t = u % a.n_tmpl;
        const cx<T>* inter = (const cx<T>*)a.inter + ul * N;
        const __amdgpu_buffer_rsrc_t irs = buffer_rsrc(inter, (int)(N * (int64_t)sizeof(cx<T>)));
        const int P = a.p_bands;
        const int32_t* tab = a.band_tab + t * band_tab_stride(P);
        const int wb = tab[P + 1];
        const int32_t* slot0 = tab + P + 2;
        const cx<T>* slots = (const cx<T>*)a.qbuf + ul * band_slot_stride(N, N2, P);

        if (tid < B * NS) {
            const int b = tid / NS, st = tid % NS;
            const int64_t m = (int64_t)(rb * B + b) * digit_weight(N2, st, MAXR);  // < N
            trow[b * NS + st] = root_of_unity((T)m / (T)N);
        }
        for (int m = tid; m < B * HALF; m += NT) {
            const int b = m / HALF, k1 = m % HALF;
            const int64_t jk = (int64_t)(rb * B + b) * k1 % N1;  // exact reduction
            om[m] = root_of_unity((T)jk / (T)N1);
        }
        fill_stage_twiddles<T, N2, MAXR>(tw, tid, NT);
        // stage s multiplies input r by e^{2 pi i r w_s (k N1 + j1) / N}, w_s = N2 / (span_s R_s):
        // each entry from its exactly reduced integer argument
        for (int q = tid; q < NF0; q += NT) {
            const int64_t j1 = rb * B + q / R0, r = q % R0;
            const int64_t m = ((int64_t)digit_weight(N2, 0, MAXR) * j1 % N) * r % N;
            f0[q] = root_of_unity((T)m / (T)N);
        }
        for (int q = tid; q < NF1; q += NT) {
            const int64_t j1 = rb * B + q / (R1 * SP1), r = (q / SP1) % R1, k = q % SP1;
            const int64_t m = ((int64_t)digit_weight(N2, 1, MAXR) * ((int64_t)k * N1 + j1) % N) * r % N;
            f1[q] = root_of_unity((T)m / (T)N);
        }

        const mf_bank_entry e = a.bank[t];
        const double sigma = e.sigma;
        const float inv_sigma_f = e.inv_sigma;
        const double th = a.rho_threshold * sigma;
        const T thr2 = (T)(th * th);
        const bool count_on = a.rho_threshold < INFINITY;
        const int64_t pub = t * a.n_seg + u / a.n_tmpl;
        int slot = -1;
        for (int i = 0; i < a.n_series; ++i)
            if (a.series_units[i] == pub) slot = i;

        cx<T> accz[BPTL][RL];
        T accq[BPTL][RL];
#pragma unroll
        for (int i = 0; i < BPTL; ++i)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                accz[i][r] = cx<T>{T(0), T(0)};
                accq[i][r] = T(0);
            }
        __syncthreads();

        for (int l = 0; l < P; ++l) {
            const int64_t e0 = tab[l], e1 = tab[l + 1];
            if (e0 >= e1) continue;  // empty band (uniform over the work-group)
            const bool from_inter = l == wb;
            const int sb = slot0[l];
            const int nrow = (slot0[l + 1] - sb) / N2;
            const unsigned int sl = from_inter ? 0u : (unsigned int)e0 & ~(unsigned int)(kSlotAlign - 1);
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
                        [[maybe_unused]] cx<T> base = trow[b * NS + s];
                        if constexpr (s == 0) {
                            constexpr int RB = PER_ROW * (int)sizeof(cx<T>);  // bytes between inputs r
                            if (from_inter) {
                                const unsigned int o0 = (unsigned int)(((rb * B + b) * N2 + j) * (int)sizeof(cx<T>));
#pragma unroll
                                for (int r = 0; r < R; ++r) v[i][r] = buffer_load_cx<T>(irs, o0, r * RB);
                            } else {
                                // slot row m holds the bins s_l + m N2 + k2 (zero outside the
                                // band): Y[k2] = sum_m slot[m N2 + k2] e^{2 pi i j1 m / N1}
                                const __amdgpu_buffer_rsrc_t srs =
                                    buffer_rsrc(slots + sb, nrow * N2 * (int)sizeof(cx<T>));
                                const unsigned int o0 = (unsigned int)(j * (int)sizeof(cx<T>));
#pragma unroll
                                for (int r = 0; r < R; ++r) v[i][r] = buffer_load_cx<T>(srs, o0, r * RB);
                                for (int m = 1; m < nrow; ++m) {
                                    const cx<T> w = om[b * HALF + m];
                                    const int mo = m * N2 * (int)sizeof(cx<T>);
                                    // groups of G loads issued together, so a wave waits for the
                                    // cache once per group
                                    constexpr int G = R >= 4 ? 4 : R;
#pragma unroll
                                    for (int r0 = 0; r0 < R; r0 += G) {
                                        cx<T> x[G];
#pragma unroll
                                        for (int g = 0; g < G; ++g) x[g] = buffer_load_cx<T>(srs, o0, mo + (r0 + g) * RB);
#pragma unroll
                                        for (int g = 0; g < G; ++g) {
                                            // v += x w as four fused multiply-adds
                                            v[i][r0 + g].x = fma(x[g].x, w.x, fma(-x[g].y, w.y, v[i][r0 + g].x));
                                            v[i][r0 + g].y = fma(x[g].x, w.y, fma(x[g].y, w.x, v[i][r0 + g].y));
                                        }
                                    }
                                }
                            }
                        } else {
                            const int k = j % NSPAN;
                            const cx<T>* src = buf + b * PN2;
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                if constexpr (CF && s == 1) {
                                    v[i][r] = src[cf_rd0(j, r)];
                                } else if constexpr (CF) {
                                    v[i][r] = src[cf_rd1(j, r)];
                                } else {
                                    v[i][r] = src[off<PER_ROW>(j, r)];
                                }
                            }
                            if constexpr (s >= 2 || !USE_F1) base = cmul(tw[tw_offset(N2, s, MAXR) + k], base);
                        }
                        cx<T> pw[R];
                        if constexpr (s == 0 && USE_F0) {
#pragma unroll
                            for (int r = 1; r < R; ++r) pw[r] = f0[b * R0 + r];
                        } else if constexpr (s == 1 && USE_F1) {
                            const int k = j % NSPAN;
#pragma unroll
                            for (int r = 1; r < R; ++r) pw[r] = f1[(b * R1 + r) * SP1 + k];
                        } else {
                            powers<R>(base, pw);
                        }
#pragma unroll
                        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], pw[r]);
                        IDft<R, T>::run(v[i]);
                    }
                }
                if constexpr (s == NS - 1) {
#pragma unroll
                    for (int i = 0; i < BPT; ++i) {
                        // z_l(j) is e^{2 pi i s_l j / N} times the transform of the slot
                        // (s_l = 0 for the transformed band); with j = j1 + N1 (j' + NSPAN r)
                        // the factor does not depend on r (s_l N1 NSPAN = (s_l / R) N): one
                        // per butterfly
                        const int bf = tid + i * NT;
                        const int jj = bf % PER_ROW;
                        const int b = bf / PER_ROW;
                        // both factors < 2^24 (s_l < N/2, j < N <= 2^22): a 24-bit product suffices
                        const unsigned int m = __umul24(sl, (unsigned int)(rb * B + b + N1 * jj)) & (unsigned int)(N - 1);
                        const cx<T> ph = root_of_unity((T)(int)m / (T)N);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const cx<T> y = v[i][r];
                            accz[i][r].x = fma(y.x, ph.x, fma(-y.y, ph.y, accz[i][r].x));
                            accz[i][r].y = fma(y.x, ph.y, fma(y.y, ph.x, accz[i][r].y));
                            accq[i][r] += norm2(y);
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
                                if constexpr (CF && s == 0) {
                                    dst[cf_wr0(j) ^ r] = v[i][r];
                                } else if constexpr (CF) {
                                    dst[cf_wr1(j, r)] = v[i][r];
                                } else if constexpr (NSPAN == 1 && R == 16) {
                                    dst[pad16(idxD) + r] = v[i][r];
                                } else {
                                    dst[off<NSPAN>(idxD, r)] = v[i][r];
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
            });
        }

        // chi^2, rho, series, peak and threshold count of this tile
        const double sig2 = sigma * sigma;
        double best_zz = -1.0, best_chi = 0.0;
        int best_j = 0x7fffffff;
        unsigned int cnt = 0u;
#pragma unroll
        for (int i = 0; i < BPTL; ++i) {
            const int bf = tid + i * NT;
            if (NBFL % NT == 0 || bf < NBFL) {
                const int j = bf % PER_ROWL;
                const int b = bf / PER_ROWL;
                const int j1 = rb * B + b;
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int jg = j1 + N1 * (j + r * NSPANL);
                    const T zz = norm2(accz[i][r]);
                    const double chi = ((double)P * (double)accq[i][r] - (double)zz) / sig2;
                    if (slot >= 0) {
                        if constexpr (F64) {
                            ((double*)a.rho)[(int64_t)slot * N + jg] = sqrt(zz) / sigma;
                            ((double*)a.chi_series)[(int64_t)slot * N + jg] = chi;
                        } else {
                            ((float*)a.rho)[(int64_t)slot * N + jg] = sqrtf(zz) * inv_sigma_f;
                            ((float*)a.chi_series)[(int64_t)slot * N + jg] = (float)chi;
                        }
                    }
                    if (jg >= a.j_begin && jg < a.j_end) {
                        if (count_on) cnt += (zz >= thr2) ? 1u : 0u;
                        if (better64((double)zz, jg, best_zz, best_j)) {
                            best_zz = (double)zz;
                            best_j = jg;
                            best_chi = chi;
                        }
                    }
                }
            }
        }
        const int lane = tid & 63;
        const int wave = tid >> 6;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            cnt += __shfl_xor(cnt, o, 64);
            const double ozz = __shfl_xor(best_zz, o, 64);
            const double och = __shfl_xor(best_chi, o, 64);
            const int oj = __shfl_xor(best_j, o, 64);
            if (better64(ozz, oj, best_zz, best_j)) {
                best_zz = ozz;
                best_j = oj;
                best_chi = och;
            }
        }
        if (lane == 0) {
            red_cnt[wave] = cnt;
            red_zz[wave] = best_zz;
            red_chi[wave] = best_chi;
            red_j[wave] = best_j;
        }
        __syncthreads();
        if (tid == 0) {
            for (int wv = 1; wv < NWAVE; ++wv) {
                cnt += red_cnt[wv];
                if (better64(red_zz[wv], red_j[wv], best_zz, best_j)) {
                    best_zz = red_zz[wv];
                    best_j = red_j[wv];
                    best_chi = red_chi[wv];
                }
            }
            PartialChi* part = (PartialChi*)a.partials + u * (N1 / B) + rb;
            *part = PartialChi{best_zz, best_chi, best_j, (int32_t)cnt};
        }
    }
};

template <typename T, int PH, int N1, int N2, int C, int NT>
__global__ void __launch_bounds__(NT) k_pass1_band(FilterArgs a) {
    using P = Pass1<T, PH, P1_BAND, N1, N2, C, NT>;
    __shared__ __align__(16) char smem[P::SMEM];
    P::run(a, smem, blockIdx.x, blockIdx.y);
}

// FP32 radix-16 rows, one row per work-group: at least 3 waves per SIMD, so
// 168 VGPRs hold the row, the accumulators and the transform without spills.
// Measured on MI355X (2^20, p = 16, 16 units per launch): 393 us per launch,
// against 487 us at 4 waves (128 VGPRs, where the compiler spills).  (Shapes
// with several rows per work-group are held below 4 waves by LDS anyway.)
template <typename T, int B, int R2>
constexpr int band_min_waves() {
    return MF_BAND_WAVES > 0 && sizeof(T) == 4 && R2 == 16 && B == 1 ? MF_BAND_WAVES : 1;
}

template <typename T, int N1, int N2, int B, int NT, int R2>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(band_min_waves<T, B, R2>(), 8)))
k_pass2_band(FilterArgs a) {
    using P = Pass2Band<T, N1, N2, B, NT, R2>;
    __shared__ __align__(16) char smem[P::SMEM];
    P::run(a, smem, blockIdx.x, blockIdx.y);
}

// One 64-thread work-group per unit: peak over the partials (same comparison
// as pass 2), chi^2 at the peak, threshold count.
__global__ void __launch_bounds__(64) k_finalize_band(const PartialChi* part, int n_part, const mf_bank_entry* bank,
                                                      int64_t n_tmpl, int64_t n_seg, mf_peak* peaks, double* chisq) {
    const int64_t u = blockIdx.x;
    const int64_t t = u % n_tmpl, s = u / n_tmpl;
    double bzz = -1.0, bchi = 0.0;
    int bj = 0x7fffffff;
    long long cnt = 0;
    for (int i = threadIdx.x; i < n_part; i += 64) {
        const PartialChi p = part[u * n_part + i];
        cnt += p.cnt;
        if (better64(p.zz, p.j, bzz, bj)) {
            bzz = p.zz;
            bj = p.j;
            bchi = p.chi2;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        const double ozz = __shfl_xor(bzz, off, 64);
        const double och = __shfl_xor(bchi, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (better64(ozz, oj, bzz, bj)) {
            bzz = ozz;
            bj = oj;
            bchi = och;
        }
    }
    if (threadIdx.x == 0) {
        mf_peak o;
        o.rho = sqrt(bzz) / bank[t].sigma;
        o.j = bj;
        o.n_above = (int32_t)cnt;
        peaks[t * n_seg + s] = o;
        chisq[t * n_seg + s] = bchi;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// One shape per N and precision (the default shape of the plain filter), the
// first entry for each being the default; R2 is the largest pass-2 stage
// radix (an R2 = 8 entry can be installed with mf_set_band_plan).
#define MF_BAND_SHAPES(X)                                                                                   \
    X(float, 32, 32, 16, 32, 16) X(float, 32, 64, 16, 32, 16) X(float, 64, 64, 16, 64, 16) X(float, 64, 128, 16, 32, 16)    \
    X(float, 128, 128, 16, 32, 16) X(float, 128, 256, 16, 16, 16) X(float, 256, 256, 16, 16, 16)                         \
    X(float, 256, 512, 16, 8, 16) X(float, 512, 512, 16, 8, 16) X(float, 512, 1024, 16, 4, 16)                            \
    X(float, 256, 4096, 16, 1, 16) X(float, 256, 4096, 16, 1, 8) X(float, 1024, 2048, 16, 2, 16) X(float, 2048, 2048, 8, 2, 16)                         \
    X(double, 32, 32, 8, 32, 16) X(double, 32, 64, 8, 32, 16) X(double, 64, 64, 8, 64, 16) X(double, 64, 128, 8, 32, 16)     \
    X(double, 128, 128, 8, 32, 16) X(double, 128, 256, 8, 16, 16) X(double, 256, 256, 8, 16, 16)                          \
    X(double, 256, 512, 8, 8, 16) X(double, 512, 512, 8, 8, 16) X(double, 512, 1024, 8, 4, 16)                            \
    X(double, 512, 2048, 8, 2, 16) X(double, 1024, 2048, 4, 2, 16) X(double, 2048, 2048, 2, 2, 16)

static constexpr int band_threads(int x) { return x < 64 ? 64 : (x > 1024 ? 1024 : x); }

static bool band_want(mf_precision prec, bool f64) { return (prec == MF_FP64) == f64; }

Plan default_band_plan(int log2n, mf_precision prec) {
    Plan p{};
    p.log2n = -1;
    bool found = false;
#define MF_BFIRST(T, N1, N2, C, B, R2)                                                                      \
    if (!found && band_want(prec, std::is_same<T, double>::value) && ilog2((long long)N1 * N2) == log2n &&  \
        R2 == 16) {                                                                                         \
        p.n1 = N1;                                                                                          \
        p.n2 = N2;                                                                                          \
        p.c1 = C;                                                                                           \
        p.b2 = B;                                                                                           \
        p.nt1 = band_threads(C * N1 / 16);                                                                  \
        p.nt2 = band_threads(B * N2 / R2);                                                                  \
        p.log2n = log2n;                                                                                    \
        found = true;                                                                                       \
    }
    MF_BAND_SHAPES(MF_BFIRST)
#undef MF_BFIRST
    if (!found) return p;
    // About 192 MiB of intermediates per batch (the slots add about a tenth),
    // so that pass 2 finds what pass 1 wrote still in the 256 MB last-level
    // cache (measured at 2^20 FP32, pass 2 per unit: 16 units 24.6 us, 21 units
    // 24.1 us, 24 units 23.9 us, 32 units 24.0 us).
    const size_t bytes_per_unit = ((size_t)1 << log2n) * cx_bytes(prec);
    const size_t u = ((size_t)192 << 20) / bytes_per_unit;
    p.units = (int)(u < 1 ? 1 : (u > 4096 ? 4096 : u));
    p.fused = false;
    return p;
}

bool band_plan_supported(const Plan& q, mf_precision prec) {
#define MF_BMATCH(T, N1, N2, C, B, R2)                                                                         \
    if (band_want(prec, std::is_same<T, double>::value) && q.n1 == N1 && q.n2 == N2 && q.c1 == C &&          \
        q.b2 == B && q.nt1 == band_threads(C * N1 / 16) && q.nt2 == band_threads(B * N2 / R2))               \
        return true;
    MF_BAND_SHAPES(MF_BMATCH)
#undef MF_BMATCH
    return false;
}

static size_t align256b(size_t x) { return (x + 255) & ~(size_t)255; }

BandLayout band_layout(const Plan& p, mf_precision prec, int64_t n, int64_t n_tmpl, int64_t n_seg, int p_bands) {
    BandLayout L{};
    const int64_t n_units = n_tmpl * n_seg;
    const int64_t upb = n_units < p.units ? n_units : p.units;
    L.units_per_batch = upb < 1 ? 1 : upb;
    size_t off = 0;
    L.off_w = off;
    off = align256b(off + (size_t)n_seg * (size_t)(n / 2 + 1) * cx_bytes(prec));
    L.off_tab = off;
    off = align256b(off + (size_t)n_tmpl * (size_t)band_tab_stride(p_bands) * sizeof(int32_t));
    L.off_q = off;
    off = align256b(off + (size_t)L.units_per_batch * (size_t)band_slot_stride(n, p.n2, p_bands) * cx_bytes(prec));
    L.off_inter = off;
    off = align256b(off + (size_t)L.units_per_batch * (size_t)n * cx_bytes(prec));
    L.off_part = off;
    off = align256b(off + (size_t)n_units * (size_t)(p.n1 / p.b2) * sizeof(PartialChi));
    L.total = off;
    return L;
}

hipError_t launch_band_table(int64_t n, int n2, const mf_bank_entry* bank, int64_t n_tmpl, const double* prefix,
                             int p, int32_t* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_band_table, dim3((unsigned)n_tmpl), dim3(64), 0, s, n, n2, bank, prefix, p, tab);
    return hipGetLastError();
}

template <typename T, int PH, int N1, int N2, int C>
static hipError_t run_pass1_band(const FilterArgs& a, hipStream_t s) {
    static_assert(N2 % C == 0 && C <= N2, "pass-1 columns per work-group must tile N2");
    constexpr int NT = band_threads(C * N1 / 16);
    dim3 grid(N2 / C, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass1_band<T, PH, N1, N2, C, NT>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T, int N1, int N2, int B, int R2>
static hipError_t run_pass2_band(const FilterArgs& a, hipStream_t s) {
    static_assert(N1 % B == 0 && B <= N1, "pass-2 rows per work-group must tile N1");
    constexpr int NT = band_threads(B * N2 / R2);
    dim3 grid(N1 / B, (unsigned)a.units);
    hipLaunchKernelGGL((k_pass2_band<T, N1, N2, B, NT, R2>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass1_band(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s) {
#define MF_BP1(T, N1, N2, C, B, R2)                                                                             \
    if (band_want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C &&          \
        p.b2 == B) {                                                                                          \
        if (std::is_same<T, float>::value && prec == MF_FP32) return run_pass1_band<float, 1, N1, N2, C>(a, s); \
        return run_pass1_band<T, 0, N1, N2, C>(a, s);                                                         \
    }
    MF_BAND_SHAPES(MF_BP1)
#undef MF_BP1
    return hipErrorInvalidValue;
}

hipError_t launch_pass2_band(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s) {
#define MF_BP2(T, N1, N2, C, B, R2)                                                                    \
    if (band_want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C && \
        p.b2 == B && p.nt2 == band_threads(B * N2 / R2))                                             \
        return run_pass2_band<T, N1, N2, B, R2>(a, s);
    MF_BAND_SHAPES(MF_BP2)
#undef MF_BP2
    return hipErrorInvalidValue;
}

hipError_t launch_finalize_band(const Plan& p, const FilterArgs& a, mf_peak* peaks, double* chisq, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_band, dim3((unsigned)a.n_units), dim3(64), 0, s, (const PartialChi*)a.partials,
                       p.n1 / p.b2, a.bank, a.n_tmpl, a.n_seg, peaks, chisq);
    return hipGetLastError();
}

}  // namespace mf
