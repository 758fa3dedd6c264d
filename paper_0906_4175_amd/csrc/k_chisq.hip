// chi^2 time-frequency veto of arXiv:0906.4175, Eq. (5) (Sec. 1.2), evaluated
// at single samples j: each unit's peak, or listed events (template t,
// segment s, sample j):
//   z_l(j) = 4 df sum_{k in band l} conj(h_k) s_k / S_k e^{2 pi i j k / N}
//   chi^2  = p / sigma^2 sum_l |z_l - z / p|^2 = p / sigma^2 (sum_l |z_l|^2 - |z|^2 / p),
// using sum_l z_l = z.  The p bands split the template's band into equal
// shares of sigma^2 (Eq. (4)); a bin belongs to the band in which the sum of
// f^{-7/3}/S over the bins before it falls.  Band edges come from binary
// searches in the FP64 prefix sums of mf_psd.  One work-group per sample;
// FP64 phase (the time shift j k / N is reduced exactly in integers) and FP64
// sums; for FP32 data the weight and the rotor of the reduced phase are FP32
// (hardware sine and cosine of a fraction of a cycle), as in the filter.
#include <hip/hip_runtime.h>

#include <math.h>

#include <type_traits>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

constexpr int kMaxBands = 64;

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tot += scratch[w];
    return tot;
}

// One work-group per output: a unit's peak (peaks != nullptr; output u =
// t * n_seg + s) or an event record (events [n_seg][n_per_seg]; entries with
// t < 0 give 0).
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_chisq(int64_t n, double df, const mf_bank_entry* bank, int64_t n_tmpl,
                                              int64_t n_seg, const cx<T>* stilde, const double* Sn, const double* P,
                                              int p, const mf_peak* peaks, const mf_event* events, int64_t n_per_seg,
                                              double* chisq, double* rho_out) {
    __shared__ int64_t edge[kMaxBands + 1];
    __shared__ double zr[kMaxBands], zi[kMaxBands];
    __shared__ double scratch[NT / 64];
    const int tid = threadIdx.x;
    const int64_t u = blockIdx.x;
    int64_t t, s, j;
    if (events) {
        const mf_event ev = events[u];
        if (ev.t < 0) {
            if (tid == 0) {
                chisq[u] = 0.0;
                if (rho_out) rho_out[u] = 0.0;
            }
            return;
        }
        t = ev.t;
        s = u / n_per_seg;
        j = ev.j;
    } else {
        t = u / n_seg;
        s = u % n_seg;
        j = peaks[u].j;
    }
    const mf_bank_entry e = bank[t < n_tmpl ? t : 0];
    const int64_t klo = e.k_lo, khi = e.k_hi;
    if (t >= n_tmpl || j < 0 || j >= n || khi > n / 2 - 1 || klo < 1 || khi < klo) {
        if (tid == 0) {
            chisq[u] = NAN;
            if (rho_out) rho_out[u] = NAN;
        }
        return;
    }
    // equal-share band edges: e_l = min{k : P[k-1] - P[klo-1] >= l/p * (P[khi] - P[klo-1])}
    if (tid == 0) {
        edge[0] = klo;
        edge[p] = khi + 1;
    }
    if (tid >= 1 && tid < p) {
        const double base = P[klo - 1];
        const double target = (double)tid / (double)p * (P[khi] - base);
        int64_t lo = klo + 1, hi = khi + 1;  // answer in [klo+1, khi+1]
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (P[mid - 1] - base >= target) hi = mid; else lo = mid + 1;
        }
        edge[tid] = lo;
    }
    __syncthreads();
    const PhaseCoef pc = load_coef(e);
    const double c4 = 4.0 * df * pow(df, -7.0 / 6.0);  // 4 df f^{-7/6} = c4 k^{-7/6}
    const double inv_n = 1.0 / (double)n;                // exact: n is a power of two
    const float c4f = (float)c4;
    const cx<T>* sp = stilde + s * (n / 2 + 1);
    // n <= 2^23, so bins and (j k mod n) fit 32-bit integers: the product is
    // taken mod 2^32, which n divides
    const unsigned int nmask = (unsigned int)(n - 1), ju = (unsigned int)j;
    for (int l = 0; l < p; ++l) {
        double ar = 0.0, ai = 0.0;
        for (int k = (int)edge[l] + tid; k < (int)edge[l + 1]; k += NT) {
            const double kd = (double)k;
            // k^{-1/3}: relative error ~1e-13 after one FP64 Newton step, ~1e-16 after two
            const double u = sizeof(T) == 4 ? inv_cbrt_f64(kd) : inv_cbrt_f64_full(kd);
            const double uu = u * u;
            double ph = fma(u, fma(u, fma(u, fma(uu, pc.b5, pc.b3), pc.b2), pc.b1), pc.c0);
            ph -= rint(ph);
            ph += (double)((ju * (unsigned int)k) & nmask) * inv_n;  // time shift, exact
            ph -= rint(ph);
            const cx<T> sv = sp[k];
            if constexpr (sizeof(T) == 4) {
                // FP32 data: FP32 weight (hardware square root and reciprocal,
                // about 1 ulp each) and hardware rotor of the reduced FP64 phase
                const float uf = (float)u;
                const float g = c4f * uf * uf * uf * __builtin_amdgcn_sqrtf(uf) * __builtin_amdgcn_rcpf((float)Sn[k]);
                const cx<float> rot = rotor_rev((float)ph);
                const float wr = sv.x * g, wi = sv.y * g;
                ar += (double)(wr * rot.x - wi * rot.y);
                ai += (double)(wr * rot.y + wi * rot.x);
            } else {
                double sn, cs;
                sincospi(2.0 * ph, &sn, &cs);
                const double g = c4 * u * uu * sqrt(u) / Sn[k];
                const double wr = sv.x * g, wi = sv.y * g;
                ar += wr * cs - wi * sn;
                ai += wr * sn + wi * cs;
            }
        }
        ar = block_sum<NT>(ar, scratch);
        ai = block_sum<NT>(ai, scratch);
        if (tid == 0) {
            zr[l] = ar;
            zi[l] = ai;
        }
    }
    if (tid == 0) {
        double sr = 0.0, si = 0.0, sq = 0.0;
        for (int l = 0; l < p; ++l) {
            sr += zr[l];
            si += zi[l];
            sq += zr[l] * zr[l] + zi[l] * zi[l];
        }
        const double s2 = e.sigma * e.sigma;
        const double zz = sr * sr + si * si;
        chisq[u] = (double)p / s2 * (sq - zz / (double)p);
        if (rho_out) rho_out[u] = sqrt(zz) / e.sigma;
    }
}

hipError_t launch_chisq(int64_t n, double fs, mf_precision prec, const mf_bank_entry* bank, int64_t n_tmpl,
                        const void* stilde, int64_t n_seg, const double* Sn, const double* prefix, int p,
                        const mf_peak* peaks, const mf_event* events, int64_t n_per_seg, double* chisq, double* rho,
                        hipStream_t s) {
    const double df = fs / (double)n;
    const unsigned blocks = (unsigned)(events ? n_seg * n_per_seg : n_tmpl * n_seg);
    // Events are few (often fewer than the CUs): a work-group of 1024 threads
    // per event halves the time of each and of the launch's tail.
    auto go = [&](auto nt_) {
        constexpr int NT = decltype(nt_)::value;
        if (prec == MF_FP64)
            hipLaunchKernelGGL((k_chisq<double, NT>), dim3(blocks), dim3(NT), 0, s, n, df, bank, n_tmpl, n_seg,
                               (const cx<double>*)stilde, Sn, prefix, p, peaks, events, n_per_seg, chisq, rho);
        else
            hipLaunchKernelGGL((k_chisq<float, NT>), dim3(blocks), dim3(NT), 0, s, n, df, bank, n_tmpl, n_seg,
                               (const cx<float>*)stilde, Sn, prefix, p, peaks, events, n_per_seg, chisq, rho);
    };
    if (events)
        go(std::integral_constant<int, 1024>{});
    else
        go(std::integral_constant<int, 512>{});
    return hipGetLastError();
}

}  // namespace mf
