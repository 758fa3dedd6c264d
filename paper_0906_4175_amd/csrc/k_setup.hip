// Setup kernels of libmf: the analytic PSD of Eq. (2), the per-segment data
// weights, the template norm of Eq. (4) and the materialised stationary-phase
// template (arXiv:0906.4175, Sec. 1.1).
#include <hip/hip_runtime.h>

#include <math.h>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

// Eq. (2): S_n(f) = (4.49 f/f0)^-56 + 0.16 (f/f0)^-4.52 + 0.52 + 0.32 (f/f0)^2
__device__ __forceinline__ double psd_eq2(double f, double f0) {
    const double x = f / f0;
    return pow(4.49 * x, -56.0) + 0.16 * pow(x, -4.52) + 0.52 + 0.32 * x * x;
}

__global__ void k_psd(int64_t n, double df, double f0, int k_lo, double* Sn) {
    const int64_t nb = n / 2 + 1;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
        Sn[k] = (k >= k_lo && k < n / 2) ? psd_eq2((double)k * df, f0) : INFINITY;
    }
}

// P_k = sum_{k' <= k} f_k'^(-7/3) / S_k'  (one work-group; setup only)
__global__ void __launch_bounds__(1024) k_prefix(int64_t nb, double df, const double* Sn, double* P) {
    __shared__ double part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (nb + 1023) / 1024;
    const int64_t b = tid * chunk;
    const int64_t e = b + chunk < nb ? b + chunk : nb;
    double acc = 0.0;
    for (int64_t k = b; k < e; ++k) {
        const double S = Sn[k];
        if (isfinite(S) && k > 0) acc += pow((double)k * df, -7.0 / 3.0) / S;
    }
    part[tid] = acc;
    __syncthreads();
    // exclusive scan of the chunk sums (Hillis-Steele in place, then shift)
    for (int off = 1; off < 1024; off <<= 1) {
        const double add = tid >= off ? part[tid - off] : 0.0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    double run = tid > 0 ? part[tid - 1] : 0.0;
    for (int64_t k = b; k < e; ++k) {
        const double S = Sn[k];
        if (isfinite(S) && k > 0) run += pow((double)k * df, -7.0 / 3.0) / S;
        P[k] = run;
    }
}

// w_k = 4 df f_k^(-7/6) s_k / S_k on [k_lo, N/2-1], 0 elsewhere.
template <typename T>
__global__ void k_weights(int64_t n, double df, int k_lo, const cx<T>* stilde, int64_t n_seg, const double* Sn,
                          cx<T>* w) {
    const int64_t nb = n / 2 + 1;
    const int64_t total = nb * n_seg;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i % nb;
        cx<T> out{T(0), T(0)};
        if (k >= k_lo && k < n / 2) {
            const double g = 4.0 * df * pow((double)k * df, -7.0 / 6.0) / Sn[k];
            const cx<T> sv = stilde[i];
            out = cx<T>{(T)((double)sv.x * g), (T)((double)sv.y * g)};
        }
        w[i] = out;
    }
}

// sigma^2 = 4 df sum_{k=k_lo}^{k_hi} f_k^(-7/3) / S_k, one work-group per template.
template <int MODE>
__global__ void __launch_bounds__(256) k_sigma(double df, const double* Sn, mf_bank_entry* bank) {
    __shared__ double sh[256];
    __shared__ float shf[256];
    __shared__ float shc[256];
    const int tid = threadIdx.x;
    mf_bank_entry* e = bank + blockIdx.x;
    const int64_t klo = e->k_lo, khi = e->k_hi;
    if (MODE == MF_SIGMA_FP64) {
        double acc = 0.0;
        for (int64_t k = klo + tid; k <= khi; k += 256) acc += pow((double)k * df, -7.0 / 3.0) / Sn[k];
        sh[tid] = acc;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off) sh[tid] += sh[tid + off];
            __syncthreads();
        }
        if (tid == 0) {
            const double s2 = 4.0 * df * sh[0];
            e->sigma = sqrt(s2);
            e->inv_sigma = (float)(1.0 / e->sigma);
        }
    } else {
        // Kahan-compensated FP32 per thread, then a compensated pairwise tree.
        float sum = 0.0f, comp = 0.0f;
        for (int64_t k = klo + tid; k <= khi; k += 256) {
            const float term = (float)(pow((double)k * df, -7.0 / 3.0) / Sn[k]);
            const float y = term - comp;
            const float t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        }
        shf[tid] = sum;
        shc[tid] = comp;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off) {
                // two-sum of the partial sums, carrying both compensations
                const float a = shf[tid], b = shf[tid + off];
                const float s = a + b;
                const float bb = s - a;
                const float err = (a - (s - bb)) + (b - bb);
                shf[tid] = s;
                shc[tid] = shc[tid] + shc[tid + off] - err;
            }
            __syncthreads();
        }
        if (tid == 0) {
            const float s2 = 4.0f * (float)df * (shf[0] - shc[0]);
            e->sigma = (double)sqrtf(s2);
            e->inv_sigma = 1.0f / sqrtf(s2);
        }
    }
}

// h_c(f_k) = f_k^(-7/6) e^{-i Psi_k} in band, 0 outside.
template <typename T>
__global__ void k_spa_synth(int64_t n, double df, const mf_bank_entry* bank, cx<T>* h) {
    const int64_t nb = n / 2 + 1;
    const mf_bank_entry e = bank[blockIdx.y];
    const PhaseCoef p = load_coef(e);
    cx<T>* out = h + (int64_t)blockIdx.y * nb;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
        cx<T> v{T(0), T(0)};
        if (k >= e.k_lo && k <= e.k_hi) {
            double ph = spa_cycles_f64(p, (double)k);
            ph -= rint(ph);
            const double a = pow((double)k * df, -7.0 / 6.0);
            if constexpr (sizeof(T) == 8) {
                double sn, cs;
                sincospi(2.0 * ph, &sn, &cs);
                v = cx<T>{(T)(a * cs), (T)(-a * sn)};
            } else {
                float sn, cs;
                sincospif(2.0f * (float)ph, &sn, &cs);
                v = cx<T>{(T)(a * cs), (T)(-a * sn)};
            }
        }
        out[k] = v;
    }
}

static unsigned grid_for(int64_t work, int threads, unsigned cap = 65536) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    return (unsigned)(b > cap ? cap : b);
}

hipError_t launch_psd(int64_t n, double fs, double f_low, double f0, int k_lo, double* Sn, hipStream_t s) {
    (void)f_low;
    const double df = fs / (double)n;
    hipLaunchKernelGGL(k_psd, dim3(grid_for(n / 2 + 1, 256)), dim3(256), 0, s, n, df, f0, k_lo, Sn);
    return hipGetLastError();
}

hipError_t launch_prefix(int64_t n, double fs, const double* Sn, double* prefix, hipStream_t s) {
    const double df = fs / (double)n;
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, s, n / 2 + 1, df, Sn, prefix);
    return hipGetLastError();
}

hipError_t launch_weights(int64_t n, double fs, int k_lo, mf_precision prec, const void* stilde, int64_t n_seg,
                          const double* Sn, void* wgt, hipStream_t s) {
    const double df = fs / (double)n;
    const unsigned g = grid_for((n / 2 + 1) * n_seg, 256);
    if (prec == MF_FP64)
        hipLaunchKernelGGL(k_weights<double>, dim3(g), dim3(256), 0, s, n, df, k_lo, (const cx<double>*)stilde, n_seg,
                           Sn, (cx<double>*)wgt);
    else
        hipLaunchKernelGGL(k_weights<float>, dim3(g), dim3(256), 0, s, n, df, k_lo, (const cx<float>*)stilde, n_seg,
                           Sn, (cx<float>*)wgt);
    return hipGetLastError();
}

hipError_t launch_sigma(int64_t n, double fs, mf_sigma_mode mode, const double* Sn, mf_bank_entry* bank,
                        int64_t n_tmpl, hipStream_t s) {
    const double df = fs / (double)n;
    if (mode == MF_SIGMA_FP64)
        hipLaunchKernelGGL(k_sigma<MF_SIGMA_FP64>, dim3((unsigned)n_tmpl), dim3(256), 0, s, df, Sn, bank);
    else
        hipLaunchKernelGGL(k_sigma<MF_SIGMA_COMP32>, dim3((unsigned)n_tmpl), dim3(256), 0, s, df, Sn, bank);
    return hipGetLastError();
}

hipError_t launch_spa_synth(int64_t n, double fs, mf_precision prec, const mf_bank_entry* bank, int64_t n_tmpl,
                            void* htilde, hipStream_t s) {
    const double df = fs / (double)n;
    dim3 grid(grid_for(n / 2 + 1, 256, 1024), (unsigned)n_tmpl);
    if (prec == MF_FP64)
        hipLaunchKernelGGL(k_spa_synth<double>, grid, dim3(256), 0, s, n, df, bank, (cx<double>*)htilde);
    else
        hipLaunchKernelGGL(k_spa_synth<float>, grid, dim3(256), 0, s, n, df, bank, (cx<float>*)htilde);
    return hipGetLastError();
}

}  // namespace mf
