// rho^2 at continuous template parameters and its adjoint (gradient
// refinement of triggers off the bank grid).
//
// For theta = (M_c, eta, t_c) and a frozen band [k_lo, k_hi]:
//   Z(theta)  = 4 df sum_k a_k e^{+i Psi_k(theta)} w_k,  a_k = f_k^{-7/6},
//               w_k = s_k / S_k   (Eq. (1) of arXiv:0906.4175 at t = t_c)
//   sigma^2   = 4 df sum_k a_k^2 / S_k                   (Eq. (4))
//   F         = |Z|^2 / sigma^2                           (Eq. (3) squared)
//   dF/dth    = 2 Re(conj(Z) dZ/dth) / sigma^2,
//   dZ/dth    = 4 df sum_k i a_k w_k e^{i Psi_k} dPsi_k/dth.
// Psi/2pi is the power series sum_n b_n u^n (u = k^{-1/3}) of the 2PN
// stationary-phase phase plus -1/8 + t_c df k; the b_n depend on M_c through
// (pi M)^{e_n} with M = M_c eta^{-3/5} G M_sun / c^3, and on eta through
// 3/(128 eta), the PN coefficients and M.  One work-group reduces one trigger
// in FP64.
#include <hip/hip_runtime.h>

#include <math.h>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

// 1/x for a positive normal x: hardware estimate, then two Newton steps
// (r <- r + r (1 - x r)), each doubling the correct bits, to full FP64 precision
// (within an ulp) without the special-case handling of an IEEE division.
__device__ __forceinline__ double rcp_pos_f64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// sqrt(x) for a positive normal x: y = 1/sqrt(x) from the hardware estimate and
// two Newton steps (y <- y (3 - x y^2) / 2), then sqrt(x) = x y with one
// correction (s + y (x - s^2) / 2).
__device__ __forceinline__ double sqrt_pos_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    const double s = x * y;
    return fma(0.5 * y, fma(-s, s, x), s);
}

struct GradCoef {
    double b[4];   // u^1, u^2, u^3, u^5 coefficients (cycles)
    double dm[4];  // d b / d M_c
    double de[4];  // d b / d eta
};

__device__ __forceinline__ GradCoef grad_coef(double mc, double eta, double df) {
    const double M = mc * pow(eta, -0.6) * kTsun;
    const double x = M_PI * M * df;  // (pi M df)
    const double C = 3.0 / (128.0 * eta);
    const double inv2pi = 0.5 / M_PI;
    const double p[4] = {15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0,  // u^1
                         -16.0 * M_PI,                                                               // u^2
                         3715.0 / 756.0 + 55.0 * eta / 9.0,                                          // u^3
                         1.0};                                                                       // u^5
    const double dp[4] = {27145.0 / 504.0 + 3085.0 * eta / 36.0, 0.0, 55.0 / 9.0, 0.0};
    const double e[4] = {-1.0 / 3.0, -2.0 / 3.0, -1.0, -5.0 / 3.0};  // exponent of (pi M df)
    GradCoef g;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double xe = pow(x, e[i]);
        g.b[i] = C * p[i] * xe * inv2pi;
        g.dm[i] = g.b[i] * e[i] / mc;
        g.de[i] = g.b[i] * (-1.0 - 0.6 * e[i]) / eta + C * dp[i] * xe * inv2pi;
    }
    return g;
}

__device__ __forceinline__ double series5(const double* c, double u) {
    // c0 u + c1 u^2 + c2 u^3 + c3 u^5
    const double uu = u * u;
    return u * fma(u, fma(u, fma(uu, c[3], c[2]), c[1]), c[0]);
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_snr_grad(int64_t n, double df, double seg_T, int k_lo, const double* theta,
                                                 const int32_t* khi_in, const int32_t* seg, int64_t n_seg,
                                                 const cx<T>* stilde,
                                                 const double* Sn, double* Zout, double* rho2, const double* gbar,
                                                 double* grad) {
    constexpr int NV = 9;  // Z(2) sigma2(1) G_mc(2) G_eta(2) G_tc(2)
    __shared__ double red[NV][NT];
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const double mc = theta[3 * i + 0], eta = theta[3 * i + 1], tc = theta[3 * i + 2];
    const int64_t nb = n / 2 + 1;
    int64_t khi;
    if (khi_in) {
        khi = khi_in[i];
    } else {
        const double M = mc * pow(eta, -0.6) * kTsun;
        const double fisco = 1.0 / (sqrt(216.0) * M_PI * M);
        khi = (int64_t)floor(fisco * seg_T);
        if (khi > n / 2 - 1) khi = n / 2 - 1;
    }
    const bool do_grad = gbar != nullptr;
    const int64_t sidx = seg[i];
    if (sidx < 0 || sidx >= n_seg || khi > n / 2 - 1) {
        // invalid segment index or band edge: report NaN instead of reading out of range
        if (tid == 0) {
            Zout[2 * i] = NAN;
            Zout[2 * i + 1] = NAN;
            rho2[i] = NAN;
            if (do_grad)
                for (int q = 0; q < 3; ++q) grad[3 * i + q] = NAN;
        }
        return;
    }
    const GradCoef g = grad_coef(mc, eta, df);
    const double bt = tc * df;
    const cx<T>* s = stilde + sidx * nb;
    const double amp0 = pow(df, -7.0 / 6.0);

    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const int khi32 = (int)khi;  // bins < N/2 <= 2^21
    for (int k = k_lo + tid; k <= khi32; k += NT) {
        const double kd = (double)k;
        const double u = inv_cbrt_f64_full(kd);
        double ph = series5(g.b, u) + fma(bt, kd, -0.125);
        ph -= rint(ph);
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double a = amp0 * u * u * u * sqrt_pos_f64(u);  // f^{-7/6} = df^{-7/6} u^{7/2}
        const double invS = rcp_pos_f64(Sn[k]);                // S > 0 inside the band
        const cx<T> sv = s[k];
        const double wr = (double)sv.x * invS * a, wi = (double)sv.y * invS * a;
        const double tr = wr * cs - wi * sn, ti = wr * sn + wi * cs;  // a w e^{i Psi}
        acc[0] += tr;
        acc[1] += ti;
        acc[2] += a * a * invS;
        if (do_grad) {
            const double dmc = series5(g.dm, u);
            const double deta = series5(g.de, u);
            const double dtc = df * kd;
            acc[3] += tr * dmc;
            acc[4] += ti * dmc;
            acc[5] += tr * deta;
            acc[6] += ti * deta;
            acc[7] += tr * dtc;
            acc[8] += ti * dtc;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][tid] = acc[v];
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (tid < off) {
#pragma unroll
            for (int v = 0; v < NV; ++v) red[v][tid] += red[v][tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double c = 4.0 * df;
        const double Zr = c * red[0][0], Zi = c * red[1][0];
        const double s2 = c * red[2][0];
        const double F = (Zr * Zr + Zi * Zi) / s2;
        Zout[2 * i] = Zr;
        Zout[2 * i + 1] = Zi;
        rho2[i] = khi >= k_lo ? F : NAN;
        if (do_grad) {
            // dZ = c * 2 pi * i * G ;  dF = 2 Re(conj(Z) dZ) / s2 = 2 c 2pi (Zi Gr - Zr Gi) / s2
            const double fac = 2.0 * c * 2.0 * M_PI / s2 * gbar[i];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double Gr = red[3 + 2 * q][0], Gi = red[4 + 2 * q][0];
                grad[3 * i + q] = fac * (Zi * Gr - Zr * Gi);
            }
        }
    }
}

// Template-space metric at theta over the frozen band: with weights
// W_k = f_k^{-7/3} / S_k (= |h_k|^2 / S_k) and d_k = dPsi_k / dtheta (radians),
//   g_ij = <d_i d_j> - <d_i><d_j>,  <x> = sum_k W_k x_k / sum_k W_k,
// the phase-maximised mismatch metric: near a maximum of rho^2,
// F(theta + delta) ~ F(theta) (1 - g_ij delta_i delta_j).  Output per trigger:
// (g_mm, g_me, g_mt, g_ee, g_et, g_tt).
template <int NT>
__global__ void __launch_bounds__(NT) k_metric(int64_t n, double df, int k_lo, const double* theta,
                                               const int32_t* khi_in, const double* Sn, double* metric) {
    constexpr int NV = 10;  // W, W d_i (3), W d_i d_j (6)
    __shared__ double red[NV][NT];
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const double mc = theta[3 * i + 0], eta = theta[3 * i + 1];
    int64_t khi = khi_in[i];
    if (khi > n / 2 - 1) khi = n / 2 - 1;
    const GradCoef g = grad_coef(mc, eta, df);
    const double amp2 = pow(df, -7.0 / 3.0);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const int khi32 = (int)khi;  // bins < N/2 <= 2^21
    for (int k = k_lo + tid; k <= khi32; k += NT) {
        const double kd = (double)k;
        const double u = inv_cbrt_f64_full(kd);
        const double u7 = u * u * u * u * u * u * u;
        const double W = amp2 * u7 / Sn[k];  // f^{-7/3} / S
        const double d0 = 2.0 * M_PI * series5(g.dm, u);
        const double d1 = 2.0 * M_PI * series5(g.de, u);
        const double d2 = 2.0 * M_PI * df * kd;
        acc[0] += W;
        acc[1] += W * d0;
        acc[2] += W * d1;
        acc[3] += W * d2;
        acc[4] += W * d0 * d0;
        acc[5] += W * d0 * d1;
        acc[6] += W * d0 * d2;
        acc[7] += W * d1 * d1;
        acc[8] += W * d1 * d2;
        acc[9] += W * d2 * d2;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][tid] = acc[v];
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (tid < off) {
#pragma unroll
            for (int v = 0; v < NV; ++v) red[v][tid] += red[v][tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double w = red[0][0];
        const double m0 = red[1][0] / w, m1 = red[2][0] / w, m2 = red[3][0] / w;
        double* out = metric + 6 * i;
        out[0] = red[4][0] / w - m0 * m0;
        out[1] = red[5][0] / w - m0 * m1;
        out[2] = red[6][0] / w - m0 * m2;
        out[3] = red[7][0] / w - m1 * m1;
        out[4] = red[8][0] / w - m1 * m2;
        out[5] = red[9][0] / w - m2 * m2;
    }
}

hipError_t launch_metric(int64_t n, double fs, int k_lo, const double* theta, const int32_t* khi, int64_t count,
                         const double* Sn, double* metric, hipStream_t s) {
    const double df = fs / (double)n;
    constexpr int NT = 256;
    hipLaunchKernelGGL((k_metric<NT>), dim3((unsigned)count), dim3(NT), 0, s, n, df, k_lo, theta, khi, Sn, metric);
    return hipGetLastError();
}

hipError_t launch_snr_grad(int64_t n, double fs, int k_lo, mf_precision prec, const double* theta,
                           const int32_t* khi, const int32_t* seg, int64_t count, const void* stilde,
                           int64_t n_seg, const double* Sn, double* Z, double* rho2, const double* gbar, double* grad,
                           hipStream_t s) {
    const double df = fs / (double)n;
    constexpr int NT = 256;
    if (prec == MF_FP64)
        hipLaunchKernelGGL((k_snr_grad<double, NT>), dim3((unsigned)count), dim3(NT), 0, s, n, df, (double)n / fs, k_lo, theta, khi,
                           seg, n_seg, (const cx<double>*)stilde, Sn, Z, rho2, gbar, grad);
    else
        hipLaunchKernelGGL((k_snr_grad<float, NT>), dim3((unsigned)count), dim3(NT), 0, s, n, df, (double)n / fs, k_lo, theta, khi,
                           seg, n_seg, (const cx<float>*)stilde, Sn, Z, rho2, gbar, grad);
    return hipGetLastError();
}

}  // namespace mf
