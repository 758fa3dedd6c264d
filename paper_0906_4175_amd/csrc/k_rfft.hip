// Forward transform of real time-domain segments into the one-sided data
// spectrum the filter consumes (arXiv:0906.4175, Sec. 3.1: the forward FFTs of
// the data are the other part of the transform time; discretisation of
// Eq. (1) as s_k = dt sum_j x_j e^{-2 pi i jk/N}, k = 0..N/2).
//
// A real N-point transform as one N/2-point complex transform: with
// y_m = x_{2m} + i x_{2m+1} and Y = DFT_{N/2}(y),
//   E_k = (Y_k + conj(Y_{N/2-k})) / 2            (transform of the even samples)
//   O_k = (Y_k - conj(Y_{N/2-k})) / (2i)         (transform of the odd samples)
//   X_k = E_k + e^{-2 pi i k / N} O_k ,  k = 0..N/2.
// The forward DFT is taken with the library's inverse two-pass transform as
// DFT(y) = conj(IDFT(conj(y))): k_rfft_pack writes conj(y), the two passes run
// in their diagnostic (raw) mode, and k_rfft_post reads conj of their output.
#include <hip/hip_runtime.h>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

template <typename T>
__global__ void k_rfft_pack(const T* x, cx<T>* y, int64_t m, int64_t total) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / m, k = i % m;
        const T* xs = x + b * 2 * m;
        y[i] = cx<T>{xs[2 * k], -xs[2 * k + 1]};
    }
}

template <typename T>
__global__ void k_rfft_post(const cx<T>* z, cx<T>* out, int64_t m, int64_t total, double dt) {
    const int64_t nb = m + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / nb, k = i % nb;
        const cx<T>* zs = z + b * m;
        const cx<T> zk = zs[k % m];            // Y_k = conj(zk)
        const cx<T> zr = zs[(m - k) % m];      // conj(Y_{m-k}) = zr
        const cx<T> yk{zk.x, -zk.y};
        const cx<T> e{(T)0.5 * (yk.x + zr.x), (T)0.5 * (yk.y + zr.y)};
        // (Y_k - conj(Y_{m-k})) / (2i) = -i/2 (Y_k - zr)
        const cx<T> d{yk.x - zr.x, yk.y - zr.y};
        const cx<T> o{(T)0.5 * d.y, (T)-0.5 * d.x};
        const cx<T> w = root_of_unity(-(T)k / (T)(2 * m));  // e^{-2 pi i k / N}
        const cx<T> x = cx<T>{e.x + (w.x * o.x - w.y * o.y), e.y + (w.x * o.y + w.y * o.x)};
        out[i] = cx<T>{(T)(x.x * (T)dt), (T)(x.y * (T)dt)};
    }
}

static unsigned grid_cover(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_rfft_pack(mf_precision prec, const void* x, void* y, int64_t m, int64_t batch, hipStream_t s) {
    const int64_t total = m * batch;
    if (prec == MF_FP64)
        hipLaunchKernelGGL(k_rfft_pack<double>, dim3(grid_cover(total, 256)), dim3(256), 0, s, (const double*)x,
                           (cx<double>*)y, m, total);
    else
        hipLaunchKernelGGL(k_rfft_pack<float>, dim3(grid_cover(total, 256)), dim3(256), 0, s, (const float*)x,
                           (cx<float>*)y, m, total);
    return hipGetLastError();
}

hipError_t launch_rfft_post(mf_precision prec, const void* z, void* out, int64_t m, int64_t batch, double dt,
                            hipStream_t s) {
    const int64_t total = (m + 1) * batch;
    if (prec == MF_FP64)
        hipLaunchKernelGGL(k_rfft_post<double>, dim3(grid_cover(total, 256)), dim3(256), 0, s, (const cx<double>*)z,
                           (cx<double>*)out, m, total, dt);
    else
        hipLaunchKernelGGL(k_rfft_post<float>, dim3(grid_cover(total, 256)), dim3(256), 0, s, (const cx<float>*)z,
                           (cx<float>*)out, m, total, dt);
    return hipGetLastError();
}

}  // namespace mf
