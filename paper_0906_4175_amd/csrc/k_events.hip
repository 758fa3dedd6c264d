// Events of arXiv:0906.4175, Sec. 3.3 (triggers reported with their SNR and
// chi^2): threshold and clustering of rho(t).  The paper gives no rule; the
// one used here (series cut into windows of W = 2^log2w samples):
//  * time clustering, per (template, segment) unit: a window's winner is its
//    loudest sample at or above rho_th (pass 2 keeps it in a u64 key per
//    window); it is an event unless the winner of an adjacent window lies
//    within W samples of it with a larger rho (or an equal rho at a lower
//    index);
//  * template clustering, per segment: each window's loudest unit event
//    across templates (ties: lowest template index), kept under the same
//    adjacent-window rule.
// One thread per (unit or segment, window), one wave per segment window for
// the template maximum; deterministic, no atomics.
#include <hip/hip_runtime.h>

#include <math.h>

#include "mf_device.hpp"
#include "mf_internal.hpp"

namespace mf {

struct KeyVal {
    bool has;
    double zz;
    int64_t j;
};

// Inverse of event_key32 / event_key64 (pass 2).
__device__ __forceinline__ KeyVal decode_key(unsigned long long key, bool f64, int64_t w, int log2w) {
    KeyVal v{key != 0ull, 0.0, 0};
    if (!v.has) return v;
    if (f64) {
        v.zz = __longlong_as_double((long long)(key & ~0xffffull));
        v.j = (w << log2w) + (int64_t)(0xffffu - (unsigned int)(key & 0xffffull));
    } else {
        v.zz = (double)__uint_as_float((unsigned int)(key >> 32));
        v.j = (int64_t)(0xffffffffu - (unsigned int)(key & 0xffffffffull));
    }
    return v;
}

__device__ __forceinline__ bool beats(double v2, int64_t j2, double v, int64_t j) {
    return v2 > v || (v2 == v && j2 < j);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// keys [n_units][n_win] in batch order u = s * n_tmpl + t; unit_ev [n_tmpl][n_seg][n_win]
__global__ void k_events_unit(const unsigned long long* keys, int64_t n_tmpl, int64_t n_seg, int64_t n_win,
                              int log2w, bool f64, const mf_bank_entry* bank, mf_event* unit_ev) {
    const int64_t total = n_tmpl * n_seg * n_win;
    const int64_t W = (int64_t)1 << log2w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = i / n_win, w = i % n_win;
        const int64_t t = u % n_tmpl, s = u / n_tmpl;
        const unsigned long long* ku = keys + u * n_win;
        const KeyVal me = decode_key(ku[w], f64, w, log2w);
        bool keep = me.has;
        if (keep) {
#pragma unroll
            for (int d = -1; d <= 1; d += 2) {
                const int64_t w2 = w + d;
                if (w2 < 0 || w2 >= n_win) continue;
                const KeyVal o = decode_key(ku[w2], f64, w2, log2w);
                if (o.has && llabs(o.j - me.j) <= W && beats(o.zz, o.j, me.zz, me.j)) keep = false;
            }
        }
        mf_event ev;
        ev.rho = keep ? sqrt(me.zz) / bank[t].sigma : 0.0;
        ev.j = keep ? (int32_t)me.j : -1;
        ev.t = keep ? (int32_t)t : -1;
        unit_ev[(t * n_seg + s) * n_win + w] = ev;
    }
}

// e beats b: an event against none, a larger rho, or an equal rho of a lower template
__device__ __forceinline__ bool louder(const mf_event& e, const mf_event& b) {
    if (e.t < 0) return false;
    if (b.t < 0) return true;
    return e.rho > b.rho || (e.rho == b.rho && e.t < b.t);
}

// loudest unit event of each (segment, window) across templates: one 64-lane
// wave per (segment, window), lanes stride over the templates
__global__ void __launch_bounds__(256) k_events_best(const mf_event* unit_ev, int64_t n_tmpl, int64_t n_seg,
                                                     int64_t n_win, mf_event* best) {
    const int64_t total = n_seg * n_win;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < total; i += waves) {
        const int64_t s = i / n_win, w = i % n_win;
        mf_event b{0.0, -1, -1};
        for (int64_t t = lane; t < n_tmpl; t += 64) {
            const mf_event e = unit_ev[(t * n_seg + s) * n_win + w];
            if (louder(e, b)) b = e;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mf_event o;
            o.rho = __shfl_xor(b.rho, off, 64);
            o.j = __shfl_xor(b.j, off, 64);
            o.t = __shfl_xor(b.t, off, 64);
            if (louder(o, b)) b = o;
        }
        if (lane == 0) best[i] = b;
    }
}

// adjacent-window rule on the segment winners
__global__ void k_events_merge(const mf_event* best, int64_t n_seg, int64_t n_win, int log2w, mf_event* seg_ev) {
    const int64_t total = n_seg * n_win;
    const int64_t W = (int64_t)1 << log2w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = i % n_win;
        const mf_event me = best[i];
        bool keep = me.t >= 0;
        if (keep) {
#pragma unroll
            for (int d = -1; d <= 1; d += 2) {
                const int64_t w2 = w + d;
                if (w2 < 0 || w2 >= n_win) continue;
                const mf_event o = best[i + d];
                if (o.t >= 0 && llabs((int64_t)o.j - (int64_t)me.j) <= W && beats(o.rho, o.j, me.rho, me.j))
                    keep = false;
            }
        }
        seg_ev[i] = keep ? me : mf_event{0.0, -1, -1};
    }
}

static unsigned cover(int64_t total) {
    const int64_t g = (total + 255) / 256;
    return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(cover(count)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_events(const unsigned long long* keys, int64_t n_tmpl, int64_t n_seg, int64_t n_win, int log2w,
                         bool f64, const mf_bank_entry* bank, mf_event* unit_ev, mf_event* best, mf_event* seg_ev,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_events_unit, dim3(cover(n_tmpl * n_seg * n_win)), dim3(256), 0, s, keys, n_tmpl, n_seg,
                       n_win, log2w, f64, bank, unit_ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t wave_blocks = (n_seg * n_win + 3) / 4;  // four waves per block
    hipLaunchKernelGGL(k_events_best, dim3((unsigned)(wave_blocks > 65536 ? 65536 : wave_blocks)), dim3(256), 0, s,
                       unit_ev, n_tmpl, n_seg, n_win, best);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_events_merge, dim3(cover(n_seg * n_win)), dim3(256), 0, s, best, n_seg, n_win, log2w,
                       seg_ev);
    return hipGetLastError();
}

}  // namespace mf
