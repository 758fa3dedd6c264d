// Persistent pass 1 of the matched filter (plan flag bit 5): one work order per
// batch, longest first, then resident work-groups that take pass-1 tiles from a
// queue.  The tile itself is Pass1 of filter_tiles.hpp, as in k_filter.hip.
#include <hip/hip_runtime.h>

#include <atomic>

#include "filter_shapes.hpp"
#include "filter_tiles.hpp"

namespace mf {

// Persistent pass 1: as many work-groups as stay resident take tiles from a
// queue (one atomic per tile) in the order k_lpt_order wrote, so the units with
// the most band rows start first.  Every work-group leaves once the counter has
// passed the batch's tiles.
template <typename T, int PH, int MODE, int N1, int N2, int C, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass1_min_waves<T, NT>())))
k_pass1_lpt(FilterArgs a) {
    using P = Pass1<T, PH, MODE, N1, N2, C, NT>;
    __shared__ __align__(16) char smem[P::SMEM];
    __shared__ int item;
    constexpr int W = N2 / C;  // tiles per unit
    const int total = (int)a.units * W;
    for (;;) {
        if (threadIdx.x == 0) item = (int)atomicAdd(a.lpt_ctr, 1u);
        __syncthreads();
        const int w = item;
        if (w >= total) break;  // uniform over the work-group
        P::run(a, smem, w % W, a.lpt_order[w / W]);
        __syncthreads();  // the next tile reuses the LDS and `item`
    }
}

// Work order of a persistent pass-1 batch, longest first: the batch's units by
// the number of product rows their template fills (rows k1 <= k_hi / N2, in
// kLptBuckets classes), most first, by a counting sort; the order within a
// class is arbitrary and changes no result.  Also resets the queue counter.
constexpr int kLptBuckets = 64;
static_assert(kLptBuckets == 64, "the class prefix below is one wave of 64 lanes");
__global__ void __launch_bounds__(1024) k_lpt_order(const mf_bank_entry* bank, int64_t n_tmpl, int64_t unit0,
                                                    int units, int n2, int half_rows, int32_t* order,
                                                    unsigned int* ctr) {
    __shared__ int pos[kLptBuckets];
    const int tid = threadIdx.x;
    if (tid < kLptBuckets) pos[tid] = 0;
    __syncthreads();
    auto bucket = [&](int i) {
        const mf_bank_entry e = bank[(unit0 + i) % n_tmpl];  // u = s n_tmpl + t
        const int64_t rows = e.k_hi >= e.k_lo ? e.k_hi / n2 + 1 : 0;  // <= half_rows
        const int64_t c = rows * kLptBuckets / (half_rows + 1);
        return (int)(c < kLptBuckets - 1 ? c : kLptBuckets - 1);
    };
    for (int i = tid; i < units; i += 1024) atomicAdd(&pos[bucket(i)], 1);
    __syncthreads();
    if (tid < 64) {
        // exclusive prefix over the classes from the heaviest down (one wave)
        const int c = pos[kLptBuckets - 1 - tid];
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (tid >= o) incl += v;
        }
        pos[kLptBuckets - 1 - tid] = incl - c;
        if (tid == 0) *ctr = 0u;
    }
    __syncthreads();
    for (int i = tid; i < units; i += 1024) order[atomicAdd(&pos[bucket(i)], 1)] = i;
}

// resident work-groups of a kernel on the current device (occupancy x CUs)
static hipError_t resident_groups(const void* kern, int nt, std::atomic<int>& per_cu, int64_t* out) {
    if (per_cu.load() == 0) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, nt, 0);
        if (e != hipSuccess) return e;
        per_cu.store(nb < 1 ? 1 : nb);
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *out = (int64_t)per_cu.load() * cus;
    return hipSuccess;
}

template <typename T, int PH, int MODE, int N1, int N2, int C>
static hipError_t run_pass1_lpt(const FilterArgs& a, hipStream_t s) {
    constexpr int NT = clamp_threads(C * N1 / 16);
    auto kern = k_pass1_lpt<T, PH, MODE, N1, N2, C, NT>;
    static std::atomic<int> per_cu{0};  // resident work-groups per CU (a property of the kernel)
    int64_t resident = 0;
    hipError_t e = resident_groups((const void*)kern, NT, per_cu, &resident);
    if (e != hipSuccess) return e;
    const int64_t tiles = a.units * (N2 / C);
    const int64_t grid = tiles < resident ? tiles : resident;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass1_lpt(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s) {
    if (a.units <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lpt_order, dim3(1), dim3(1024), 0, s, a.bank, a.n_tmpl, a.unit0, (int)a.units, p.n2,
                       p.n1 / 2, (int32_t*)a.lpt_order, a.lpt_ctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define MF_P1L(T, N1, N2, C, B, R2, XS)                                                                         \
    if (want(prec, std::is_same<T, double>::value) && p.n1 == N1 && p.n2 == N2 && p.c1 == C && p.b2 == B) {    \
        if (a.pre0_r0 > 0) {                                                                                   \
            if (std::is_same<T, float>::value && prec == MF_FP32)                                              \
                return run_pass1_lpt<float, 1, P1_PRODUCT_PRE, N1, N2, C>(a, s);                               \
            return run_pass1_lpt<T, 0, P1_PRODUCT_PRE, N1, N2, C>(a, s);                                       \
        }                                                                                                      \
        if (std::is_same<T, float>::value && prec == MF_FP32)                                                  \
            return run_pass1_lpt<float, 1, P1_PRODUCT, N1, N2, C>(a, s);                                       \
        return run_pass1_lpt<T, 0, P1_PRODUCT, N1, N2, C>(a, s);                                               \
    }
    MF_SHAPES(MF_P1L)
#undef MF_P1L
    return hipErrorInvalidValue;
}

}  // namespace mf
