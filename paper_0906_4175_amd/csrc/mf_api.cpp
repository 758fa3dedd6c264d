// extern "C" entry points of libmf (include/mf.h): argument validation,
// host-side FP64 template coefficients and band edges, workspace carve-up and
// the launch sequence of the matched filter.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mf.h"
#include "mf_internal.hpp"

namespace {

thread_local std::string g_err;

// Measurement hook state (event pairs around sampled pass launches).
struct TimedLaunch {
    hipEvent_t start, stop;
    int64_t units1, units2;  // units of the pass-1 and pass-2 roles in the launch
};
struct TimingState {
    int32_t stride = 0;
    int64_t batch_counter = 0;
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
};
TimingState g_timing;

hipEvent_t timing_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

mf_status fail(mf_status st, const char* fmt, ...);
mf_status hip_fail(hipError_t e, const char* where);

// Runs launch(); every stride-th call gets an event pair on the stream
// (measurement hook).  units1 / units2: units of the pass-1 / pass-2 roles.
template <typename F>
mf_status timed_launch(hipStream_t s, int64_t units1, int64_t units2, F&& launch) {
    const bool timed = g_timing.stride > 0 && (g_timing.batch_counter++ % g_timing.stride) == 0;
    TimedLaunch t{};
    if (timed) {
        t = TimedLaunch{timing_event(), timing_event(), units1, units2};
        if (!t.start || !t.stop) return fail(MF_E_HIP, "timing event creation failed");
        hipEventRecord(t.start, s);
    }
    hipError_t le = launch();
    if (le != hipSuccess) return hip_fail(le, "pass launch");
    if (timed) {
        hipEventRecord(t.stop, s);
        g_timing.pending.push_back(t);
    }
    return MF_OK;
}

mf_status fail(mf_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mf_status ok() {
    g_err.clear();
    return MF_OK;
}

mf_status hip_fail(hipError_t e, const char* where) {
    return fail(MF_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool valid_prec(mf_precision p) { return p == MF_FP64 || p == MF_FP32_PH64 || p == MF_FP32; }

int log2_exact(int64_t n) {
    if (n <= 0 || (n & (n - 1)) != 0) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

// Validates the grid; k_lo = ceil(f_low T) is the first band bin.
mf_status check_grid(const mf_grid* g, int* log2n, int* k_lo) {
    if (!g) return fail(MF_E_ARG, "grid is null");
    const int l = log2_exact(g->n);
    if (l < mf::kMinLog2N || l > mf::kMaxLog2N)
        return fail(MF_E_SHAPE, "n=%lld must be a power of two in [2^%d, 2^%d]", (long long)g->n, mf::kMinLog2N,
                    mf::kMaxLog2N);
    if (!(g->fs > 0.0) || !isfinite(g->fs)) return fail(MF_E_ARG, "fs=%g must be positive and finite", g->fs);
    if (!(g->f0 > 0.0) || !isfinite(g->f0)) return fail(MF_E_ARG, "f0=%g must be positive and finite", g->f0);
    if (!(g->f_low > 0.0) || !(g->f_low < 0.5 * g->fs))
        return fail(MF_E_BAND, "f_low=%g must lie in (0, fs/2=%g)", g->f_low, 0.5 * g->fs);
    const double T = (double)g->n / g->fs;
    const double kl = ceil(g->f_low * T);
    if (kl < 1.0 || kl > (double)(g->n / 2 - 1))
        return fail(MF_E_BAND, "f_low=%g gives first bin %g outside [1, N/2-1]", g->f_low, kl);
    *log2n = l;
    *k_lo = (int)kl;
    return MF_OK;
}

// Upper band edge: min(floor(f_ISCO T), N/2 - 1), f_ISCO = 1/(6^{3/2} pi M).
int64_t band_hi(const mf_grid* g, double mc, double eta) {
    const double m_total = mc * pow(eta, -0.6);
    const double M = m_total * mf::kTsun;
    const double fisco = 1.0 / (sqrt(216.0) * M_PI * M);
    const double T = (double)g->n / g->fs;
    const double kh = floor(fisco * T);
    const double cap = (double)(g->n / 2 - 1);
    return (int64_t)(kh < cap ? kh : cap);
}

// FP64 coefficients of the stationary-phase phase in cycles, as a power
// series in u = k^{-1/3}:  Psi/2pi = b1 u + b2 u^2 + b3 u^3 + b5 u^5 - 1/8.
// With v = (pi M f)^{1/3} and f = k df, 3/(128 eta v^5) v^n = C (pi M df)^{(n-5)/3} u^{5-n}.
void spa_coefficients(double mc, double eta, double df, mf_bank_entry* e) {
    const double M = mc * pow(eta, -0.6) * mf::kTsun;
    const double x = M_PI * M * df;
    const double C = 3.0 / (128.0 * eta);
    const double inv2pi = 0.5 / M_PI;
    const double p2 = 3715.0 / 756.0 + 55.0 * eta / 9.0;
    const double p3 = -16.0 * M_PI;
    const double p4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta * eta / 72.0;
    e->b5 = C * pow(x, -5.0 / 3.0) * inv2pi;
    e->b3 = C * p2 / x * inv2pi;
    e->b2 = C * p3 * pow(x, -2.0 / 3.0) * inv2pi;
    e->b1 = C * p4 * pow(x, -1.0 / 3.0) * inv2pi;
    e->c0 = -0.125;
}

}  // namespace

namespace mf {

// Plans installed by mf_set_plan (the tuner), keyed by (log2 N, FP64 or not).
std::mutex g_plan_mu;
std::map<std::pair<int, bool>, Plan> g_plans;

Plan select_plan(int log2n, mf_precision prec) {
    Plan p = default_plan(log2n, prec);
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find({log2n, prec == MF_FP64});
        if (it != g_plans.end()) p = it->second;
    }
    return p;
}

// Band-mode plans installed by mf_set_band_plan, keyed like g_plans.
std::map<std::pair<int, bool>, Plan> g_band_plans;

Plan band_plan(int log2n, mf_precision prec) {
    Plan p = default_band_plan(log2n, prec);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_band_plans.find({log2n, prec == MF_FP64});
    if (it != g_band_plans.end()) p = it->second;
    return p;
}

}  // namespace mf

extern "C" {

const char* mf_last_error(void) { return g_err.c_str(); }

const char* mf_version(void) { return "libmf 0.1.0 gfx950"; }

size_t mf_bank_bytes(int64_t n_tmpl) { return n_tmpl > 0 ? (size_t)n_tmpl * sizeof(mf_bank_entry) : 0; }

size_t mf_filter_workspace_bytes(const mf_grid* grid, mf_precision prec, int64_t n_tmpl, int64_t n_seg) {
    int l, klo;
    if (check_grid(grid, &l, &klo) != MF_OK) return 0;
    if (!valid_prec(prec) || n_tmpl < 1 || n_seg < 1) {
        fail(MF_E_ARG, "bad precision or counts");
        return 0;
    }
    const mf::Plan p = mf::select_plan(l, prec);
    return mf::filter_layout(p, prec, grid->n, n_tmpl, n_seg).total;
}

mf_status mf_filter_plan(const mf_grid* grid, mf_precision prec, int32_t plan[8]) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!valid_prec(prec) || !plan) return fail(MF_E_ARG, "bad precision or null plan");
    const mf::Plan p = mf::select_plan(l, prec);
    const int32_t v[8] = {p.n1, p.n2, p.c1, p.b2, p.nt1, p.nt2, p.units, mf::plan_flags(p)};
    for (int i = 0; i < 8; ++i) plan[i] = v[i];
    return ok();
}

int32_t mf_plan_candidates(const mf_grid* grid, mf_precision prec, int32_t* plans, int32_t cap) {
    int l, klo;
    if (check_grid(grid, &l, &klo) != MF_OK) return -1;
    if (!valid_prec(prec) || cap < 0 || (cap > 0 && !plans)) {
        fail(MF_E_ARG, "bad precision or output buffer");
        return -1;
    }
    std::vector<mf::Plan> v((size_t)(cap > 0 ? cap : 0));
    const int n = mf::plan_candidates(l, prec, v.data(), cap);
    for (int i = 0; i < n && i < cap; ++i) {
        const mf::Plan& p = v[(size_t)i];
        const int32_t row[8] = {p.n1, p.n2, p.c1, p.b2, p.nt1, p.nt2, 0, mf::plan_flags(p)};
        for (int k = 0; k < 8; ++k) plans[8 * i + k] = row[k];
    }
    ok();
    return n;
}

mf_status mf_set_plan(const mf_grid* grid, mf_precision prec, const int32_t plan[8]) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    std::lock_guard<std::mutex> lk(mf::g_plan_mu);
    if (!plan) {
        mf::g_plans.erase({l, prec == MF_FP64});
        return ok();
    }
    mf::Plan q = mf::default_plan(l, prec);
    q.n1 = plan[0];
    q.n2 = plan[1];
    q.c1 = plan[2];
    q.b2 = plan[3];
    auto clampt = [](long long x) { return (int)(x < 64 ? 64 : (x > 1024 ? 1024 : x)); };
    q.nt1 = clampt((long long)q.c1 * q.n1 / 16);
    // pass-2 threads select the largest stage radix: B N2 / 16 (default) or B N2 / 8
    const int nt16 = clampt((long long)q.b2 * q.n2 / 16), nt8 = clampt((long long)q.b2 * q.n2 / 8);
    q.nt2 = plan[5] == nt8 ? nt8 : nt16;
    q.units = plan[6];
    if ((plan[7] & ~63) || (plan[7] & 6) == 4)
        return fail(MF_E_ARG,
                    "plan flags %d: bits 0 (pipelined step), 1 (split exchange), 2 (conflict-free layouts, with bit 1), "
                    "3 (narrow-band pass 1), 4 (pass 1 applies the first row factor), 5 (persistent pass 1)",
                    plan[7]);
    q.fused = (plan[7] & 1) != 0;
    q.xs = (plan[7] & 4) ? 2 : ((plan[7] & 2) ? 1 : 0);
    q.prune1 = (plan[7] & 8) != 0;
    q.pre0 = (plan[7] & 16) != 0;
    q.persist = (plan[7] & 32) != 0;
    if ((int64_t)q.n1 * q.n2 != grid->n || !mf::plan_supported(q, prec))
        return fail(MF_E_UNSUPPORTED,
                    "plan %dx%d c=%d b=%d (pass-2 threads %d, flags %d) is not built for this N/precision", q.n1, q.n2,
                    q.c1, q.b2, q.nt2, plan[7]);
    if (q.units < 1 || q.units > 4096) return fail(MF_E_ARG, "units per batch %d outside [1, 4096]", q.units);
    if (q.pre0 && q.fused)
        return fail(MF_E_UNSUPPORTED, "flag bit 4 (pass 1 applies the first row factor) is not built for the pipelined step");
    if (q.persist && q.fused)
        return fail(MF_E_UNSUPPORTED, "flag bit 5 (persistent pass 1) is not built for the pipelined step");
    if (q.pre0 && !mf::pre0_fits(q))
        return fail(MF_E_UNSUPPORTED, "flag bit 4 needs the pass-1 columns (%d) to divide N2/R0 = %d", q.c1,
                    q.n2 / mf::plan_r2(q));
    if (q.fused && (q.nt1 != q.nt2 || q.nt2 != nt16))
        return fail(MF_E_UNSUPPORTED, "pipelined step needs equal work-group sizes and radix-16 row stages");
    mf::g_plans[{l, prec == MF_FP64}] = q;
    return ok();
}

mf_status mf_set_band_plan(const mf_grid* grid, mf_precision prec, const int32_t plan[8]) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    std::lock_guard<std::mutex> lk(mf::g_plan_mu);
    if (!plan) {
        mf::g_band_plans.erase({l, prec == MF_FP64});
        return ok();
    }
    mf::Plan q = mf::default_band_plan(l, prec);
    if (q.log2n != l) return fail(MF_E_UNSUPPORTED, "no band-mode plan for n=%lld", (long long)grid->n);
    q.n1 = plan[0];
    q.n2 = plan[1];
    q.c1 = plan[2];
    q.b2 = plan[3];
    q.nt1 = plan[4];
    q.nt2 = plan[5];
    q.units = plan[6];
    if (plan[7] != 0) return fail(MF_E_ARG, "band-mode plan flags %d: must be 0", plan[7]);
    if ((int64_t)q.n1 * q.n2 != grid->n || !mf::band_plan_supported(q, prec))
        return fail(MF_E_UNSUPPORTED, "band-mode plan %dx%d c=%d b=%d (threads %d/%d) is not built for this N/precision",
                    q.n1, q.n2, q.c1, q.b2, q.nt1, q.nt2);
    if (q.units < 1 || q.units > 4096) return fail(MF_E_ARG, "units per batch %d outside [1, 4096]", q.units);
    mf::g_band_plans[{l, prec == MF_FP64}] = q;
    return ok();
}

mf_status mf_psd(const mf_grid* grid, double* Sn_dev, double* prefix_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!Sn_dev) return fail(MF_E_ARG, "Sn_dev is null");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mf::launch_psd(grid->n, grid->fs, grid->f_low, grid->f0, klo, Sn_dev, s);
    if (e != hipSuccess) return hip_fail(e, "mf_psd");
    if (prefix_dev) {
        e = mf::launch_prefix(grid->n, grid->fs, Sn_dev, prefix_dev, s);
        if (e != hipSuccess) return hip_fail(e, "mf_psd prefix");
    }
    return ok();
}

mf_status mf_spa_bank(const mf_grid* grid, const double* mc_host, const double* eta_host, int64_t n_tmpl,
                      const double* Sn_dev, mf_precision prec, mf_sigma_mode sigma_mode, void* bank_dev,
                      int32_t* khi_host, double* sigma_host, void* htilde_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!mc_host || !eta_host || !Sn_dev || !bank_dev) return fail(MF_E_ARG, "null pointer argument");
    if (n_tmpl < 1 || n_tmpl > (int64_t(1) << 31) - 1) return fail(MF_E_ARG, "n_tmpl=%lld", (long long)n_tmpl);
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (sigma_mode != MF_SIGMA_FP64 && sigma_mode != MF_SIGMA_COMP32)
        return fail(MF_E_ARG, "bad sigma mode %d", (int)sigma_mode);
    if (htilde_dev && n_tmpl > 65535) return fail(MF_E_ARG, "materialised templates limited to 65535");
    const double df = grid->fs / (double)grid->n;
    std::vector<mf_bank_entry> h((size_t)n_tmpl);
    for (int64_t t = 0; t < n_tmpl; ++t) {
        const double mc = mc_host[t], eta = eta_host[t];
        if (!(mc > 0.0) || !isfinite(mc)) return fail(MF_E_ARG, "template %lld: chirp mass %g", (long long)t, mc);
        if (!(eta > 0.0) || !(eta <= 0.25)) return fail(MF_E_ARG, "template %lld: eta %g", (long long)t, eta);
        mf_bank_entry& e = h[(size_t)t];
        e = mf_bank_entry{};
        spa_coefficients(mc, eta, df, &e);
        e.k_lo = klo;
        const int64_t khi = band_hi(grid, mc, eta);
        if (khi < klo)
            return fail(MF_E_BAND, "template %lld: empty band (k_hi=%lld < k_lo=%d)", (long long)t, (long long)khi, klo);
        e.k_hi = (int32_t)khi;
        if (khi_host) khi_host[t] = (int32_t)khi;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(bank_dev, h.data(), h.size() * sizeof(mf_bank_entry), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "mf_spa_bank copy");
    e = mf::launch_sigma(grid->n, grid->fs, sigma_mode, Sn_dev, (mf_bank_entry*)bank_dev, n_tmpl, s);
    if (e != hipSuccess) return hip_fail(e, "mf_spa_bank sigma");
    if (htilde_dev) {
        e = mf::launch_spa_synth(grid->n, grid->fs, prec, (const mf_bank_entry*)bank_dev, n_tmpl, htilde_dev, s);
        if (e != hipSuccess) return hip_fail(e, "mf_spa_bank synth");
    }
    if (sigma_host) {
        e = hipMemcpyAsync(h.data(), bank_dev, h.size() * sizeof(mf_bank_entry), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "mf_spa_bank sigma copy");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "mf_spa_bank sync");
    if (sigma_host)
        for (int64_t t = 0; t < n_tmpl; ++t) sigma_host[t] = h[(size_t)t].sigma;
    return ok();
}

}  // extern "C"

namespace {

// Body of mf_filter; ev_keys (nullable, zeroed by the caller) turns on the
// per-window event keys of pass 2; plan_in (nullable) replaces the selected
// launch plan.
mf_status filter_impl(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev,
                      int64_t n_seg, const double* Sn_dev, mf_precision prec, const mf_filter_opts* opts,
                      void* workspace_dev, size_t workspace_bytes, mf_peak* peaks_dev, void* rho_dev,
                      mf_stream_t stream, unsigned long long* ev_keys, int ev_log2w,
                      const mf::Plan* plan_in = nullptr) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!bank_dev || !stilde_dev || !Sn_dev || !peaks_dev || !workspace_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (n_tmpl < 1 || n_seg < 1) return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld", (long long)n_tmpl, (long long)n_seg);
    if (n_tmpl * n_seg > (int64_t(1) << 40)) return fail(MF_E_ARG, "too many units");
    const int64_t n = grid->n;
    mf_filter_opts o{INFINITY, 0, 0, nullptr, 0};
    if (opts) o = *opts;
    if (o.j_end == 0) o.j_end = n;
    if (o.j_begin < 0 || o.j_end > n || o.j_begin >= o.j_end)
        return fail(MF_E_SHAPE, "window [%lld, %lld) outside [0, %lld)", (long long)o.j_begin, (long long)o.j_end,
                    (long long)n);
    if (o.rho_threshold != o.rho_threshold) return fail(MF_E_ARG, "rho_threshold is NaN");
    if (o.n_series < 0) return fail(MF_E_ARG, "n_series < 0");
    if (o.n_series > 0 && (!o.series_units_dev || !rho_dev))
        return fail(MF_E_ARG, "series requested without series_units_dev / rho_dev");
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(MF_E_ARG, "workspace must be 256-byte aligned");
    const mf::Plan p = plan_in ? *plan_in : mf::select_plan(l, prec);
    if (p.log2n != l || (int64_t)p.n1 * p.n2 != n || p.n2 % p.c1 != 0 || p.n1 % p.b2 != 0 ||
        !mf::plan_supported(p, prec))
        return fail(MF_E_UNSUPPORTED, "no plan for n=%lld", (long long)n);
    const mf::FilterLayout L = mf::filter_layout(p, prec, n, n_tmpl, n_seg);
    if (L.units_per_batch * (int64_t)(p.n2 / p.c1 + p.n1 / p.b2) > (int64_t)0x7fffffff)
        return fail(MF_E_UNSUPPORTED, "batch too large for one launch");
    if (workspace_bytes < L.total)
        return fail(MF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, L.total);

    char* ws = (char*)workspace_dev;
    mf::FilterArgs a{};
    a.wgt = ws + L.off_w;
    a.bank = (const mf_bank_entry*)bank_dev;
    a.inter = ws + L.off_inter;
    a.keys = prec == MF_FP64 ? nullptr : (unsigned long long*)(ws + L.off_keys);
    a.counts = prec == MF_FP64 ? nullptr : (unsigned int*)(ws + L.off_counts);
    a.partials = prec == MF_FP64 ? (void*)(ws + L.off_part) : nullptr;
    a.n_tmpl = n_tmpl;
    a.n_seg = n_seg;
    a.n_units = n_tmpl * n_seg;
    a.j_begin = o.j_begin;
    a.j_end = o.j_end;
    a.rho_threshold = o.rho_threshold;
    a.series_units = o.series_units_dev;
    a.n_series = o.n_series;
    a.rho = rho_dev;
    a.ev_keys = ev_keys;
    a.ev_log2w = ev_log2w;
    a.tw2 = ws + L.off_tw2;
    a.prune1 = p.prune1 ? 1 : 0;
    a.pre0_r0 = p.pre0 && !p.fused && mf::pre0_fits(p) ? mf::plan_r2(p) : 0;
    const bool persist = p.persist && !p.fused;
    if (persist) {
        a.lpt_order = (const int32_t*)(ws + L.off_lpt);
        a.lpt_ctr = (unsigned int*)(ws + L.off_lpt_ctr);
    }

    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mf::launch_weights(n, grid->fs, klo, prec, stilde_dev, n_seg, Sn_dev, (void*)a.wgt, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter weights");
    if (mf::pass2_uses_tw2(prec, p.n2, p.b2, p.nt2)) {
        e = mf::launch_tw2_fill(prec, ws + L.off_tw2, s);
        if (e != hipSuccess) return hip_fail(e, "mf_filter stage table");
    }
    const int64_t upb = L.units_per_batch;
    const int64_t nb = (a.n_units + upb - 1) / upb;
    auto batch = [&](mf::FilterArgs& x, int64_t b, int buf) {
        x.inter = ws + L.off_inter + (size_t)buf * L.inter_bytes;
        if (b < 0 || b >= nb) {
            x.unit0 = 0;
            x.units = 0;
        } else {
            x.unit0 = b * upb;
            x.units = (a.n_units - x.unit0) < upb ? (a.n_units - x.unit0) : upb;
        }
    };
    if (p.fused) {
        // step b: pass 1 of batch b into buffer b%2, pass 2 of batch b-1 from buffer (b-1)%2
        for (int64_t b = 0; b <= nb; ++b) {
            mf::FilterArgs a1 = a, a2 = a;
            batch(a1, b, (int)(b & 1));
            batch(a2, b - 1, (int)((b + 1) & 1));
            st = timed_launch(s, a1.units, a2.units, [&] { return mf::launch_step(p, prec, a1, a2, s); });
            if (st != MF_OK) return st;
        }
    } else {
        for (int64_t b = 0; b < nb; ++b) {
            mf::FilterArgs a1 = a, none = a;
            batch(a1, b, 0);
            batch(none, -1, 0);
            st = timed_launch(s, a1.units, none.units, [&] {
                return persist ? mf::launch_pass1_lpt(p, prec, a1, s) : mf::launch_pass1(p, prec, false, a1, s);
            });
            if (st != MF_OK) return st;
            st = timed_launch(s, none.units, a1.units, [&] { return mf::launch_pass2(p, prec, false, a1, s); });
            if (st != MF_OK) return st;
        }
    }
    e = mf::launch_finalize(p, prec, a, peaks_dev, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter finalize");
    return ok();
}

size_t events_scratch_bytes(int64_t n, int64_t n_tmpl, int64_t n_seg, int log2w) {
    const int64_t n_win = n >> log2w;
    const size_t keys = (size_t)(n_tmpl * n_seg * n_win) * 8;
    const size_t unit_ev = (size_t)(n_tmpl * n_seg * n_win) * sizeof(mf_event);
    const size_t best = (size_t)(n_seg * n_win) * sizeof(mf_event);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(keys) + al(unit_ev) + al(best);
}

// Scratch of mf_filter_noalloc: a file-scope device array, one copy per GPU
// the library runs on, resident until the process ends.  Host code never
// passes its name to a kernel: it uses the address hipGetSymbolAddress
// returns for the current device (kept per device below).
static __device__ __align__(256) unsigned char scratch[MF_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of that device's copy

// Address of the current device's scratch; the first call on a device looks
// it up (with that device current) and keeps it.
mf_status scratch_address(mf_stream_t stream, void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_noalloc device");
    if (stream) {
        int sdev = -1;
        e = hipStreamGetDevice((hipStream_t)stream, &sdev);
        if (e != hipSuccess) return hip_fail(e, "mf_filter_noalloc stream device");
        if (sdev != dev) return fail(MF_E_ARG, "stream belongs to device %d, current device is %d", sdev, dev);
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "mf_filter_noalloc scratch address");
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(MF_E_HIP, "mf_filter_noalloc: unaligned scratch");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return MF_OK;
}

mf::Plan with_units(mf::Plan p, int64_t units) {
    p.units = (int)units;
    return p;
}

// The largest units-per-batch, at most the plan's, whose workspace fits the
// static scratch; false if not even one unit per batch fits.
bool scratch_units(const mf::Plan& p, mf_precision prec, int64_t n, int64_t n_tmpl, int64_t n_seg, int64_t* units) {
    const size_t cap = (size_t)MF_NOALLOC_SCRATCH_BYTES;
    if (mf::filter_layout(with_units(p, 1), prec, n, n_tmpl, n_seg).total > cap) return false;
    int64_t lo = 1, hi = p.units;  // invariant: lo fits
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (mf::filter_layout(with_units(p, mid), prec, n, n_tmpl, n_seg).total <= cap) lo = mid;
        else hi = mid - 1;
    }
    *units = lo;
    return true;
}

}  // namespace

extern "C" {

mf_status mf_filter(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev, int64_t n_seg,
                    const double* Sn_dev, mf_precision prec, const mf_filter_opts* opts, void* workspace_dev,
                    size_t workspace_bytes, mf_peak* peaks_dev, void* rho_dev, mf_stream_t stream) {
    return filter_impl(grid, bank_dev, n_tmpl, stilde_dev, n_seg, Sn_dev, prec, opts, workspace_dev, workspace_bytes,
                       peaks_dev, rho_dev, stream, nullptr, 0);
}

size_t mf_filter_events_workspace_bytes(const mf_grid* grid, mf_precision prec, int64_t n_tmpl, int64_t n_seg,
                                        int32_t log2_window) {
    int l, klo;
    if (check_grid(grid, &l, &klo) != MF_OK || !valid_prec(prec) || n_tmpl < 1 || n_seg < 1 || log2_window < 4 ||
        log2_window > 16 || log2_window > l)
        return 0;
    const size_t base = mf_filter_workspace_bytes(grid, prec, n_tmpl, n_seg);
    if (base == 0) return 0;
    return ((base + 255) & ~(size_t)255) + events_scratch_bytes(grid->n, n_tmpl, n_seg, log2_window);
}

mf_status mf_filter_events(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev,
                           int64_t n_seg, const double* Sn_dev, mf_precision prec, double rho_threshold,
                           int32_t log2_window, void* workspace_dev, size_t workspace_bytes, mf_peak* peaks_dev,
                           mf_event* unit_events_dev, mf_event* seg_events_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!seg_events_dev || !workspace_dev || !peaks_dev || !bank_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (!(rho_threshold > 0.0) || !isfinite(rho_threshold))
        return fail(MF_E_ARG, "rho_threshold must be positive and finite");
    if (log2_window < 4 || log2_window > 16 || log2_window > l)
        return fail(MF_E_ARG, "log2_window=%d outside [4, min(16, log2 N)]", (int)log2_window);
    if (n_tmpl < 1 || n_seg < 1 || n_tmpl * n_seg > (int64_t(1) << 31) - 1)
        return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld", (long long)n_tmpl, (long long)n_seg);
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(MF_E_ARG, "workspace must be 256-byte aligned");
    const size_t need = mf_filter_events_workspace_bytes(grid, prec, n_tmpl, n_seg, log2_window);
    if (workspace_bytes < need) return fail(MF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, need);
    const size_t base = (mf_filter_workspace_bytes(grid, prec, n_tmpl, n_seg) + 255) & ~(size_t)255;
    const int64_t n_win = grid->n >> log2_window;
    char* ev = (char*)workspace_dev + base;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    unsigned long long* keys = (unsigned long long*)ev;
    mf_event* unit_ev = (mf_event*)(ev + al((size_t)(n_tmpl * n_seg * n_win) * 8));
    mf_event* best = (mf_event*)((char*)unit_ev + al((size_t)(n_tmpl * n_seg * n_win) * sizeof(mf_event)));
    if (unit_events_dev) unit_ev = unit_events_dev;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mf::launch_fill_u64(keys, n_tmpl * n_seg * n_win, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_events clear");
    mf_filter_opts o{rho_threshold, 0, 0, nullptr, 0};
    st = filter_impl(grid, bank_dev, n_tmpl, stilde_dev, n_seg, Sn_dev, prec, &o, workspace_dev, base, peaks_dev,
                     nullptr, stream, keys, log2_window);
    if (st != MF_OK) return st;
    e = mf::launch_events(keys, n_tmpl, n_seg, n_win, log2_window, prec == MF_FP64, (const mf_bank_entry*)bank_dev,
                          unit_ev, best, seg_events_dev, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_events clustering");
    return ok();
}

mf_status mf_filter_noalloc(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev,
                            int64_t n_seg, const double* Sn_dev, mf_precision prec, const mf_filter_opts* opts,
                            mf_peak* peaks_dev, void* rho_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!bank_dev || !stilde_dev || !Sn_dev || !peaks_dev) return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (n_tmpl < 1 || n_seg < 1 || n_tmpl * n_seg > (int64_t(1) << 40))
        return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld", (long long)n_tmpl, (long long)n_seg);
    mf::Plan p = mf::select_plan(l, prec);
    int64_t units;
    if (!scratch_units(p, prec, grid->n, n_tmpl, n_seg, &units))
        return fail(MF_E_WORKSPACE,
                    "request needs %zu bytes of scratch at one unit per batch; the static scratch holds %zu "
                    "(MF_NOALLOC_SCRATCH_BYTES)",
                    mf::filter_layout(with_units(p, 1), prec, grid->n, n_tmpl, n_seg).total,
                    (size_t)MF_NOALLOC_SCRATCH_BYTES);
    p = with_units(p, units);
    void* ws = nullptr;
    st = scratch_address(stream, &ws);
    if (st != MF_OK) return st;
    return filter_impl(grid, bank_dev, n_tmpl, stilde_dev, n_seg, Sn_dev, prec, opts, ws,
                       (size_t)MF_NOALLOC_SCRATCH_BYTES, peaks_dev, rho_dev, stream, nullptr, 0, &p);
}

size_t mf_ifft_workspace_bytes(int64_t n, mf_precision prec, int64_t batch) {
    const int l = log2_exact(n);
    if (l < mf::kMinLog2N || l > mf::kMaxLog2N || !valid_prec(prec) || batch < 1) {
        fail(MF_E_ARG, "bad n/precision/batch");
        return 0;
    }
    const mf::Plan p = mf::select_plan(l, prec);
    const int64_t u = batch < p.units ? batch : p.units;
    return (size_t)u * (size_t)n * mf::cx_bytes(prec);
}

mf_status mf_ifft(int64_t n, mf_precision prec, const void* q_dev, void* z_dev, int64_t batch, void* workspace_dev,
                  size_t workspace_bytes, mf_stream_t stream) {
    const int l = log2_exact(n);
    if (l < mf::kMinLog2N || l > mf::kMaxLog2N)
        return fail(MF_E_SHAPE, "n=%lld must be a power of two in [2^%d, 2^%d]", (long long)n, mf::kMinLog2N,
                    mf::kMaxLog2N);
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (!q_dev || !z_dev || !workspace_dev) return fail(MF_E_ARG, "null pointer argument");
    if (batch < 1) return fail(MF_E_ARG, "batch=%lld", (long long)batch);
    const size_t need = mf_ifft_workspace_bytes(n, prec, batch);
    if (workspace_bytes < need) return fail(MF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, need);
    const mf::Plan p = mf::select_plan(l, prec);
    const int64_t upb = batch < p.units ? batch : p.units;
    mf::FilterArgs a{};
    a.inter = workspace_dev;
    a.raw_in = q_dev;
    a.raw_out = z_dev;
    a.n_tmpl = 1;
    a.n_seg = batch;
    a.n_units = batch;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t u0 = 0; u0 < batch; u0 += upb) {
        a.unit0 = u0;
        a.units = (batch - u0) < upb ? (batch - u0) : upb;
        hipError_t e = mf::launch_pass1(p, prec, true, a, s);
        if (e != hipSuccess) return hip_fail(e, "mf_ifft pass1");
        e = mf::launch_pass2(p, prec, true, a, s);
        if (e != hipSuccess) return hip_fail(e, "mf_ifft pass2");
    }
    return ok();
}

size_t mf_rfft_workspace_bytes(int64_t n, mf_precision prec, int64_t batch) {
    const int l = log2_exact(n);
    if (l < mf::kMinLog2N + 1 || l > mf::kMaxLog2N + 1 || !valid_prec(prec) || batch < 1) {
        fail(MF_E_ARG, "bad n/precision/batch");
        return 0;
    }
    const size_t half = (size_t)batch * (size_t)(n / 2) * mf::cx_bytes(prec);
    const size_t inter = mf_ifft_workspace_bytes(n / 2, prec, batch);
    return 2 * ((half + 255) & ~(size_t)255) + inter;
}

mf_status mf_rfft(int64_t n, double fs, mf_precision prec, const void* x_dev, void* stilde_dev, int64_t batch,
                  void* workspace_dev, size_t workspace_bytes, mf_stream_t stream) {
    const int l = log2_exact(n);
    if (l < mf::kMinLog2N + 1 || l > mf::kMaxLog2N + 1)
        return fail(MF_E_SHAPE, "n=%lld must be a power of two in [2^%d, 2^%d]", (long long)n, mf::kMinLog2N + 1,
                    mf::kMaxLog2N + 1);
    if (!(fs > 0.0) || !isfinite(fs)) return fail(MF_E_ARG, "fs must be positive and finite");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (!x_dev || !stilde_dev || !workspace_dev) return fail(MF_E_ARG, "null pointer argument");
    if (batch < 1) return fail(MF_E_ARG, "batch=%lld", (long long)batch);
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(MF_E_ARG, "workspace must be 256-byte aligned");
    const size_t need = mf_rfft_workspace_bytes(n, prec, batch);
    if (workspace_bytes < need) return fail(MF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, need);
    const int64_t m = n / 2;
    const size_t half = (((size_t)batch * (size_t)m * mf::cx_bytes(prec)) + 255) & ~(size_t)255;
    char* ws = (char*)workspace_dev;
    void* y = ws;
    void* z = ws + half;
    void* inter = ws + 2 * half;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mf::launch_rfft_pack(prec, x_dev, y, m, batch, s);
    if (e != hipSuccess) return hip_fail(e, "mf_rfft pack");
    mf_status st = mf_ifft(m, prec, y, z, batch, inter, workspace_bytes - 2 * half, stream);
    if (st != MF_OK) return st;
    e = mf::launch_rfft_post(prec, z, stilde_dev, m, batch, 1.0 / fs, s);
    if (e != hipSuccess) return hip_fail(e, "mf_rfft post");
    return ok();
}

mf_status mf_psd_prefix(const mf_grid* grid, const double* Sn_dev, double* prefix_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!Sn_dev || !prefix_dev) return fail(MF_E_ARG, "null pointer argument");
    hipError_t e = mf::launch_prefix(grid->n, grid->fs, Sn_dev, prefix_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_psd_prefix");
    return ok();
}

mf_status mf_snr_grad(const mf_grid* grid, const double* theta_dev, const int32_t* khi_dev, const int32_t* seg_dev,
                      int64_t n, const void* stilde_dev, int64_t n_seg, const double* Sn_dev, mf_precision prec,
                      double* Z_dev, double* rho2_dev, const double* gbar_dev, double* grad_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!theta_dev || !seg_dev || !stilde_dev || !Sn_dev || !Z_dev || !rho2_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (gbar_dev && !grad_dev) return fail(MF_E_ARG, "gbar_dev given without grad_dev");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (n < 1 || n > (int64_t(1) << 31) - 1 || n_seg < 1) return fail(MF_E_ARG, "n=%lld n_seg=%lld", (long long)n,
                                                                       (long long)n_seg);
    hipError_t e = mf::launch_snr_grad(grid->n, grid->fs, klo, prec, theta_dev, khi_dev, seg_dev, n, stilde_dev, n_seg, Sn_dev,
                                       Z_dev, rho2_dev, gbar_dev, grad_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_snr_grad");
    return ok();
}

size_t mf_filter_chisq_workspace_bytes(const mf_grid* grid, mf_precision prec, int64_t n_tmpl, int64_t n_seg,
                                       int32_t p_bands) {
    int l, klo;
    if (check_grid(grid, &l, &klo) != MF_OK || !valid_prec(prec) || n_tmpl < 1 || n_seg < 1 || p_bands < 2 ||
        p_bands > 64)
        return 0;
    const mf::Plan p = mf::band_plan(l, prec);
    if (p.log2n != l) return 0;
    return mf::band_layout(p, prec, grid->n, n_tmpl, n_seg, p_bands).total;
}

mf_status mf_filter_chisq_plan(const mf_grid* grid, mf_precision prec, int32_t plan[8]) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!valid_prec(prec) || !plan) return fail(MF_E_ARG, "bad precision or null plan");
    const mf::Plan p = mf::band_plan(l, prec);
    if (p.log2n != l) return fail(MF_E_UNSUPPORTED, "no band-mode plan for n=%lld", (long long)grid->n);
    const int32_t v[8] = {p.n1, p.n2, p.c1, p.b2, p.nt1, p.nt2, p.units, 0};
    for (int i = 0; i < 8; ++i) plan[i] = v[i];
    return ok();
}

mf_status mf_filter_chisq(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev,
                          int64_t n_seg, const double* Sn_dev, const double* prefix_dev, mf_precision prec,
                          int32_t p_bands, const mf_filter_opts* opts, void* workspace_dev, size_t workspace_bytes,
                          mf_peak* peaks_dev, double* chisq_dev, void* rho_dev, void* chisq_series_dev,
                          mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!bank_dev || !stilde_dev || !Sn_dev || !prefix_dev || !peaks_dev || !chisq_dev || !workspace_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (p_bands < 2 || p_bands > 64) return fail(MF_E_ARG, "p_bands=%d outside [2, 64]", (int)p_bands);
    if (n_tmpl < 1 || n_seg < 1 || n_tmpl * n_seg > (int64_t(1) << 31) - 1)
        return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld", (long long)n_tmpl, (long long)n_seg);
    const int64_t n = grid->n;
    mf_filter_opts o{INFINITY, 0, 0, nullptr, 0};
    if (opts) o = *opts;
    if (o.j_end == 0) o.j_end = n;
    if (o.j_begin < 0 || o.j_end > n || o.j_begin >= o.j_end)
        return fail(MF_E_SHAPE, "window [%lld, %lld) outside [0, %lld)", (long long)o.j_begin, (long long)o.j_end,
                    (long long)n);
    if (o.rho_threshold != o.rho_threshold) return fail(MF_E_ARG, "rho_threshold is NaN");
    if (o.n_series < 0) return fail(MF_E_ARG, "n_series < 0");
    if (o.n_series > 0 && (!o.series_units_dev || !rho_dev || !chisq_series_dev))
        return fail(MF_E_ARG, "series requested without series_units_dev / rho_dev / chisq_series_dev");
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(MF_E_ARG, "workspace must be 256-byte aligned");
    const mf::Plan p = mf::band_plan(l, prec);
    if (p.log2n != l) return fail(MF_E_UNSUPPORTED, "no band-mode plan for n=%lld", (long long)n);
    const mf::BandLayout L = mf::band_layout(p, prec, n, n_tmpl, n_seg, p_bands);
    if (L.units_per_batch * (int64_t)(p.n2 / p.c1 + p.n1 / p.b2) > (int64_t)0x7fffffff)
        return fail(MF_E_UNSUPPORTED, "batch too large for one launch");
    if (workspace_bytes < L.total)
        return fail(MF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, L.total);

    char* ws = (char*)workspace_dev;
    mf::FilterArgs a{};
    a.wgt = ws + L.off_w;
    a.bank = (const mf_bank_entry*)bank_dev;
    a.inter = ws + L.off_inter;
    a.partials = ws + L.off_part;
    a.n_tmpl = n_tmpl;
    a.n_seg = n_seg;
    a.n_units = n_tmpl * n_seg;
    a.j_begin = o.j_begin;
    a.j_end = o.j_end;
    a.rho_threshold = o.rho_threshold;
    a.series_units = o.series_units_dev;
    a.n_series = o.n_series;
    a.rho = rho_dev;
    a.band_tab = (const int32_t*)(ws + L.off_tab);
    a.p_bands = p_bands;
    a.qbuf = ws + L.off_q;
    a.chi_series = chisq_series_dev;

    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mf::launch_weights(n, grid->fs, klo, prec, stilde_dev, n_seg, Sn_dev, (void*)a.wgt, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_chisq weights");
    e = mf::launch_band_table(n, p.n2, a.bank, n_tmpl, prefix_dev, p_bands, (int32_t*)(ws + L.off_tab), s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_chisq band table");
    const int64_t upb = L.units_per_batch;
    for (int64_t u0 = 0; u0 < a.n_units; u0 += upb) {
        mf::FilterArgs x = a;
        x.unit0 = u0;
        x.units = (a.n_units - u0) < upb ? (a.n_units - u0) : upb;
        st = timed_launch(s, x.units, 0, [&] { return mf::launch_pass1_band(p, prec, x, s); });
        if (st != MF_OK) return st;
        st = timed_launch(s, 0, x.units, [&] { return mf::launch_pass2_band(p, prec, x, s); });
        if (st != MF_OK) return st;
    }
    e = mf::launch_finalize_band(p, a, peaks_dev, chisq_dev, s);
    if (e != hipSuccess) return hip_fail(e, "mf_filter_chisq finalize");
    return ok();
}

mf_status mf_chisq(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev, int64_t n_seg,
                   const double* Sn_dev, const double* prefix_dev, mf_precision prec, int32_t p_bands,
                   const mf_peak* peaks_dev, double* chisq_dev, double* rho_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!bank_dev || !stilde_dev || !Sn_dev || !prefix_dev || !peaks_dev || !chisq_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (p_bands < 2 || p_bands > 64) return fail(MF_E_ARG, "p_bands=%d outside [2, 64]", (int)p_bands);
    if (n_tmpl < 1 || n_seg < 1 || n_tmpl * n_seg > (int64_t(1) << 31) - 1)
        return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld", (long long)n_tmpl, (long long)n_seg);
    hipError_t e = mf::launch_chisq(grid->n, grid->fs, prec, (const mf_bank_entry*)bank_dev, n_tmpl, stilde_dev, n_seg,
                                    Sn_dev, prefix_dev, p_bands, peaks_dev, nullptr, 0, chisq_dev, rho_dev,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_chisq");
    return ok();
}

mf_status mf_chisq_events(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev,
                          int64_t n_seg, const double* Sn_dev, const double* prefix_dev, mf_precision prec,
                          int32_t p_bands, const mf_event* events_dev, int64_t n_per_seg, double* chisq_dev,
                          double* rho_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!bank_dev || !stilde_dev || !Sn_dev || !prefix_dev || !events_dev || !chisq_dev)
        return fail(MF_E_ARG, "null pointer argument");
    if (!valid_prec(prec)) return fail(MF_E_ARG, "bad precision %d", (int)prec);
    if (p_bands < 2 || p_bands > 64) return fail(MF_E_ARG, "p_bands=%d outside [2, 64]", (int)p_bands);
    if (n_tmpl < 1 || n_seg < 1 || n_per_seg < 1 || n_seg * n_per_seg > (int64_t(1) << 31) - 1)
        return fail(MF_E_ARG, "n_tmpl=%lld n_seg=%lld n_per_seg=%lld", (long long)n_tmpl, (long long)n_seg,
                    (long long)n_per_seg);
    hipError_t e = mf::launch_chisq(grid->n, grid->fs, prec, (const mf_bank_entry*)bank_dev, n_tmpl, stilde_dev, n_seg,
                                    Sn_dev, prefix_dev, p_bands, nullptr, events_dev, n_per_seg, chisq_dev, rho_dev,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_chisq_events");
    return ok();
}

mf_status mf_template_metric(const mf_grid* grid, const double* theta_dev, const int32_t* khi_dev, int64_t n,
                             const double* Sn_dev, double* metric_dev, mf_stream_t stream) {
    int l, klo;
    mf_status st = check_grid(grid, &l, &klo);
    if (st != MF_OK) return st;
    if (!theta_dev || !khi_dev || !Sn_dev || !metric_dev) return fail(MF_E_ARG, "null pointer argument");
    if (n < 1 || n > (int64_t(1) << 31) - 1) return fail(MF_E_ARG, "n=%lld", (long long)n);
    hipError_t e = mf::launch_metric(grid->n, grid->fs, klo, theta_dev, khi_dev, n, Sn_dev, metric_dev,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_template_metric");
    return ok();
}

mf_status mf_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, mf_stream_t stream) {
    if (!src_dev || !dst_dev) return fail(MF_E_ARG, "null pointer argument");
    if (bytes == 0 || (bytes & 15) != 0 || ((uintptr_t)src_dev & 15) != 0 || ((uintptr_t)dst_dev & 15) != 0)
        return fail(MF_E_ARG, "bytes and pointers must be non-zero multiples of 16");
    hipError_t e = mf::launch_copy_probe(src_dev, dst_dev, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mf_probe_copy");
    return ok();
}

mf_status mf_timing_enable(int32_t stride) {
    if (stride < 0) return fail(MF_E_ARG, "stride < 0");
    g_timing.stride = stride;
    g_timing.batch_counter = 0;
    return ok();
}

mf_status mf_timing_read_split(double ms[3], int64_t launches[3], int64_t pass1_units[3], int64_t pass2_units[3]) {
    if (!ms || !launches || !pass1_units || !pass2_units) return fail(MF_E_ARG, "null pointer argument");
    for (int c = 0; c < 3; ++c) {
        ms[c] = 0.0;
        launches[c] = pass1_units[c] = pass2_units[c] = 0;
    }
    mf_status st = MF_OK;
    for (const TimedLaunch& t : g_timing.pending) {
        hipError_t e = hipEventSynchronize(t.stop);
        float el = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&el, t.start, t.stop);
        if (e != hipSuccess && st == MF_OK) st = hip_fail(e, "mf_timing_read");
        const int c = t.units2 == 0 ? 0 : (t.units1 == 0 ? 1 : 2);
        ms[c] += el;
        launches[c] += 1;
        pass1_units[c] += t.units1;
        pass2_units[c] += t.units2;
        g_timing.pool.push_back(t.start);
        g_timing.pool.push_back(t.stop);
    }
    g_timing.pending.clear();
    return st == MF_OK ? ok() : st;
}

mf_status mf_timing_read(double* ms, int64_t* launches, int64_t* pass1_units, int64_t* pass2_units) {
    if (!ms || !launches || !pass1_units || !pass2_units) return fail(MF_E_ARG, "null pointer argument");
    double m[3];
    int64_t n[3], u1[3], u2[3];
    mf_status st = mf_timing_read_split(m, n, u1, u2);
    *ms = m[0] + m[1] + m[2];
    *launches = n[0] + n[1] + n[2];
    *pass1_units = u1[0] + u1[1] + u1[2];
    *pass2_units = u2[0] + u2[1] + u2[2];
    return st;
}

}  // extern "C"
