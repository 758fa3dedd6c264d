// Host-side internals of libmf: launch plans, workspace layout, launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/mf.h"

namespace mf {

constexpr double kTsun = 4.925490947641267e-6;  // G M_sun / c^3 [s] (IAU 2015 nominal)
constexpr int kMinLog2N = 10;
constexpr int kMaxLog2N = 22;

// Two-pass decomposition N = n1 * n2 of the inverse DFT and the work-group
// shapes of the two passes.
struct Plan {
    int log2n;
    int n1, n2;      // column length (pass 1) and row length (pass 2)
    int c1;          // columns per pass-1 work-group
    int nt1;         // threads per pass-1 work-group
    int b2;          // rows per pass-2 work-group
    int nt2;         // threads per pass-2 work-group
    int units;       // (template, segment) units per batch
    bool fused;      // pipelined step kernel (pass 1 of batch b with pass 2 of batch b-1)
    int xs;          // pass-2 exchange: 0 complex values, 1 real and imaginary parts one
                     // after the other (half the LDS), 2 as 1 with bank-conflict-free layouts
    bool prune1;     // pass 1 skips the stage-0 transform where a band has only rows k1 < N1/16
    bool pre0;       // pass 1 applies the row factor of pass 2's first stage (see FilterArgs::pre0_r0)
    bool persist;    // pass 1 as a persistent kernel over a queue of tiles, heaviest units first
};
// plan flags (last entry of the public plan array)
inline int plan_flags(const Plan& p) {
    return (p.fused ? 1 : 0) | (p.xs >= 1 ? 2 : 0) | (p.xs == 2 ? 4 : 0) | (p.prune1 ? 8 : 0) | (p.pre0 ? 16 : 0) |
           (p.persist ? 32 : 0);
}
// largest radix of the pass-2 stages (16 or 8), from the pass-2 threads
inline int plan_r2(const Plan& p) { return p.nt2 == p.b2 * p.n2 / 8 ? 8 : 16; }
// pre0 needs every pass-1 work-group inside one block of N2/R0 columns
inline bool pre0_fits(const Plan& p) { return (p.n2 / plan_r2(p)) % p.c1 == 0; }

Plan default_plan(int log2n, mf_precision prec);
bool plan_supported(const Plan& p, mf_precision prec);
// instantiated shapes for this N and precision (units = 0); returns the count
int plan_candidates(int log2n, mf_precision prec, Plan* out, int cap);
// the default plan, or the one installed by mf_set_plan
Plan select_plan(int log2n, mf_precision prec);

size_t cx_bytes(mf_precision prec);

// Workspace carve-up of mf_filter.
struct FilterLayout {
    size_t off_w, off_inter, inter_bytes, off_keys, off_counts, off_part, off_tw2, off_lpt, off_lpt_ctr, total;
    int64_t units_per_batch;
};
// FP64 pass 2 of the 4096-point rows (three radix-16 stages, one row per
// work-group) applies the whole four-step factor at stage 0 and reads the last
// stage's factors w^(k r), k < 256, 1 <= r < 16, from a constant table in the
// workspace.
constexpr int kTw2Span = 256, kTw2Radix = 16;
inline bool pass2_uses_tw2(mf_precision prec, int n2, int b2, int nt2) {
    return prec == MF_FP64 && n2 == kTw2Span * kTw2Radix && b2 == 1 && nt2 == 256;
}
hipError_t launch_tw2_fill(mf_precision prec, void* tw2, hipStream_t s);
FilterLayout filter_layout(const Plan& p, mf_precision prec, int64_t n, int64_t n_tmpl, int64_t n_seg);

struct FilterArgs {
    const void* wgt;          // [n_seg][n/2+1] weighted data
    const mf_bank_entry* bank;
    void* inter;              // [units][n]
    unsigned long long* keys; // [n_units] (FP32 modes)
    unsigned int* counts;     // [n_units] (FP32 modes)
    void* partials;           // [n_units][n1/b2] (FP64)
    int64_t n_tmpl, n_seg, n_units;
    int64_t unit0, units;     // batch
    int64_t j_begin, j_end;
    double rho_threshold;
    const int32_t* series_units;
    int32_t n_series;
    void* rho;                // series output
    const void* raw_in;       // mf_ifft input  [units][n]
    void* raw_out;            // mf_ifft output [units][n]
    // chi^2 band mode (Eq. (5))
    const int32_t* band_tab;  // [n_tmpl][2 p_bands + 3]: edges e_0..e_p, index of the transformed band, slot starts
    int32_t p_bands;
    void* qbuf;               // [units][band_slot_stride]: the template x weight product of the bands pass 1 does not transform
    void* chi_series;         // chi^2 series output [n_series][n]
    // events: per (unit, window of 2^ev_log2w samples) u64 keys of the loudest
    // sample at or above the threshold (see event_key32 / event_key64)
    unsigned long long* ev_keys;  // [n_units][n >> ev_log2w], unit u = s * n_tmpl + t
    int32_t ev_log2w;
    const void* tw2;              // [kTw2Radix - 1][kTw2Span] last-stage factors (see pass2_uses_tw2)
    int32_t prune1;               // pass 1 skips the stage-0 transform of narrow bands (plan flag bit 3)
    // pre0_r0 > 0 (plan flag bit 4): pass 1 multiplies its output Y[j1][k2] by
    // e^{2 pi i j1 floor(k2 / (N2/R0)) / (N1 R0)}, the factor pass 2's first
    // stage (radix R0 = pre0_r0) would apply to that input, and pass 2 skips it
    int32_t pre0_r0;
    // persistent pass 1 (plan flag bit 5): the batch's units in the order their
    // tiles are taken (most band rows first) and the queue counter, both
    // written by k_lpt_order before each pass-1 launch
    const int32_t* lpt_order;  // [units]
    unsigned int* lpt_ctr;
};

// Workspace carve-up of mf_filter_chisq (band mode).
struct BandLayout {
    size_t off_w, off_tab, off_q, off_inter, off_part, total;
    int64_t units_per_batch;
};
// the built-in band-mode shape for this N and precision (log2n = -1 if none)
Plan default_band_plan(int log2n, mf_precision prec);
bool band_plan_supported(const Plan& p, mf_precision prec);
// the default band-mode plan, or the one installed by mf_set_band_plan
Plan band_plan(int log2n, mf_precision prec);
BandLayout band_layout(const Plan& p, mf_precision prec, int64_t n, int64_t n_tmpl, int64_t n_seg, int p_bands);

// Launchers (return hipError_t of the launch)
hipError_t launch_pass1(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s);
// persistent pass 1: the batch's work order and queue reset, then the kernel
hipError_t launch_pass1_lpt(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s);
hipError_t launch_pass2(const Plan& p, mf_precision prec, bool raw, const FilterArgs& a, hipStream_t s);
hipError_t launch_step(const Plan& p, mf_precision prec, const FilterArgs& a1, const FilterArgs& a2, hipStream_t s);
hipError_t launch_finalize(const Plan& p, mf_precision prec, const FilterArgs& a, mf_peak* peaks, hipStream_t s);

hipError_t launch_band_table(int64_t n, int n2, const mf_bank_entry* bank, int64_t n_tmpl, const double* prefix,
                             int p, int32_t* tab, hipStream_t s);
hipError_t launch_pass1_band(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s);
hipError_t launch_pass2_band(const Plan& p, mf_precision prec, const FilterArgs& a, hipStream_t s);
hipError_t launch_finalize_band(const Plan& p, const FilterArgs& a, mf_peak* peaks, double* chisq, hipStream_t s);

hipError_t launch_rfft_pack(mf_precision prec, const void* x, void* y, int64_t m, int64_t batch, hipStream_t s);
hipError_t launch_rfft_post(mf_precision prec, const void* z, void* out, int64_t m, int64_t batch, double dt,
                            hipStream_t s);

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t s);
hipError_t launch_events(const unsigned long long* keys, int64_t n_tmpl, int64_t n_seg, int64_t n_win, int log2w,
                         bool f64, const mf_bank_entry* bank, mf_event* unit_ev, mf_event* best, mf_event* seg_ev,
                         hipStream_t s);

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_psd(int64_t n, double fs, double f_low, double f0, int k_lo, double* Sn, hipStream_t s);
hipError_t launch_prefix(int64_t n, double fs, const double* Sn, double* prefix, hipStream_t s);
hipError_t launch_weights(int64_t n, double fs, int k_lo, mf_precision prec, const void* stilde, int64_t n_seg,
                          const double* Sn, void* wgt, hipStream_t s);
hipError_t launch_sigma(int64_t n, double fs, mf_sigma_mode mode, const double* Sn, mf_bank_entry* bank,
                        int64_t n_tmpl, hipStream_t s);
hipError_t launch_spa_synth(int64_t n, double fs, mf_precision prec, const mf_bank_entry* bank, int64_t n_tmpl,
                            void* htilde, hipStream_t s);
hipError_t launch_chisq(int64_t n, double fs, mf_precision prec, const mf_bank_entry* bank, int64_t n_tmpl,
                        const void* stilde, int64_t n_seg, const double* Sn, const double* prefix, int p,
                        const mf_peak* peaks, const mf_event* events, int64_t n_per_seg, double* chisq, double* rho,
                        hipStream_t s);
hipError_t launch_metric(int64_t n, double fs, int k_lo, const double* theta, const int32_t* khi, int64_t count,
                         const double* Sn, double* metric, hipStream_t s);
hipError_t launch_snr_grad(int64_t n, double fs, int k_lo, mf_precision prec, const double* theta,
                           const int32_t* khi, const int32_t* seg, int64_t count, const void* stilde,
                           int64_t n_seg, const double* Sn, double* Z, double* rho2, const double* gbar, double* grad,
                           hipStream_t s);

}  // namespace mf
