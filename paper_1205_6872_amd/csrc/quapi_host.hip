// Host runtime of the QUAPI library: parameter validation, footprint,
// quadrature planning, workspace layout, step planning, and the C ABI
// declared in include/quapi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "quapi.h"
#include "quapi_internal.h"

using namespace quapi;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
constexpr int kRhoStage = 1024;          // rho slots of the blocking-call staging buffer
constexpr double kOhmicCutoffFactor = 46.0;  // exp(-46) ~ 1e-20 of the integrand left out
// Full-window steps of tensors up to this many entries are replayed from
// captured graphs (two single steps, or one fused launch): they are bound by
// their launches, not by HBM.  The single step takes mirror mode only above it.
constexpr size_t kGraphMaxEntries = size_t(1) << 22;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool checked_pow(size_t base, int e, size_t *out) {
    size_t r = 1;
    for (int i = 0; i < e; ++i) {
        if (base != 0 && r > std::numeric_limits<size_t>::max() / base) return false;
        r *= base;
    }
    *out = r;
    return true;
}

long long ipow_ll(int b, int e) {
    long long r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// ---------------------------------------------------------------- planning
// Digit split of the m index of a step (see step_kernel): d_lo digits per
// thread, d_mid swept by the block loop, the rest indexed by the block.
struct DigitSplit {
    int d_lo, d_mid, R, Q, grid;
};

DigitSplit split_digits(int N, int n_digits) {
    int d_lo_max = 0, d_mid_target = 0;
    switch (N) {
    case 4: d_lo_max = 4; d_mid_target = 2; break;    // R = 256 = block, Q <= 16
    case 9: d_lo_max = 2; d_mid_target = 2; break;    // R = 81 (243 threads active), Q <= 81
    case 16: d_lo_max = 1; d_mid_target = 1; break;   // R = 16, Q <= 16 (LDS budget)
    default: break;                                   // N = 1: a single entry
    }
    DigitSplit s;
    s.d_lo = std::min(d_lo_max, n_digits);
    const int avail = n_digits - s.d_lo;
    s.d_mid = std::min(d_mid_target, avail);
    // keep at least ~1024 blocks in flight when the tensor allows it
    while (s.d_mid > 0 && ipow_ll(N, avail - s.d_mid) < 1024) --s.d_mid;
    // One sweep row leaves threads without an item: at N = 9 all but 81 of
    // a block's 256, at N = 16 (MFMA, a row per wave) three of its four
    // waves.  One middle digit pays from 512 blocks at N = 9 (M = 3, L = 7,
    // rho every step: 0.081 -> 0.062 ms per step) and from 256 at N = 16
    // (M = 4, L = 5: 0.034 -> 0.021 ms).
    if (N == 9 && s.d_mid == 0 && avail >= 1 && ipow_ll(N, avail - 1) >= 512) s.d_mid = 1;
    if (N == 16 && s.d_mid == 0 && avail >= 1 && ipow_ll(N, avail - 1) >= 256) s.d_mid = 1;
    s.R = (int)ipow_ll(N, s.d_lo);
    s.Q = (int)ipow_ll(N, s.d_mid);
    s.grid = (int)ipow_ll(N, avail - s.d_mid);
    return s;
}

// Digit split of m for the fused two-step kernel (N = 4, L - 2 digits): the
// low digits per thread (R <= 64, so that the four tables of per-thread
// products fit in LDS), two sweep digits, the rest per block.
DigitSplit split_digits2(int n_digits) {
    constexpr int N = 4;
    DigitSplit s;
    s.d_lo = std::min(3, n_digits);
    const int avail = n_digits - s.d_lo;
    s.d_mid = std::min(3, avail);
    while (s.d_mid > 0 && ipow_ll(N, avail - s.d_mid) < 1024) --s.d_mid;
    s.R = (int)ipow_ll(N, s.d_lo);
    s.Q = (int)ipow_ll(N, s.d_mid);
    s.grid = (int)ipow_ll(N, avail - s.d_mid);
    return s;
}

// The fused two-step kernel applies to N = 4 (its N^2 inputs per item fit in
// registers) and L >= 3: two points to sum out, and the factor of the second
// oldest point seen from the first new one at lag L-1 >= 2, so that it carries
// no K and its rows of the diagonal points are ones (the kernel uses that).
bool fused_ok(int N, int L) { return N == 4 && L >= 3; }

// The three-step kernel runs for N = 4, L >= 4 (three points to sum out; the
// step-n group factors at lags L-1 and L-2 >= 2, for the same reason).
bool triple_ok(int N, int L) { return N == 4 && L >= 4; }

// Full-window steps per launch chosen by default: three from L = 13 at
// complex128 and at complex64 with FP32 arithmetic (4^10 items and more; the
// step is HBM bound there, and a third step in registers saves a third of
// the traffic); two otherwise.  A three-step item runs one wave per SIMD
// through three dependent stages, so with fewer items than that the two-step
// kernel finishes first; with complex64 storage and FP64 arithmetic the
// three-step kernel is bound by its arithmetic (measured on one GPU with rho
// every step, both kernels in mirror mode: L = 15 1.14 ms per step with three
// steps per launch, 1.00 with two; L = 12 complex128 0.061 and 0.048).
int fusion_width(int N, int L, int prec) {
    const int from = prec == kPrecC64F64 ? 1 << 20 : 13;
    if (triple_ok(N, L) && L >= from) return 3;
    return fused_ok(N, L) ? 2 : 1;
}

int max_grid(int N, int L) {
    int g = 1;
    for (int nd = 0; nd <= L - 1; ++nd) g = std::max(g, split_digits(N, nd).grid);
    if (fused_ok(N, L)) g = std::max(g, split_digits2(L - 2).grid);
    if (triple_ok(N, L)) g = std::max(g, split_digits2(L - 3).grid);
    return g;
}

// Gauss-Legendre rule on [-1, 1]: nodes are the roots of P_n found by Newton's
// method from the Chebyshev-like initial guesses cos(pi (i + 3/4) / (n + 1/2)),
// with P_n from the three-term recurrence k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2},
// P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1), and weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Panels of the w-quadrature of G(t) for t <= t_max.  Each Gauss-Legendre
// panel spans at most: one radian of w t_max (oscillation); the distance
// max(2 pi kT, w) to the nearest pole of coth(w / 2kT) at w = 2 pi kT i
// (analyticity); omega_c for the Ohmic exp(-w / omega_c) (scale).  Panels
// never straddle a table node, where J has a kink.
void plan_panels(const quapi_params &p, double t_max, std::vector<double> &pa,
                 std::vector<double> &ph, std::vector<int> &pseg) {
    pa.clear();
    ph.clear();
    pseg.clear();
    const double inf = std::numeric_limits<double>::infinity();
    const double h_osc = t_max > 0.0 ? 1.0 / t_max : inf;
    const double d_pole = p.kT > 0.0 ? 2.0 * M_PI * p.kT : inf;
    std::vector<double> edges{0.0};
    double h_cut = inf;
    if (p.bath.kind == QUAPI_BATH_OHMIC) {
        edges.push_back(kOhmicCutoffFactor * p.bath.omega_c);
        h_cut = p.bath.omega_c;
    } else {
        for (int i = 0; i < p.bath.n_tab; ++i) edges.push_back(p.bath.omega[i]);
    }
    for (size_t k = 0; k + 1 < edges.size(); ++k) {
        const double lo = edges[k], hi = edges[k + 1];
        double x = lo;
        while (x < hi) {
            const double hmax = std::min(std::min(h_osc, h_cut), std::max(d_pole, x));
            const bool last = hi - x <= hmax * (1.0 + 1e-12);   // no sliver panels
            const double hh = last ? hi - x : hmax;
            pa.push_back(x);
            ph.push_back(hh);
            pseg.push_back(p.bath.kind == QUAPI_BATH_OHMIC ? -1 : (int)k);
            x = last ? hi : x + hh;
        }
    }
}

// ------------------------------------------------------------- validation
// Empty if H (M x M complex, interleaved) is finite and Hermitian to 1e-12 of
// its largest entry, else what is wrong.
std::string hermitian_error(const double *H, int M, const char *name) {
    double hmax = 0.0;
    for (int i = 0; i < 2 * M * M; ++i) {
        if (!std::isfinite(H[i])) return std::string(name) + " has a non-finite entry";
        hmax = std::max(hmax, std::fabs(H[i]));
    }
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            const double re = H[2 * (a * M + b)], im = H[2 * (a * M + b) + 1];
            const double re2 = H[2 * (b * M + a)], im2 = H[2 * (b * M + a) + 1];
            if (std::fabs(re - re2) > 1e-12 * hmax || std::fabs(im + im2) > 1e-12 * hmax)
                return std::string(name) + " is not Hermitian";
        }
    return "";
}

// Largest N^dk_max (as a power of two) of a dense context, and of a filtered
// one (its keys are 64-bit flat indices).
constexpr int kDenseMaxLog2 = 40;
constexpr int kFilterMaxLog2 = 62;

std::string validate(const quapi_params *p, int max_log2 = kDenseMaxLog2) {
    char buf[256];
    if (!p) return "params is NULL";
    if (p->M < 1 || p->M > kMaxM) {
        snprintf(buf, sizeof buf, "M = %d outside 1..%d", p->M, kMaxM);
        return buf;
    }
    if (!p->s || !p->H || !p->rho0) return "s, H and rho0 must be non-NULL";
    const int M = p->M;
    for (int i = 0; i < M; ++i)
        if (!std::isfinite(p->s[i])) return "s has a non-finite entry";
    for (int i = 0; i < 2 * M * M; ++i)
        if (!std::isfinite(p->rho0[i])) return "rho0 has a non-finite entry";
    std::string herr = hermitian_error(p->H, M, "H");
    if (!herr.empty()) return herr;
    if (p->n_H < 0 || p->n_H > 1000000) return "n_H must be in 0..1000000";
    if (p->n_H > 0 && !p->H_t) return "H_t must be non-NULL when n_H > 0";
    for (int k = 0; k < p->n_H; ++k) {
        herr = hermitian_error(p->H_t + (size_t)2 * M * M * k, M, "an H_t matrix");
        if (!herr.empty()) {
            snprintf(buf, sizeof buf, "%s (index %d)", herr.c_str(), k);
            return buf;
        }
    }
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return "dt must be finite and > 0";
    if (p->dk_max < 1 || p->dk_max > kMaxL) {
        snprintf(buf, sizeof buf, "dk_max = %d outside 1..%d", p->dk_max, kMaxL);
        return buf;
    }
    if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return "kT must be finite and >= 0";
    if (p->dtype != QUAPI_C128 && p->dtype != QUAPI_C64 && p->dtype != QUAPI_C64_F64)
        return "dtype must be QUAPI_C128, QUAPI_C64 or QUAPI_C64_F64";
    const quapi_bath &b = p->bath;
    if (b.kind == QUAPI_BATH_OHMIC) {
        if (!(b.xi >= 0.0) || !std::isfinite(b.xi)) return "Ohmic xi must be finite and >= 0";
        if (!(b.omega_c > 0.0) || !std::isfinite(b.omega_c)) return "Ohmic omega_c must be finite and > 0";
    } else if (b.kind == QUAPI_BATH_TABLE) {
        if (b.n_tab < 1 || b.n_tab > 1000000) return "table n_tab must be in 1..1000000";
        if (!b.omega || !b.J) return "table omega and J must be non-NULL";
        for (int i = 0; i < b.n_tab; ++i) {
            if (!std::isfinite(b.omega[i]) || !std::isfinite(b.J[i])) return "table has a non-finite entry";
            if (b.J[i] < 0.0) return "table J must be >= 0";
            if (i == 0 ? !(b.omega[0] > 0.0) : !(b.omega[i] > b.omega[i - 1]))
                return "table omega must be > 0 and strictly increasing";
        }
    } else {
        return "bath.kind must be QUAPI_BATH_OHMIC or QUAPI_BATH_TABLE";
    }
    size_t entries;
    if (!checked_pow((size_t)M * M, p->dk_max, &entries) || entries > (size_t)1 << max_log2)
        return "N^dk_max is too large";
    return "";
}

// ------------------------------------------------------------------ layout
struct Layout {
    size_t a_bytes;                  // one tensor buffer
    size_t off_a0, off_a1, off_bank, off_bankf, off_g, off_eta, off_U, off_s, off_H, off_Ht, off_Ut, off_rho0;
    size_t off_pa, off_ph, off_pseg, off_tw, off_tJ, off_glx, off_glw, off_partials, off_stage;
    size_t off_plan, off_plan2, off_coef, off_plan3, off_coef3, off_blk3, off_low3, off_blk2, off_low2, off_blk1,
        off_low1, off_pairs, off_sink;
    // filtered contexts: keys and values of the two tensors, flags, segment
    // starts, scan partials, counters, rho partials, factor-level tables
    size_t off_fkeys[2], off_fvals[2], off_fmask, off_fbofs, off_fctr, off_fpart, off_fplan;
    size_t fplan_entries;            // entries of one factor-level table set
    size_t total;
    int n_panels, n_tables, partial_blocks;
    int n_canon3, n_diag3, parts3, span3;   // mirror mode of the three-step kernel (high-digit blocks)
    int n_low3;                             // items of a block below their mirror (mode 2's list)
    int n_canon2, n_diag2, parts2, span2;   // mirror mode of the two-step kernel
    int n_low2;                             // items of a block below their mirror (its list)
    int n_canon1, n_diag1, parts1, span1;   // mirror mode of the single step (main split)
    int n_low1;                             // N = 9: items of a block below their mirror (its list)
    DigitSplit main_split;   // digit split of the full-window steps
    DigitSplit split2;       // digit split of the fused two-step kernel
    DigitSplit split3;       // digit split of the three-step kernel
};

constexpr int kSlots = 4;    // rho partial buffers: a fused launch takes two

// The three-step mirror launch of the self-mirror items (mode 3) runs
// concurrently with the mode-1 launch from 2^28 entries, in its tail (below
// 2^28 entries the fork and join cost more than they hide).
bool step3_concurrent(size_t entries, int prec) {
    (void)prec;
    return entries >= (size_t(1) << 28);
}

// Blocks per high-digit value in mirror mode 2: about one block per compute
// unit (256 on MI355X) over the n_diag values, at most one per sweep pass.
int mirror_parts(int passes, int n_diag) {
    const int want = n_diag > 0 ? (256 + n_diag - 1) / n_diag : 1;
    return std::max(1, std::min(passes, want));
}

// The full-window single step has a mirror mode at N = 4, 9 (vector kernel)
// and N = 16 (MFMA kernel, which needs R = 16), from L = 2.
bool single_mirror_ok(int N, int L, const DigitSplit &main_split) {
    return L >= 2 && (N == 4 || N == 9 || (N == 16 && main_split.R == 16));
}

// filter_cap > 0: a filtered context holding up to filter_cap kept entries
// (no dense tensors, no dense-step plans, mirror or fused-step buffers).
Layout make_layout(const quapi_params &p, int n_panels, size_t filter_cap = 0) {
    Layout l{};
    const int M = p.M, N = M * M, L = p.dk_max;
    const bool filtered = filter_cap > 0;
    size_t entries = 1;
    checked_pow((size_t)N, L, &entries);
    const size_t cs = p.dtype == QUAPI_C128 ? 16 : 8;
    l.n_panels = n_panels;
    l.n_tables = BankLayout{L}.count();
    const DigitSplit none{0, 0, 1, 1, 1};
    l.partial_blocks = filtered ? 1 : max_grid(N, L);
    l.main_split = filtered ? none : split_digits(N, L - 1);
    l.split2 = !filtered && fused_ok(N, L) ? split_digits2(L - 2) : none;
    const bool triple = !filtered && triple_ok(N, L);
    l.split3 = triple ? split_digits2(L - 3) : DigitSplit{0, 0, 1, 1, 1};
    if (triple) {
        // mirror mode: blocks whose high digits are below their mirror, and
        // those equal to it (all diagonal), split into one sweep row per thread
        const DigitSplit &s3 = l.split3;
        for (int h = 0; h < s3.grid; ++h) {
            const long long hb = mirror4(h);
            if (h < hb) ++l.n_canon3;
            else if (h == hb) ++l.n_diag3;
        }
        // the blocks of the diagonal values walk the list of a block's items
        // below their mirror, one item per thread, two passes per block, as
        // the tail of the mode-1 launch
        for (int low = 0; low < s3.R * s3.Q; ++low)
            if (mirror4(low) > low) ++l.n_low3;
        const int passes = (l.n_low3 + kBlock - 1) / kBlock;
        l.parts3 = std::max(1, (passes + 1) / 2);
        l.span3 = ((passes + l.parts3 - 1) / l.parts3) * kBlock;
        l.partial_blocks = std::max(l.partial_blocks, l.n_canon3 + l.n_diag3 * (l.parts3 + 1));
    }
    if (!filtered && fused_ok(N, L)) {
        // the two-step kernel: the same partition over its block digits
        const DigitSplit &s2 = l.split2;
        for (int h = 0; h < s2.grid; ++h) {
            const long long hb = mirror4(h);
            if (h < hb) ++l.n_canon2;
            else if (h == hb) ++l.n_diag2;
        }
        for (int low = 0; low < s2.R * s2.Q; ++low)
            if (mirror4(low) > low) ++l.n_low2;
        const int passes = (l.n_low2 + kBlock - 1) / kBlock;
        l.parts2 = std::max(1, (passes + 1) / 2);
        l.span2 = ((passes + l.parts2 - 1) / l.parts2) * kBlock;
        l.partial_blocks = std::max(l.partial_blocks, l.n_canon2 + l.n_diag2 * (l.parts2 + 1));
    }
    if (!filtered && single_mirror_ok(N, L, l.main_split)) {
        // the N = 9 step and the N = 16 MFMA step: the same partition over
        // their block digits; a block sweeps its rows with its 4 waves (MFMA)
        // or its kBlock / R thread columns
        const DigitSplit &s1 = l.main_split;
        for (int h = 0; h < s1.grid; ++h) {
            const long long hb = mirror_n(N, h);
            if (h < hb) ++l.n_canon1;
            else if (h == hb) ++l.n_diag1;
        }
        if (N == 9) {
            // the listed items of the diagonal values, one per active thread
            // (kBlock / R columns of R), two passes per block, in the tail of
            // the mode-1 launch
            for (int low = 0; low < s1.R * s1.Q; ++low)
                if (mirror9(low) > low) ++l.n_low1;
            const int active = (kBlock / s1.R) * s1.R;
            const int passes = (l.n_low1 + active - 1) / active;
            l.parts1 = std::max(1, (passes + 1) / 2);
            l.span1 = ((passes + l.parts1 - 1) / l.parts1) * active;
        } else {
            const int rows_per_pass = N == 16 ? kBlock / 64 : kBlock / s1.R;
            const int passes = (s1.Q + rows_per_pass - 1) / rows_per_pass;
            l.parts1 = mirror_parts(passes, l.n_diag1);
            l.span1 = ((passes + l.parts1 - 1) / l.parts1) * rows_per_pass;
        }
        l.partial_blocks = std::max(l.partial_blocks, l.n_canon1 + l.n_diag1 * (l.parts1 + 1));
    }
    l.a_bytes = filtered ? 0 : entries * cs;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.off_a0 = take(l.a_bytes);
    l.off_a1 = take(l.a_bytes);
    l.off_bank = take((size_t)l.n_tables * N * N * 16);
    l.off_bankf = take(p.dtype == QUAPI_C64 ? (size_t)l.n_tables * N * N * 8 : 0);
    l.off_g = take((size_t)(2 * L + 3) * 16);
    l.off_eta = take((size_t)(4 * L + 2) * 16);
    l.off_U = take((size_t)M * M * 16);
    l.off_s = take((size_t)M * 8);
    l.off_H = take((size_t)M * M * 16);
    l.off_Ht = take((size_t)std::max(p.n_H, 0) * M * M * 16);
    l.off_Ut = take((size_t)std::max(p.n_H, 0) * M * M * 16);
    l.off_rho0 = take((size_t)N * 16);
    l.off_pa = take((size_t)n_panels * 8);
    l.off_ph = take((size_t)n_panels * 8);
    l.off_pseg = take((size_t)n_panels * 4);
    const int nt = p.bath.kind == QUAPI_BATH_TABLE ? p.bath.n_tab : 1;
    l.off_tw = take((size_t)nt * 8);
    l.off_tJ = take((size_t)nt * 8);
    l.off_glx = take(kGL * 8);
    l.off_glw = take(kGL * 8);
    l.off_partials = take((size_t)kSlots * l.partial_blocks * N * 16);
    l.off_stage = take((size_t)kRhoStage * N * 16);
    l.off_pairs = take((size_t)kRhoSlices * N * 2 * 16);
    l.off_sink = take(sizeof(RhoSink));
    // six FP64 factor tables of the full-window split: [N][R], [N][Q], [N][grid], x2 classes
    const DigitSplit &ms = l.main_split;
    l.off_plan = take(filtered ? 0 : (size_t)2 * N * (ms.R + ms.Q + ms.grid) * 16);
    // four table sets (interior / final, steps n and n+1) of the fused split
    const DigitSplit &s2 = l.split2;
    const bool fused = !filtered && fused_ok(N, L);
    l.off_plan2 = take(fused ? (size_t)4 * N * (s2.R + s2.Q + s2.grid) * 16 : 0);
    l.off_coef = take(fused ? (size_t)kCoefCount * 16 : 0);
    // six table sets (interior / final, steps n, n+1, n+2) of the three-step split
    const DigitSplit &s3 = l.split3;
    l.off_plan3 = take(triple ? (size_t)6 * N * (s3.R + s3.Q + s3.grid) * 16 : 0);
    l.off_coef3 = take(triple ? (size_t)kC3Count * 16 : 0);
    l.off_blk3 = take(triple ? (size_t)(l.n_canon3 + l.n_diag3) * sizeof(int) : 0);
    l.off_low3 = take(triple ? (size_t)l.n_low3 * sizeof(int) : 0);
    l.off_blk2 = take((size_t)(l.n_canon2 + l.n_diag2) * sizeof(int));
    l.off_low2 = take((size_t)l.n_low2 * sizeof(int));
    l.off_blk1 = take((size_t)(l.n_canon1 + l.n_diag1) * sizeof(int));
    l.off_low1 = take((size_t)l.n_low1 * sizeof(int));
    const size_t fc = filtered ? filter_cap : 0;
    for (int b = 0; b < 2; ++b) {
        l.off_fkeys[b] = take(fc * 8);
        l.off_fvals[b] = take(fc * cs);
    }
    l.off_fmask = take(fc * 2);                      // a keep mask per input entry (segment heads)
    l.off_fbofs = take(filtered ? (size_t)N * kFilterStepBlocks * 8 : 0);
    l.off_fctr = take(filtered ? 8 * 8 : 0);          // entry counts of both buffers, overflow flag
    l.off_fpart = take(filtered ? (size_t)kFilterStepBlocks * N * 16 : 0);
    l.fplan_entries = filtered ? std::max<size_t>(1, filter_plan_entries(N, L - 1)) : 0;
    l.off_fplan = take(l.fplan_entries * 2 * 16);
    l.total = off;
    return l;
}

int count_panels(const quapi_params &p) {
    std::vector<double> a, h;
    std::vector<int> s;
    plan_panels(p, (p.dk_max + 1) * p.dt, a, h, s);
    return (int)a.size();
}

}  // namespace

// ----------------------------------------------------------------- context
struct quapi_ctx {
    int M = 0, N = 0, L = 0;
    int prec = kPrecC128;         // quapi_dtype
    size_t csize = 16;            // bytes per stored tensor entry
    double dt = 0.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // one stream only (quapi_propagate_static): no side or aux streams, no
    // events, the rho finalize on the context's stream, no graphs
    bool one_stream = false;
    // rho finalize kernels run on a side stream, overlapped with the next
    // step; the block partials rotate over kSlots buffers between the streams
    hipStream_t side = nullptr;
    hipEvent_t ev_step[kSlots] = {}, ev_fin[kSlots] = {};
    // the small mirror-mode launches of a three-step group (modes 2, 3) run
    // on a third stream, concurrently with mode 1, joined before the next work
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool fin_pending[kSlots] = {};
    int next_slot = 0;
    char *ws = nullptr;
    bool own_ws = false;
    Layout lay{};
    void *A[2] = {nullptr, nullptr};
    int cur = 0;                  // A[cur] holds the tensor after global step `step`
    int step = 0;
    double2 *bank = nullptr, *g = nullptr, *eta = nullptr, *U = nullptr, *rho0_d = nullptr;
    double2 *partials[kSlots] = {};
    double2 *stage = nullptr, *plan = nullptr, *plan2 = nullptr, *pairs = nullptr;
    void *coef = nullptr;         // fused-step coefficients (compute precision)
    int n_H = 0;                  // driven: per-interval Hamiltonians on the device
    const double2 *Ht_d = nullptr;
    double2 *Ut_d = nullptr;      // driven: U_k = exp(-i H_t[k] dt), computed at create
    std::vector<double> Ht_h;
    TablesArgs drive_ta{};        // the setup tables call, reused per step with k_only
    float2 *bank_f = nullptr;     // the bank rounded to complex64 (FP32 arithmetic only)
    RhoSink *sink = nullptr;
    // captured full-window steps, [without / with rho]: graph1 two single steps
    // A[0] -> A[1] -> A[0]; graph2[.][p] one fused launch A[p] -> A[1-p]
    hipGraphExec_t graph1[2] = {}, graph2[2][2] = {}, graph3[2][2] = {};
    bool graph_failed = false;
    bool plan_ready = false;      // full-window factor tables computed
    bool plan2_ready = false;     // fused-step factor tables computed
    bool plan3_ready = false;     // three-step factor tables computed
    int fuse = 1;                 // full-window steps per launch (fusion_width)
    bool fuse_pinned = false;     // quapi_set_fused_steps chose a width
    // persistent path (small tensors, quapi_small.hip): 0 off, 1 tensor in
    // LDS, 2 tensor in the context's global buffers
    int small = 0;
    // Mirror mode of the full-window kernels: they read and write only the
    // entries not above their mirror; half_cur says A[cur] holds only those.
    bool mirror_ok = false;       // M = 2, 3, 4, L >= 2, rho0 exactly Hermitian
    int mirror = 0;               // 0 off, 1 where it pays, 2 at every size (quapi_set_mirror)
    bool half_cur = false;
    int *blk3 = nullptr;          // high-digit values: n_canon3 below their mirror, then n_diag3 equal
    std::vector<int> blk3_h;
    int *low3 = nullptr;          // mode 2's list of the items qm * R + r below their mirror
    std::vector<int> low3_h;
    int *blk2 = nullptr;          // the same for the two-step kernel (n_canon2, n_diag2)
    std::vector<int> blk2_h;
    int *low2 = nullptr;          // its list of the items below their mirror
    std::vector<int> low2_h;
    int *blk1 = nullptr;          // the same for the single step (n_canon1, n_diag1)
    std::vector<int> blk1_h;
    int *low1 = nullptr;          // N = 9: its list of the items below their mirror
    std::vector<int> low1_h;
    double2 *plan3 = nullptr;
    void *coef3 = nullptr;
    // Filtered propagation (quapi_create_filtered): the kept entries as sorted
    // (key, value) pairs in two buffers of fcap entries, fkeys[cur] / fvals[cur]
    // the current tensor; fctr[0], fctr[1] their entry counts, fctr[2] (as int)
    // the sticky overflow flag; fmask the keep masks, fbofs the per-(o, block)
    // counts and offsets of a step.
    bool filtered = false;
    double theta = 0.0;
    size_t fcap = 0;
    unsigned long long *fkeys[2] = {nullptr, nullptr};
    void *fvals[2] = {nullptr, nullptr};
    unsigned short *fmask = nullptr;
    unsigned long long *fbofs = nullptr, *fctr = nullptr;
    double2 *fpart = nullptr, *fplan = nullptr;
    size_t fplan_entries = 0;
    int fplan_for = -1;           // the step set fplan holds: 0 the full window, n growth step n
    std::vector<double> rho0_h;
    // host copies of uploaded inputs (kept alive until the uploads complete)
    std::vector<double> s_h, H_h, pa_h, ph_h, tw_h, tJ_h, glx_h, glw_h;
    // N = 16: the new points grouped by the classes of their oldest-point
    // rows for the MFMA step (Cls16), when such a grouping exists
    bool cls_ok = false;
    unsigned long long cls_out = 0;
    unsigned cls_rep = 0, cls_selb = 0;
    std::vector<int> pseg_h;
    std::string err;
    std::atomic<int> busy{0};
    // timing
    bool timing = false;
    double setup_ms = 0.0;
    // steps: full-window steps covered; width: steps per launch of a fused or
    // single step (1..3), 0 for a persistent launch
    struct Rec { int kind; hipEvent_t a, b; int steps; int width; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double acc_ms[3] = {0, 0, 0};
    long long acc_n[3] = {0, 0, 0};
    long long acc_steps = 0;      // full-window steps covered by timed step launches
    double acc_width_ms[4] = {0, 0, 0, 0};      // full-window launches by the steps they cover
    long long acc_width_n[4] = {0, 0, 0, 0};
};

namespace {

quapi_status fail(quapi_ctx *ctx, quapi_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (ctx) ctx->err = buf;
    return st;
}

#define HIP_TRY(ctx, call)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, QUAPI_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct BusyGuard {
    quapi_ctx *c;
    bool ok;
    explicit BusyGuard(quapi_ctx *cx) : c(cx) {
        int z = 0;
        ok = c->busy.compare_exchange_strong(z, 1);
    }
    ~BusyGuard() {
        if (ok) c->busy.store(0);
    }
};

hipEvent_t take_event(quapi_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Build the step arguments for global step n (1-based).
struct StepPlan {
    StepArgs args;
    DigitSplit split;
    bool grow;
};

// The bank tables of global step n: a.n_digits, a.tab / a.tabf per digit of
// m, and the oldest-point (full window) or self (growth) tables.
void step_tables(int L, int n, StepArgs &a) {
    const BankLayout B{L};
    const bool grow = n < L;
    a.n_digits = grow ? n : L - 1;
    if (grow) {
        // digits are points 0 .. n-1; point 0 couples through the initial-point classes
        for (int j = 0; j < n; ++j) {
            if (j == 0) {
                a.tab[j] = (int16_t)(n == 1 ? B.k_init1() : B.init(n));
                a.tabf[j] = (int16_t)(n == 1 ? B.k_fin_init1() : B.fin_init(n));
            } else {
                const int lag = n - j;
                a.tab[j] = (int16_t)(lag == 1 ? B.k_lag1() : B.lag(lag));
                a.tabf[j] = (int16_t)(lag == 1 ? B.k_fin1() : B.fin(lag));
            }
        }
        a.old_tab = B.self_int();
        a.oldf_tab = B.self_end();
    } else {
        // digits are points n-L+1 .. n-1 (lags L-1 .. 1); the oldest point n-L is summed
        for (int j = 0; j < L - 1; ++j) {
            const int lag = L - 1 - j;
            a.tab[j] = (int16_t)(lag == 1 ? B.k_lag1() : B.lag(lag));
            a.tabf[j] = (int16_t)(lag == 1 ? B.k_fin1() : B.fin(lag));
        }
        a.old_tab = n == L ? B.old_first() : B.old_main();
        a.oldf_tab = n == L ? B.oldf_first() : B.oldf_main();
    }
}

// QUAPI_STEP16_CLASSES=0 in the environment at context creation keeps every
// output's own row in the M = 4 MFMA step (for comparisons of the two forms).
bool cls16_disabled() {
    const char *v = std::getenv("QUAPI_STEP16_CLASSES");
    return v && std::strcmp(v, "0") == 0;
}

// The new points o = (a, b) of M = 4 whose oldest-point influence rows are
// equal (s_a - s_b equal to 8 ulps of the largest difference: the rows are
// equal in exact arithmetic, and differ by rounding only), packed onto the
// MFMA step's 4 lane groups of 4 outputs with at most 2 classes per group.
// Returns false when no such packing exists (the step then contracts every
// output's own row).
bool pack_classes16(const std::vector<double> &s, unsigned long long *out, unsigned *rep, unsigned *selb) {
    if (s.size() != 4) return false;
    double del[16], scale = 0.0;
    for (int o = 0; o < 16; ++o) {
        del[o] = s[o / 4] - s[o % 4];
        scale = std::max(scale, std::fabs(del[o]));
    }
    const double tol = 8.0 * DBL_EPSILON * scale;
    int cls[16], reps[16], n_cls = 0;
    for (int o = 0; o < 16; ++o) {
        cls[o] = -1;
        for (int k = 0; k < n_cls && cls[o] < 0; ++k)
            if (std::fabs(del[o] - del[reps[k]]) <= tol) cls[o] = k;
        if (cls[o] < 0) {
            reps[n_cls] = o;
            cls[o] = n_cls++;
        }
    }
    // depth-first assignment of the outputs, class by class, to the groups
    int order[16], n = 0;
    for (int k = 0; k < n_cls; ++k)
        for (int o = 0; o < 16; ++o)
            if (cls[o] == k) order[n++] = o;
    int grp[16], cnt[4] = {0, 0, 0, 0}, ca[4] = {-1, -1, -1, -1}, cb[4] = {-1, -1, -1, -1};
    std::function<bool(int)> place = [&](int i) -> bool {
        if (i == 16) return true;
        const int k = cls[order[i]];
        bool tried_empty = false;
        for (int g = 0; g < 4; ++g) {
            if (cnt[g] == 4) continue;
            if (cnt[g] == 0) {
                if (tried_empty) continue;          // empty groups are interchangeable
                tried_empty = true;
            }
            const int sa = ca[g], sb = cb[g];
            if (sa >= 0 && sa != k && sb >= 0 && sb != k) continue;
            if (sa < 0) ca[g] = k;
            else if (sa != k && sb < 0) cb[g] = k;
            grp[i] = g;
            ++cnt[g];
            if (place(i + 1)) return true;
            --cnt[g];
            ca[g] = sa;
            cb[g] = sb;
        }
        return false;
    };
    if (!place(0)) return false;
    // per group: slot 0 the class of at least two outputs, listed first, then
    // the other class (slot 1; slot 1 repeats slot 0 when there is one
    // class).  The class counts are 4, 3 + 1 or 2 + 2, so outputs q = 0, 1
    // always take slot 0 and q = 3 slot 1 (the kernel fixes those); only
    // q = 2 is looked up
    unsigned long long po = 0;
    unsigned pr = 0, ps = 0;
    for (int g = 0; g < 4; ++g) {
        int na = 0, nb = 0;
        for (int i = 0; i < 16; ++i)
            if (grp[i] == g) (cls[order[i]] == ca[g] ? na : nb)++;
        const int ka = na >= nb ? ca[g] : cb[g];
        const int kb = nb == 0 ? ka : (na >= nb ? cb[g] : ca[g]);
        pr |= (unsigned)reps[ka] << (4 * (2 * g));
        pr |= (unsigned)reps[kb] << (4 * (2 * g + 1));
        int q = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < 16; ++i) {
                const int o = order[i];
                if (grp[i] != g || (pass == 0) != (cls[o] == ka)) continue;
                po |= (unsigned long long)o << (4 * (4 * g + q));
                if (pass == 1) ps |= 1u << (4 * g + q);
                ++q;
            }
        const unsigned gs = (ps >> (4 * g)) & 15u;
        if ((gs & 3u) != 0 || (nb > 0 && !(gs & 8u))) return false;   // not the fixed pattern
    }
    *out = po;
    *rep = pr;
    *selb = ps;
    return true;
}

StepPlan plan_step(const quapi_ctx *c, int n) {
    const int N = c->N, L = c->L;
    StepPlan sp{};
    StepArgs &a = sp.args;
    sp.grow = n < L;
    step_tables(L, n, a);
    a.m_count = ipow_ll(N, a.n_digits);
    sp.split = split_digits(N, a.n_digits);
    a.d_lo = sp.split.d_lo;
    a.d_mid = sp.split.d_mid;
    a.R = sp.split.R;
    a.Q = sp.split.Q;
    a.bank = c->bank;
    a.bank_c = c->bank_f ? (const void *)c->bank_f : (const void *)c->bank;
    if (c->cls_ok && !sp.grow) {
        const BankLayout B{L};
        a.cls_on = 1;
        a.cls_tab = n == L ? B.init(L) : B.lag(L);
        a.clsf_tab = n == L ? B.fin_init(L) : B.fin(L);
        a.cls_self = B.self_int();
        a.cls_selff = B.self_end();
        a.cls_out = c->cls_out;
        a.cls_rep = c->cls_rep;
        a.cls_selb = c->cls_selb;
    }
    return sp;
}

// Step arguments of global step n, checked against the buffers, with the
// full-window factor tables (computed on first use).
quapi_status prepare_step(quapi_ctx *c, int n, bool rho, StepPlan *out) {
    StepPlan sp = plan_step(c, n);
    StepArgs &a = sp.args;
    const int N = c->N;
    const size_t cap = c->lay.a_bytes / c->csize;
    const size_t in_entries = (size_t)a.m_count * (sp.grow ? 1 : N);
    const size_t out_entries = (size_t)a.m_count * N;
    const size_t lds = step_lds_bytes(N, c->prec, rho, sp.grow, a.R, a.Q);
    // host-side launch checks: the grid must tile m exactly and stay in the buffers
    if ((long long)sp.split.grid * a.R * a.Q != a.m_count || in_entries > cap || out_entries > cap ||
        sp.split.grid > c->lay.partial_blocks || lds > (size_t)kLdsLimit || a.R > kBlock)
        return fail(c, QUAPI_ERR_DEVICE, "internal launch check failed at step %d", n);
    if (!sp.grow) {
        const DigitSplit &ms = c->lay.main_split;
        if (ms.R != a.R || ms.Q != a.Q || ms.grid != sp.split.grid)
            return fail(c, QUAPI_ERR_DEVICE, "internal split mismatch at step %d", n);
        const size_t nr = (size_t)N * ms.R, nq = (size_t)N * ms.Q, nh = (size_t)N * ms.grid;
        double2 *t_lo = c->plan, *t_lof = t_lo + nr, *t_mid = t_lof + nr, *t_midf = t_mid + nq;
        double2 *t_hi = t_midf + nq, *t_hif = t_hi + nh;
        if (!c->plan_ready) {
            PlanArgs pa{};
            pa.bank = c->bank;
            pa.N = N;
            pa.d_lo = a.d_lo;
            pa.d_mid = a.d_mid;
            pa.n_digits = a.n_digits;
            pa.R = a.R;
            pa.Q = a.Q;
            pa.grid = sp.split.grid;
            std::memcpy(pa.tab, a.tab, sizeof pa.tab);
            std::memcpy(pa.tabf, a.tabf, sizeof pa.tabf);
            pa.t_lo = t_lo;
            pa.t_lof = t_lof;
            pa.t_mid = t_mid;
            pa.t_midf = t_midf;
            pa.t_hi = t_hi;
            pa.t_hif = t_hif;
            hipError_t e = launch_plan_tables(pa, c->stream);
            if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "plan kernel launch: %s", hipGetErrorString(e));
            c->plan_ready = true;
        }
        a.t_lo = t_lo;
        a.t_lof = t_lof;
        a.t_mid = t_mid;
        a.t_midf = t_midf;
        a.t_hi = t_hi;
        a.t_hif = t_hif;
    }
    a.grid = sp.split.grid;
    *out = sp;
    return QUAPI_OK;
}

// Partial-buffer slots rotate; a slot may be rewritten only after the
// finalize that reads it (on the side stream) is done.
int take_slot(quapi_ctx *c) {
    const int s = c->next_slot;
    c->next_slot = (s + 1) % kSlots;
    return s;
}

quapi_status wait_slot(quapi_ctx *c, int s) {
    if (c->fin_pending[s]) {
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_fin[s], 0));
        c->fin_pending[s] = false;
    }
    return QUAPI_OK;
}

// Order the main stream after every finalize still running on the side stream.
quapi_status join_side(quapi_ctx *c) {
    for (int k = 0; k < kSlots; ++k) {
        quapi_status st = wait_slot(c, k);
        if (st != QUAPI_OK) return st;
    }
    return QUAPI_OK;
}

// Before any kernel or copy that reads every entry of A[cur]: if the last
// step ran in mirror mode, fill the entries above their mirror.
quapi_status ensure_full(quapi_ctx *c) {
    if (!c->half_cur) return QUAPI_OK;
    hipError_t e = launch_mirror_complete(c->N, c->prec, c->A[c->cur], ipow_ll(c->N, c->L), c->stream);
    if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "mirror completion launch: %s", hipGetErrorString(e));
    c->half_cur = false;
    return QUAPI_OK;
}

// Finalize the rho partials of `slots` (in order) on the side stream, after
// the step kernel that wrote them.
quapi_status finalize_side(quapi_ctx *c, const int *slots, int n, int grid) {
    if (c->one_stream) {
        for (int k = 0; k < n; ++k) {
            hipError_t e = launch_rho_finalize(c->N, c->partials[slots[k]], grid, c->pairs, c->sink, c->stream);
            if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "rho finalize launch: %s", hipGetErrorString(e));
        }
        return QUAPI_OK;
    }
    HIP_TRY(c, hipEventRecord(c->ev_step[slots[0]], c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_step[slots[0]], 0));
    for (int k = 0; k < n; ++k) {
        const int sl = slots[k];
        hipEvent_t f0 = nullptr, f1 = nullptr;
        if (c->timing) {
            f0 = take_event(c);
            f1 = take_event(c);
            if (f0) (void)hipEventRecord(f0, c->side);
        }
        hipError_t e = launch_rho_finalize(c->N, c->partials[sl], grid, c->pairs, c->sink, c->side);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "rho finalize launch: %s", hipGetErrorString(e));
        if (c->timing && f0 && f1) {
            (void)hipEventRecord(f1, c->side);
            c->recs.push_back({2, f0, f1, 0, 0});
        }
        HIP_TRY(c, hipEventRecord(c->ev_fin[sl], c->side));
        c->fin_pending[sl] = true;
    }
    return QUAPI_OK;
}

// Enqueue step n (1-based); with rho, also rho(t_n) into the sink's next slot.
// The finalize runs on the side stream, overlapped with the next step.
// The full-window single step runs in mirror mode (half of the entries) for
// tensors above the graph size: smaller steps are bound by their launches,
// and the three mirror launches then cost more than the bytes they save
// (measured crossover: M = 2 at L = 11-12, M = 3 at L = 7, M = 4 at L = 5-6).
bool single_mirror_on(const quapi_ctx *c) {
    return c->mirror != 0 && single_mirror_ok(c->N, c->L, c->lay.main_split) &&
           (c->mirror == 2 || (size_t)ipow_ll(c->N, c->L) > kGraphMaxEntries);
}

// Launch a full-window single step with the arguments of prepare_step: one
// launch, or in mirror mode the launches over the high-digit values below
// their mirror (mode 1) and equal to it (modes 2, 3).  *rows: the rho
// partial rows written.
hipError_t launch_full_step(quapi_ctx *c, bool rho, StepArgs a, int grid, int *rows) {
    if (!single_mirror_on(c)) {
        a.mode = 0;
        *rows = grid;
        return launch_step(c->N, c->prec, rho, false, a, grid, c->stream);
    }
    const Layout &l = c->lay;
    hipError_t e = hipSuccess;
    const bool listed = c->N == 9;      // the diagonal values' items in the tail of mode 1
    if (l.n_canon1 > 0 || (listed && l.n_diag1 > 0)) {
        a.mode = 1;
        a.blk_hi = c->blk1;
        a.n_canon = l.n_canon1;
        a.n_blk = l.n_canon1 + (listed ? l.n_diag1 * l.parts1 : 0);
        a.low_list = c->low1;
        a.n_low = l.n_low1;
        a.parts = listed ? l.parts1 : 1;
        a.q_span = l.span1;
        a.part_base = 0;
        e = launch_step(c->N, c->prec, rho, false, a, grid, c->stream);
    }
    if (e == hipSuccess && l.n_diag1 > 0 && !listed) {
        a.mode = 2;
        a.blk_hi = c->blk1 + l.n_canon1;
        a.n_blk = l.n_diag1 * l.parts1;
        a.parts = l.parts1;
        a.q_span = l.span1;
        a.part_base = l.n_canon1;
        e = launch_step(c->N, c->prec, rho, false, a, grid, c->stream);
    }
    if (e == hipSuccess && l.n_diag1 > 0) {
        a.mode = 3;
        a.blk_hi = c->blk1 + l.n_canon1;
        a.n_blk = l.n_diag1;
        a.parts = 1;
        a.part_base = l.n_canon1 + l.n_diag1 * l.parts1;
        e = launch_step(c->N, c->prec, rho, false, a, grid, c->stream);
    }
    *rows = l.n_canon1 + l.n_diag1 * (l.parts1 + 1);
    return e;
}

quapi_status enqueue_step(quapi_ctx *c, int n, bool rho) {
    StepPlan sp;
    quapi_status st = prepare_step(c, n, rho, &sp);
    if (st != QUAPI_OK) return st;
    const bool half = !sp.grow && single_mirror_on(c);       // reads and writes the kept half only
    if (!half && (st = ensure_full(c)) != QUAPI_OK) return st;
    StepArgs &a = sp.args;
    a.a_in = c->A[c->cur];
    a.a_out = c->A[1 - c->cur];
    int slot = -1;
    if (rho) {
        slot = take_slot(c);
        st = wait_slot(c, slot);
        if (st != QUAPI_OK) return st;
        a.partials = c->partials[slot];
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (e0) (void)hipEventRecord(e0, c->stream);
    }
    int rows = sp.split.grid;
    hipError_t e = sp.grow ? launch_step(c->N, c->prec, rho, true, a, sp.split.grid, c->stream)
                           : launch_full_step(c, rho, a, sp.split.grid, &rows);
    if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "step kernel launch: %s", hipGetErrorString(e));
    if (c->timing && e0 && e1) {
        (void)hipEventRecord(e1, c->stream);
        c->recs.push_back({sp.grow ? 1 : 0, e0, e1, sp.grow ? 0 : 1, sp.grow ? 0 : 1});
    }
    if (rho) {
        st = finalize_side(c, &slot, 1, rows);
        if (st != QUAPI_OK) return st;
    }
    c->cur = 1 - c->cur;
    c->half_cur = half;
    c->step = n;
    return QUAPI_OK;
}

// Filtered step n (1-based) on the context's stream, with rho(t_n) into the
// sink's next slot: the factor-level tables of the step's digits (once for
// the full window, per growth step, per step when driven), the segments of
// the kept input entries, the counting pass, the scan of its keep flags, the
// writing pass, and the new entry count.  Nothing on the host waits.
quapi_status enqueue_filter_step(quapi_ctx *c, int n, bool rho) {
    const int N = c->N, L = c->L;
    StepArgs sa{};
    step_tables(L, n, sa);
    const bool full = n >= L;
    const int nd = sa.n_digits;
    const int n_lv = filter_levels(N, nd);
    if (filter_plan_entries(N, nd) > c->fplan_entries && nd > 0)
        return fail(c, QUAPI_ERR_DEVICE, "internal filter plan check failed at step %d", n);
    const int set = full ? 0 : n;
    if (c->fplan_for != set) {
        FilterPlanArgs pa{};
        pa.bank = c->bank;
        pa.N = N;
        pa.nd = nd;
        pa.n_lv = n_lv;
        std::memcpy(pa.tab, sa.tab, sizeof pa.tab);
        std::memcpy(pa.tabf, sa.tabf, sizeof pa.tabf);
        pa.t = c->fplan;
        hipError_t e = launch_filter_plan(pa, c->stream);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "filter plan launch: %s", hipGetErrorString(e));
        c->fplan_for = set;
    }
    const int in = c->cur, out = 1 - c->cur;
    unsigned long long *ctr = c->fctr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (e0) (void)hipEventRecord(e0, c->stream);
    }
    FilterStepArgs a{};
    a.bank = c->bank;
    a.count_in = ctr + in;
    a.keys_in = c->fkeys[in];
    a.vals_in = c->fvals[in];
    a.keys_out = c->fkeys[out];
    a.vals_out = c->fvals[out];
    a.masks = c->fmask;
    a.bofs = c->fbofs;
    a.partials = c->fpart;
    a.t = c->fplan;
    a.capacity = c->fcap;
    a.stride_new = (unsigned long long)ipow_ll(N, full ? L - 1 : n);
    a.theta = c->theta;
    a.full = full ? 1 : 0;
    a.n_lv = n_lv;
    a.old_tab = sa.old_tab;
    a.oldf_tab = sa.oldf_tab;
    hipError_t e = launch_filter_step(N, c->prec, a, true, rho, c->stream);
    if (e == hipSuccess) e = launch_filter_offsets(N, c->fbofs, c->fcap, ctr + out, (int *)(ctr + 2), c->stream);
    if (e == hipSuccess) e = launch_filter_step(N, c->prec, a, false, false, c->stream);
    if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "filtered step launch: %s", hipGetErrorString(e));
    if (c->timing && e0 && e1) {
        (void)hipEventRecord(e1, c->stream);
        c->recs.push_back({full ? 0 : 1, e0, e1, full ? 1 : 0, full ? 1 : 0});
    }
    if (rho) {
        e = launch_rho_finalize(N, c->fpart, kFilterStepBlocks, c->pairs, c->sink, c->stream);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "rho finalize launch: %s", hipGetErrorString(e));
    }
    c->cur = out;
    c->step = n;
    return QUAPI_OK;
}

// The overflow flag of a filtered context (waits for its stream).
quapi_status filter_overflow(quapi_ctx *c, int *overflow) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(overflow, c->fctr + 2, sizeof(int), hipMemcpyDeviceToHost));
    return QUAPI_OK;
}

// Arguments of a fused launch of steps n, n+1 (n > L); the four factor-table
// sets are computed on first use.
quapi_status prepare_step2(quapi_ctx *c, bool rho, Step2Args *out) {
    const int N = c->N, L = c->L;
    const BankLayout B{L};
    const DigitSplit &sp = c->lay.split2;
    const int nd = L - 2;
    Step2Args a{};
    a.bank = c->bank;
    a.m_count = ipow_ll(N, nd);
    a.R = sp.R;
    a.Q = sp.Q;
    a.grid = sp.grid;
    const size_t cap = c->lay.a_bytes / c->csize;
    const size_t lds = step2_lds_bytes(c->prec, rho, a.R, a.Q);
    if ((long long)a.grid * a.R * a.Q != a.m_count || (size_t)a.m_count * N * N > cap ||
        a.grid > c->lay.partial_blocks || lds > (size_t)kLdsLimit || a.R > kBlock)
        return fail(c, QUAPI_ERR_DEVICE, "internal fused launch check failed");
    // sets 0, 1, 2, 3 = interior n, interior n+1, final n, final n+1; each [N][R] [N][Q] [N][grid]
    const size_t per = (size_t)N * (sp.R + sp.Q + sp.grid);
    for (int k = 0; k < 4; ++k) {
        double2 *base = c->plan2 + per * k;
        a.t_lo[k] = base;
        a.t_mid[k] = base + (size_t)N * sp.R;
        a.t_hi[k] = base + (size_t)N * (sp.R + sp.Q);
    }
    if (!c->plan2_ready) {
        // digit j of m is point n-L+2+j: lag L-2-j from n, L-1-j from n+1
        for (int step = 0; step < 2; ++step) {
            PlanArgs pa{};
            pa.bank = c->bank;
            pa.N = N;
            pa.d_lo = sp.d_lo;
            pa.d_mid = sp.d_mid;
            pa.n_digits = nd;
            pa.R = sp.R;
            pa.Q = sp.Q;
            pa.grid = sp.grid;
            for (int j = 0; j < nd; ++j) {
                const int lag = (step == 0 ? L - 2 : L - 1) - j;
                pa.tab[j] = (int16_t)(lag == 1 ? B.k_lag1() : B.lag(lag));
                pa.tabf[j] = (int16_t)(lag == 1 ? B.k_fin1() : B.fin(lag));
            }
            pa.t_lo = (double2 *)a.t_lo[step];
            pa.t_lof = (double2 *)a.t_lo[step + 2];
            pa.t_mid = (double2 *)a.t_mid[step];
            pa.t_midf = (double2 *)a.t_mid[step + 2];
            pa.t_hi = (double2 *)a.t_hi[step];
            pa.t_hif = (double2 *)a.t_hi[step + 2];
            hipError_t e = launch_plan_tables(pa, c->stream);
            if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "plan kernel launch: %s", hipGetErrorString(e));
        }
        CoefArgs ca{};
        ca.bank = c->bank;
        ca.old_tab = B.old_main();
        ca.oldf_tab = B.oldf_main();
        ca.an_tab = L - 1 == 1 ? B.k_lag1() : B.lag(L - 1);    // point n-L+1 seen from n
        ca.anf_tab = L - 1 == 1 ? B.k_fin1() : B.fin(L - 1);
        ca.d_tab = B.k_lag1();                                // point n seen from n+1
        ca.df_tab = B.k_fin1();
        ca.prec = c->prec;
        ca.out = c->coef;
        hipError_t e = launch_step2_coef(ca, c->stream);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "coefficient kernel launch: %s", hipGetErrorString(e));
        c->plan2_ready = true;
    }
    a.coef = c->coef;
    *out = a;
    return QUAPI_OK;
}

// The two-step kernel runs in mirror mode above the graph size, as the
// single step does (the same launch-count trade-off).
bool pair_mirror_on(const quapi_ctx *c) {
    return c->mirror != 0 && fused_ok(c->N, c->L) &&
           (c->mirror == 2 || (size_t)ipow_ll(c->N, c->L) > kGraphMaxEntries);
}

// Launch the two-step kernel with the arguments of prepare_step2: every block
// (mode 0), or in mirror mode the launches over the high-digit values below
// their mirror (mode 1) and equal to it (modes 2, 3).  *rows: the rho
// partial rows written.
hipError_t launch_step2_modes(quapi_ctx *c, bool rho, Step2Args a, int *rows) {
    if (!pair_mirror_on(c)) {
        a.mode = 0;
        *rows = a.grid;
        return launch_step2(c->prec, rho, a, c->stream);
    }
    const Layout &l = c->lay;
    hipError_t e = hipSuccess;
    if (l.n_canon2 + l.n_diag2 > 0) {
        // the canonical blocks, then the listed items of the diagonal values
        a.mode = 1;
        a.blk_hi = c->blk2;
        a.n_canon = l.n_canon2;
        a.low_list = c->low2;
        a.n_low = l.n_low2;
        a.n_blk = l.n_canon2 + l.n_diag2 * l.parts2;
        a.parts = l.parts2;
        a.q_span = l.span2;
        a.part_base = 0;
        e = launch_step2(c->prec, rho, a, c->stream);
    }
    if (e == hipSuccess && l.n_diag2 > 0) {
        a.mode = 3;
        a.blk_hi = c->blk2 + l.n_canon2;
        a.n_blk = l.n_diag2;
        a.parts = 1;
        a.part_base = l.n_canon2 + l.n_diag2 * l.parts2;
        e = launch_step2(c->prec, rho, a, c->stream);
    }
    *rows = l.n_canon2 + l.n_diag2 * (l.parts2 + 1);
    return e;
}

// Enqueue the fused steps n, n+1 (n > L); rho of the selected ones goes to
// the sink in step order.
quapi_status enqueue_step2(quapi_ctx *c, int n, bool sel_n, bool sel_n1) {
    const bool half = pair_mirror_on(c);      // reads and writes the kept half only
    if (!half)
        if (quapi_status fs = ensure_full(c); fs != QUAPI_OK) return fs;
    const bool rho = sel_n || sel_n1;
    Step2Args a;
    quapi_status st = prepare_step2(c, rho, &a);
    if (st != QUAPI_OK) return st;
    a.a_in = c->A[c->cur];
    a.a_out = c->A[1 - c->cur];
    int slots[2] = {-1, -1};
    if (rho) {
        for (int k = 0; k < 2; ++k) {
            slots[k] = take_slot(c);
            st = wait_slot(c, slots[k]);
            if (st != QUAPI_OK) return st;
            a.partials[k] = c->partials[slots[k]];
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (e0) (void)hipEventRecord(e0, c->stream);
    }
    int rows = 0;
    hipError_t e = launch_step2_modes(c, rho, a, &rows);
    if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "fused step launch: %s", hipGetErrorString(e));
    if (c->timing && e0 && e1) {
        (void)hipEventRecord(e1, c->stream);
        c->recs.push_back({0, e0, e1, 2, 2});
    }
    if (rho) {
        int fin[2], nf = 0;
        if (sel_n) fin[nf++] = slots[0];
        if (sel_n1) fin[nf++] = slots[1];
        st = finalize_side(c, fin, nf, rows);
        if (st != QUAPI_OK) return st;
    }
    c->cur = 1 - c->cur;
    c->half_cur = half;
    c->step = n + 1;
    return QUAPI_OK;
}

// Arguments of a launch of steps n, n+1, n+2 (n > L); the six factor-table
// sets and the coefficients are computed on first use.
quapi_status prepare_step3(quapi_ctx *c, bool rho, Step3Args *out) {
    const int N = c->N, L = c->L;
    const BankLayout B{L};
    const DigitSplit &sp = c->lay.split3;
    const int nd = L - 3;
    Step3Args a{};
    a.m_count = ipow_ll(N, nd);
    a.R = sp.R;
    a.Q = sp.Q;
    a.grid = sp.grid;
    const size_t cap = c->lay.a_bytes / c->csize;
    const size_t lds = step3_lds_bytes(c->prec, rho, a.R, a.Q);
    if ((long long)a.grid * a.R * a.Q != a.m_count || (size_t)a.m_count * N * N * N > cap ||
        a.grid > c->lay.partial_blocks || lds > (size_t)kLdsLimitStep3 || a.R > kBlock)
        return fail(c, QUAPI_ERR_DEVICE, "internal three-step launch check failed");
    const size_t per = (size_t)N * (sp.R + sp.Q + sp.grid);
    for (int k = 0; k < 6; ++k) {
        double2 *base = c->plan3 + per * k;
        a.t_lo[k] = base;
        a.t_mid[k] = base + (size_t)N * sp.R;
        a.t_hi[k] = base + (size_t)N * (sp.R + sp.Q);
    }
    if (!c->plan3_ready) {
        // digit j of m is point n-L+3+j: lag L-3-j+s from step n+s
        for (int step = 0; step < 3; ++step) {
            PlanArgs pa{};
            pa.bank = c->bank;
            pa.N = N;
            pa.d_lo = sp.d_lo;
            pa.d_mid = sp.d_mid;
            pa.n_digits = nd;
            pa.R = sp.R;
            pa.Q = sp.Q;
            pa.grid = sp.grid;
            for (int j = 0; j < nd; ++j) {
                const int lag = L - 3 - j + step;
                pa.tab[j] = (int16_t)(lag == 1 ? B.k_lag1() : B.lag(lag));
                pa.tabf[j] = (int16_t)(lag == 1 ? B.k_fin1() : B.fin(lag));
            }
            pa.t_lo = (double2 *)a.t_lo[step];
            pa.t_lof = (double2 *)a.t_lo[step + 3];
            pa.t_mid = (double2 *)a.t_mid[step];
            pa.t_midf = (double2 *)a.t_mid[step + 3];
            pa.t_hi = (double2 *)a.t_hi[step];
            pa.t_hif = (double2 *)a.t_hi[step + 3];
            hipError_t e = launch_plan_tables(pa, c->stream);
            if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "plan kernel launch: %s", hipGetErrorString(e));
        }
        Coef3Args ca{};
        ca.bank = c->bank;
        ca.old_tab = B.old_main();
        ca.oldf_tab = B.oldf_main();
        ca.an_tab = B.lag(L - 1);                               // point n-L+1 seen from n
        ca.anf_tab = B.fin(L - 1);
        ca.f_tab = L - 2 == 1 ? B.k_lag1() : B.lag(L - 2);      // point n-L+2 seen from n
        ca.ff_tab = L - 2 == 1 ? B.k_fin1() : B.fin(L - 2);
        ca.g_tab = B.k_lag1();                                  // point n seen from n+1
        ca.gf_tab = B.k_fin1();
        ca.h_tab = B.lag(L - 1);                                // point n-L+2 seen from n+1
        ca.hf_tab = B.fin(L - 1);
        ca.p_tab = B.k_lag1();                                  // point n+1 seen from n+2
        ca.pf_tab = B.k_fin1();
        ca.q_tab = B.lag(2);                                    // point n seen from n+2
        ca.qf_tab = B.fin(2);
        ca.prec = c->prec;
        ca.out = c->coef3;
        hipError_t e = launch_step3_coef(ca, c->stream);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "coefficient kernel launch: %s", hipGetErrorString(e));
        c->plan3_ready = true;
    }
    a.coef = c->coef3;
    *out = a;
    return QUAPI_OK;
}

// Launch the three-step kernel with the arguments of prepare_step3: every
// block (mode 0), or in mirror mode the launches over the high-digit values
// below their mirror (mode 1) and equal to it (modes 2 and 3).  *rows: the
// rho partial rows written.
// concurrent: modes 2 and 3 on the aux stream (forked from and joined back
// into the context's stream) while mode 1 runs; not inside a graph capture.
hipError_t launch_step3_modes(quapi_ctx *c, bool rho, Step3Args a, int *rows, bool concurrent) {
    if (c->mirror == 0) {
        a.mode = 0;
        *rows = a.grid;
        return launch_step3(c->prec, rho, a, c->stream);
    }
    const Layout &l = c->lay;
    hipError_t e = hipSuccess;
    const bool fork = concurrent && l.n_diag3 > 0 && l.n_canon3 > 0;
    hipStream_t small = fork ? c->aux : c->stream;
    auto mode1 = [&]() {
        if (e == hipSuccess && l.n_canon3 + l.n_diag3 > 0) {
            a.mode = 1;
            a.blk_hi = c->blk3;
            a.n_canon = l.n_canon3;
            a.low_list = c->low3;
            a.n_low = l.n_low3;
            a.n_blk = l.n_canon3 + l.n_diag3 * l.parts3;
            a.parts = l.parts3;
            a.q_span = l.span3;
            a.part_base = 0;
            e = launch_step3(c->prec, rho, a, c->stream);
        }
    };
    if (fork) {
        e = hipEventRecord(c->ev_fork, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->ev_fork, 0);
    } else {
        mode1();                                  // one stream: the large launch first
    }
    if (e == hipSuccess && l.n_diag3 > 0) {
        a.mode = 3;
        a.blk_hi = c->blk3 + l.n_canon3;
        a.n_blk = l.n_diag3;
        a.parts = 1;
        a.part_base = l.n_canon3 + l.n_diag3 * l.parts3;
        e = launch_step3(c->prec, rho, a, small);
    }
    if (fork) {
        if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->aux);
        mode1();
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_join, 0);
    }
    *rows = l.n_canon3 + l.n_diag3 * (l.parts3 + 1);
    return e;
}

// Enqueue the steps n, n+1, n+2 (n > L) as one launch (three in mirror mode);
// rho of the selected ones goes to the sink in step order.
quapi_status enqueue_step3(quapi_ctx *c, int n, const bool *selk) {
    const bool rho = selk[0] || selk[1] || selk[2];
    Step3Args a;
    quapi_status st = prepare_step3(c, rho, &a);
    if (st != QUAPI_OK) return st;
    if (c->mirror == 0) {                    // mode 0 reads every entry
        st = ensure_full(c);
        if (st != QUAPI_OK) return st;
    }
    a.a_in = c->A[c->cur];
    a.a_out = c->A[1 - c->cur];
    int slots[3] = {-1, -1, -1};
    if (rho) {
        for (int k = 0; k < 3; ++k) {
            slots[k] = take_slot(c);
            st = wait_slot(c, slots[k]);
            if (st != QUAPI_OK) return st;
            a.partials[k] = c->partials[slots[k]];
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (e0) (void)hipEventRecord(e0, c->stream);
    }
    const bool concurrent = step3_concurrent((size_t)ipow_ll(c->N, c->L), c->prec) && c->aux != nullptr;
    int rows = 0;
    hipError_t e = launch_step3_modes(c, rho, a, &rows, concurrent);
    if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "three-step launch: %s", hipGetErrorString(e));
    if (c->timing && e0 && e1) {
        (void)hipEventRecord(e1, c->stream);
        c->recs.push_back({0, e0, e1, 3, 3});
    }
    if (rho) {
        int fin[3], nf = 0;
        for (int k = 0; k < 3; ++k)
            if (selk[k]) fin[nf++] = slots[k];
        st = finalize_side(c, fin, nf, rows);
        if (st != QUAPI_OK) return st;
    }
    c->cur = 1 - c->cur;
    c->half_cur = c->mirror != 0;
    c->step = n + 2;
    return QUAPI_OK;
}

// Capture full-window steps into an executable graph whose node arguments
// never change (the step tables are the same for all n > L, and rho goes
// through the sink); finalizes run on the same stream.
//   width 1: two single steps A[0] -> A[1] -> A[0]
//   width 2: one two-step launch A[par] -> A[1 - par]
//   width 3: one three-step launch A[par] -> A[1 - par]
quapi_status build_graph(quapi_ctx *c, bool rho, int width, int par, hipGraphExec_t *out) {
    StepPlan sp{};
    Step2Args a2{};
    Step3Args a3{};
    quapi_status st = width == 3 ? prepare_step3(c, rho, &a3)
                      : width == 2 ? prepare_step2(c, rho, &a2)
                                   : prepare_step(c, c->L + 1, rho, &sp);
    if (st != QUAPI_OK) return st;
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (width == 3) {
        a3.a_in = c->A[par];
        a3.a_out = c->A[1 - par];
        for (int k = 0; k < 3; ++k) a3.partials[k] = c->partials[k];
        int rows = 0;
        e = launch_step3_modes(c, rho, a3, &rows, false);
        for (int k = 0; k < 3 && rho && e == hipSuccess; ++k)
            e = launch_rho_finalize(c->N, c->partials[k], rows, c->pairs, c->sink, c->stream);
    } else if (width == 2) {
        a2.a_in = c->A[par];
        a2.a_out = c->A[1 - par];
        a2.partials[0] = c->partials[0];
        a2.partials[1] = c->partials[1];
        int rows = 0;
        e = launch_step2_modes(c, rho, a2, &rows);
        for (int k = 0; k < 2 && rho && e == hipSuccess; ++k)
            e = launch_rho_finalize(c->N, c->partials[k], rows, c->pairs, c->sink, c->stream);
    } else {
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
            StepArgs a = sp.args;
            a.a_in = c->A[k];
            a.a_out = c->A[1 - k];
            a.partials = c->partials[k];
            int rows = 0;
            e = launch_full_step(c, rho, a, sp.split.grid, &rows);
            if (e == hipSuccess && rho)
                e = launch_rho_finalize(c->N, c->partials[k], rows, c->pairs, c->sink, c->stream);
        }
    }
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, QUAPI_ERR_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(c, QUAPI_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return QUAPI_OK;
}

quapi_status check_selection(quapi_ctx *c, int n_steps, const int *sel, int n_sel, int *n_out) {
    if (n_steps < 0) return fail(c, QUAPI_ERR_INVALID, "n_steps must be >= 0");
    if ((long long)c->step + n_steps > std::numeric_limits<int>::max())
        return fail(c, QUAPI_ERR_INVALID, "step counter would overflow");
    if (!sel) {
        *n_out = n_steps;
        return QUAPI_OK;
    }
    if (n_sel < 0) return fail(c, QUAPI_ERR_INVALID, "n_sel must be >= 0");
    int prev = -1;
    for (int i = 0; i < n_sel; ++i) {
        const int k = sel[i];
        if (k <= prev) return fail(c, QUAPI_ERR_INVALID, "sel must be strictly increasing");
        if (!(k == 0 || (k > c->step && k <= c->step + n_steps)))
            return fail(c, QUAPI_ERR_INVALID, "sel[%d] = %d is neither 0 nor in (%d, %d]", i, k, c->step,
                        c->step + n_steps);
        prev = k;
    }
    *n_out = n_sel;
    return QUAPI_OK;
}

// ---------------------------------------------------------- persistent path
// Small tensors (N^L <= 2^14) run every step of a call in one launch of the
// persistent kernel, one block per context: a step costs a block barrier
// instead of three launches.  Contexts that pin a launch width, force mirror
// mode at every size, or are driven use the multi-block kernels.
bool small_on(const quapi_ctx *c) {
    return c->small != 0 && c->n_H == 0 && !c->fuse_pinned && c->mirror != 2;
}

SmallCtxArgs small_args(const quapi_ctx *c, int n_steps, int rho_mode, double2 *rho_out) {
    SmallCtxArgs s{};
    s.bank = c->bank;
    s.a0 = c->A[c->cur];
    s.a1 = c->A[1 - c->cur];
    s.rho_out = rho_out;
    s.L = c->L;
    s.step0 = c->step;
    s.n_steps = n_steps;
    s.rho_mode = rho_mode;
    return s;
}

// After a persistent launch of n steps: the tensor is in A[cur] after an
// even number of steps, in the other buffer after an odd one.
void small_advance(quapi_ctx *c, int n) {
    c->step += n;
    if (n & 1) c->cur = 1 - c->cur;
}

// The persistent path of propagate_impl: one launch per run of consecutive
// selected steps and per stretch of steps up to an isolated selected step
// (one launch for 'allPoints', 'justFinalPoint' or no selection); the
// blocking call also cuts runs at the staging buffer's size.
quapi_status propagate_small(quapi_ctx *c, int n_steps, const int *sel, int n_sel, double2 *dev_out,
                             double *host_out) {
    const int N = c->N;
    int si = 0, written = 0, staged = 0;
    if (sel && si < n_sel && sel[si] == 0) {  // rho(t_0) = rho0
        if (dev_out)
            HIP_TRY(c, hipMemcpyAsync(dev_out, c->rho0_d, (size_t)N * 16, hipMemcpyDeviceToDevice, c->stream));
        else
            std::memcpy(host_out, c->rho0_h.data(), (size_t)N * 16);
        ++si;
        ++written;
    }
    quapi_status st = join_side(c);
    if (st == QUAPI_OK) st = ensure_full(c);
    if (st != QUAPI_OK) return st;
    auto flush = [&]() -> quapi_status {
        if (!staged) return QUAPI_OK;
        HIP_TRY(c, hipMemcpyAsync(host_out + (size_t)2 * N * (written - staged), c->stage,
                                  (size_t)staged * N * 16, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        staged = 0;
        return QUAPI_OK;
    };
    const int last = c->step + n_steps;
    while (c->step < last) {
        int k, mode;
        if (!sel) {
            k = last - c->step;
            mode = 1;
        } else if (si < n_sel && sel[si] == c->step + 1) {
            // a run of consecutive selected steps: rho at every one
            k = 1;
            while (si + k < n_sel && sel[si + k] == c->step + 1 + k) ++k;
            mode = 1;
        } else if (si < n_sel) {
            k = sel[si] - c->step;    // up to the next selected step
            mode = 2;
        } else {
            k = last - c->step;
            mode = 0;
        }
        if (!dev_out && mode != 0) {
            if (staged == kRhoStage && (st = flush()) != QUAPI_OK) return st;
            if (mode == 1) k = std::min(k, kRhoStage - staged);
        }
        double2 *out = dev_out ? dev_out + (size_t)written * N : c->stage + (size_t)staged * N;
        SmallBatchArgs b;
        b.c[0] = small_args(c, k, mode, out);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            e0 = take_event(c);
            e1 = take_event(c);
            if (e0) (void)hipEventRecord(e0, c->stream);
        }
        hipError_t e = launch_small(N, c->prec, c->small == 1, b, 1, c->L, c->stream);
        if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "persistent step launch: %s", hipGetErrorString(e));
        if (c->timing && e0 && e1) {
            (void)hipEventRecord(e1, c->stream);
            // full-window steps of the launch (n >= L); a launch of growth steps only counts as growth
            const int full = std::max(0, c->step + k - std::max(c->step, c->L - 1));
            c->recs.push_back({full > 0 ? 0 : 1, e0, e1, full, 0});
        }
        const int outs = mode == 1 ? k : mode == 2 ? 1 : 0;
        small_advance(c, k);
        written += outs;
        if (!dev_out) staged += outs;
        if (sel) si += outs;
    }
    if (!dev_out) {
        st = flush();
        if (st != QUAPI_OK) return st;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return QUAPI_OK;
}

// Shared driver of the blocking and asynchronous calls.  dev_out: device
// output of n_out slots (async), or NULL to stage and copy into host_out.
//
// Dispatch per step n: growth steps and the first full-window step run one
// launch each; later full-window steps run in fused groups of F = c->fuse
// steps when N = 4 (one pass per group, groups fixed by the global step
// number), else singly; small tensors replay captured graphs.  A call that
// ends inside a group runs that group's steps singly, or, two steps into a
// three-step group, as one two-step launch.  In mirror mode the
// tensor may hold only its kept half between launches (c->half_cur); a
// launch that reads every entry fills the other half first.
quapi_status propagate_impl(quapi_ctx *c, int n_steps, const int *sel, int n_sel, double2 *dev_out,
                            double *host_out) {
    int n_out = 0;
    quapi_status st = check_selection(c, n_steps, sel, n_sel, &n_out);
    if (st != QUAPI_OK) return st;
    if (n_out > 0 && !dev_out && !host_out) return fail(c, QUAPI_ERR_INVALID, "rho_out is NULL");
    if (small_on(c)) return propagate_small(c, n_steps, sel, n_sel, dev_out, host_out);
    const int N = c->N, L = c->L;
    int si = 0;          // next selection entry
    int written = 0;     // outputs delivered so far
    int staged = 0;      // outputs in the staging buffer (blocking call)
    auto flush = [&]() -> quapi_status {
        if (!staged) return QUAPI_OK;
        quapi_status js = join_side(c);
        if (js != QUAPI_OK) return js;
        HIP_TRY(c, hipMemcpyAsync(host_out + (size_t)2 * N * (written - staged), c->stage,
                                  (size_t)staged * N * 16, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        staged = 0;
        HIP_TRY(c, launch_set_sink(c->sink, c->stage, c->stream));
        return QUAPI_OK;
    };
    auto is_sel = [&](int k, int from) { return !sel || (from < n_sel && sel[from] == k); };
    if (sel && si < n_sel && sel[si] == 0) {  // rho(t_0) = rho0
        if (dev_out)
            HIP_TRY(c, hipMemcpyAsync(dev_out, c->rho0_d, (size_t)N * 16, hipMemcpyDeviceToDevice, c->stream));
        else
            std::memcpy(host_out, c->rho0_h.data(), (size_t)N * 16);
        ++si;
        ++written;
    }
    // finalized rho values land at sink->base + k*N in step order
    HIP_TRY(c, launch_set_sink(c->sink, dev_out ? dev_out + (size_t)written * N : c->stage, c->stream));
    const size_t entries = (size_t)ipow_ll(N, L);
    const bool fused = c->fuse == 2;
    const bool graphs = !c->timing && !c->graph_failed && entries <= kGraphMaxEntries && c->n_H == 0;
    const int first = c->step + 1, last = c->step + n_steps;
    for (int n = first; n <= last; ++n) {
        const bool s0 = is_sel(n, si);
        // Three full-window steps n, n+1, n+2 at groups fixed by the global
        // step number -- (L+1, L+2, L+3), (L+4, ..), ... -- as for pairs below.
        if (c->fuse == 3 && n > L && n + 2 <= last && (n - L - 1) % 3 == 0) {
            bool selk[3];
            int nsel = 0;
            for (int k = 0; k < 3; ++k) {
                selk[k] = is_sel(n + k, si + nsel);
                nsel += selk[k] ? 1 : 0;
            }
            if (!dev_out && staged + nsel > kRhoStage) {
                st = flush();
                if (st != QUAPI_OK) return st;
            }
            bool done = false;
            if (graphs && selk[0] == selk[1] && selk[1] == selk[2]) {
                hipGraphExec_t &gx = c->graph3[s0 ? 1 : 0][c->cur];
                if (!gx && build_graph(c, s0, 3, c->cur, &gx) != QUAPI_OK) {
                    c->graph_failed = true;   // stay on direct launches
                } else {
                    st = join_side(c);        // the graph reuses partial buffers 0, 1 and 2
                    if (st == QUAPI_OK && c->mirror == 0) st = ensure_full(c);
                    if (st != QUAPI_OK) return st;
                    HIP_TRY(c, hipGraphLaunch(gx, c->stream));
                    c->cur = 1 - c->cur;
                    c->half_cur = c->mirror != 0;
                    c->step = n + 2;
                    done = true;
                }
            }
            if (!done) {
                st = enqueue_step3(c, n, selk);
                if (st != QUAPI_OK) return st;
            }
            si += sel ? nsel : 0;
            written += nsel;
            if (!dev_out) staged += nsel;
            n += 2;
            continue;
        }
        // Two full-window steps n, n+1.  Pairs are fixed by the global step
        // number -- (L+1, L+2), (L+3, L+4), ... -- so a run gives the same bits
        // however it is split into calls, as long as no call ends inside a pair.
        // A call that ends two steps into a three-step group runs those two
        // steps as one two-step launch.
        const bool pair_tail = c->fuse == 3 && n > L && n + 1 == last && (n - L - 1) % 3 == 0;
        if ((c->fuse != 3 && n > L && n < last && (n - L - 1) % 2 == 0) || pair_tail) {
            const bool s1 = is_sel(n + 1, si + (s0 ? 1 : 0));
            const int nsel = (s0 ? 1 : 0) + (s1 ? 1 : 0);
            if (!dev_out && staged + nsel > kRhoStage) {
                st = flush();
                if (st != QUAPI_OK) return st;
            }
            bool done = false;
            if (graphs && !pair_tail && s0 == s1 && (fused || c->cur == 0)) {
                hipGraphExec_t &gx = fused ? c->graph2[s0 ? 1 : 0][c->cur] : c->graph1[s0 ? 1 : 0];
                if (!gx && build_graph(c, s0, fused ? 2 : 1, c->cur, &gx) != QUAPI_OK) {
                    c->graph_failed = true;   // stay on direct launches
                } else {
                    st = join_side(c);        // the graph reuses partial buffers 0 and 1
                    const bool half = fused ? pair_mirror_on(c) : single_mirror_on(c);
                    if (st == QUAPI_OK && !half) st = ensure_full(c);
                    if (st != QUAPI_OK) return st;
                    HIP_TRY(c, hipGraphLaunch(gx, c->stream));
                    c->half_cur = half;
                    if (fused) c->cur = 1 - c->cur;
                    c->step = n + 1;
                    done = true;
                }
            }
            if (!done && (fused || pair_tail)) {
                st = enqueue_step2(c, n, s0, s1);
                if (st != QUAPI_OK) return st;
                done = true;
            }
            if (done) {
                si += sel ? nsel : 0;
                written += nsel;
                if (!dev_out) staged += nsel;
                ++n;
                continue;
            }
        }
        if (!dev_out && s0 && staged + 1 > kRhoStage) {
            st = flush();
            if (st != QUAPI_OK) return st;
        }
        if (c->n_H > 0) {
            // driven: the propagator tables of step n, and the plan tables
            // built from them, before the step
            TablesArgs ta = c->drive_ta;
            ta.U_given = c->Ut_d + (size_t)std::min(n - 1, c->n_H - 1) * c->M * c->M;
            ta.k_only = 1;
            hipError_t e = launch_tables(ta, c->stream);
            if (e != hipSuccess) return fail(c, QUAPI_ERR_DEVICE, "tables launch: %s", hipGetErrorString(e));
            c->plan_ready = false;
            c->fplan_for = -1;
        }
        st = c->filtered ? enqueue_filter_step(c, n, s0) : enqueue_step(c, n, s0);
        if (st != QUAPI_OK) return st;
        if (s0) {
            if (sel) ++si;
            ++written;
            if (!dev_out) ++staged;
        }
    }
    st = join_side(c);
    if (st != QUAPI_OK) return st;
    if (!dev_out) {
        st = flush();
        if (st != QUAPI_OK) return st;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->filtered) {
            int overflow = 0;
            st = filter_overflow(c, &overflow);
            if (st != QUAPI_OK) return st;
            if (overflow)
                return fail(c, QUAPI_ERR_NOMEM, "the filtered tensor outgrew its capacity of %zu entries by step %d",
                            c->fcap, c->step);
        }
    }
    return QUAPI_OK;
}

void release(quapi_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (int k = 0; k < kSlots; ++k) {
        if (c->ev_step[k]) (void)hipEventDestroy(c->ev_step[k]);
        if (c->ev_fin[k]) (void)hipEventDestroy(c->ev_fin[k]);
    }
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (auto &g : c->graph1)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto &row : c->graph2)
        for (auto &g : row)
            if (g) (void)hipGraphExecDestroy(g);
    for (auto &row : c->graph3)
        for (auto &g : row)
            if (g) (void)hipGraphExecDestroy(g);
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// quapi_create, and with one_stream the context of quapi_propagate_static:
// the caller's stream only (no side or aux streams, no events, no graphs) and
// the given workspace (never a device allocation).
// fcap > 0: a filtered context (quapi_create_filtered) with threshold theta.
quapi_status create_ctx(const quapi_params *p, void *hip_stream, void *workspace, size_t ws_bytes, bool one_stream,
                        quapi_ctx **out, double theta = -1.0, size_t fcap = 0) {
    if (!out) return fail(nullptr, QUAPI_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const bool filtered = fcap > 0;
    const std::string msg = validate(p, filtered ? kFilterMaxLog2 : kDenseMaxLog2);
    if (!msg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", msg.c_str());
    const int M = p->M, N = M * M, L = p->dk_max;
    std::vector<double> pa, ph;
    std::vector<int> pseg;
    plan_panels(*p, (L + 1) * p->dt, pa, ph, pseg);
    const Layout lay = make_layout(*p, (int)pa.size(), fcap);
    if (workspace) {
        if (ws_bytes < lay.total)
            return fail(nullptr, QUAPI_ERR_INVALID, "workspace of %zu bytes is smaller than the footprint %zu",
                        ws_bytes, lay.total);
        if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
            return fail(nullptr, QUAPI_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    } else if (const char *cap = std::getenv("QUAPI_FAKE_HBM_BYTES")) {
        const unsigned long long capb = std::strtoull(cap, nullptr, 10);
        if (lay.total > capb)
            return fail(nullptr, QUAPI_ERR_NOMEM,
                        "footprint %zu bytes exceeds the device memory cap %llu (did not fit on the GPU)",
                        lay.total, capb);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, QUAPI_ERR_DEVICE, "no HIP device available");

    quapi_ctx *c = new quapi_ctx();
    c->M = M;
    c->N = N;
    c->L = L;
    c->prec = p->dtype;
    c->csize = p->dtype == QUAPI_C128 ? 16 : 8;
    c->dt = p->dt;
    c->lay = lay;
    c->one_stream = one_stream;
    c->graph_failed = one_stream;
    if (hip_stream || one_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, QUAPI_ERR_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    bool side_ok = one_stream ||
                   (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
                    hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
                    hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess);
    for (int k = 0; k < kSlots && side_ok && !one_stream; ++k)
        side_ok = hipEventCreateWithFlags(&c->ev_step[k], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_fin[k], hipEventDisableTiming) == hipSuccess;
    if (!side_ok) {
        release(c);
        return fail(nullptr, QUAPI_ERR_DEVICE, "side stream / event creation failed");
    }
    if (workspace) {
        c->ws = (char *)workspace;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            release(c);
            return fail(nullptr, QUAPI_ERR_DEVICE, "hipMemGetInfo failed");
        }
        if (lay.total > free_b) {
            release(c);
            return fail(nullptr, QUAPI_ERR_NOMEM,
                        "footprint %zu bytes exceeds free device memory %zu (did not fit on the GPU)",
                        lay.total, free_b);
        }
        if (hipMalloc((void **)&c->ws, lay.total) != hipSuccess) {
            c->ws = nullptr;
            release(c);
            return fail(nullptr, QUAPI_ERR_NOMEM, "hipMalloc of %zu bytes failed", lay.total);
        }
        c->own_ws = true;
    }
    char *w = c->ws;
    c->A[0] = w + lay.off_a0;
    c->A[1] = w + lay.off_a1;
    c->bank = (double2 *)(w + lay.off_bank);
    c->bank_f = c->prec == kPrecC64 ? (float2 *)(w + lay.off_bankf) : nullptr;
    c->g = (double2 *)(w + lay.off_g);
    c->eta = (double2 *)(w + lay.off_eta);
    c->U = (double2 *)(w + lay.off_U);
    c->rho0_d = (double2 *)(w + lay.off_rho0);
    for (int k = 0; k < kSlots; ++k)
        c->partials[k] = (double2 *)(w + lay.off_partials) + (size_t)k * lay.partial_blocks * N;
    c->plan2 = (double2 *)(w + lay.off_plan2);
    c->plan3 = (double2 *)(w + lay.off_plan3);
    c->coef3 = w + lay.off_coef3;
    c->blk3 = (int *)(w + lay.off_blk3);
    c->low3 = (int *)(w + lay.off_low3);
    c->blk2 = (int *)(w + lay.off_blk2);
    c->low2 = (int *)(w + lay.off_low2);
    c->blk1 = (int *)(w + lay.off_blk1);
    c->low1 = (int *)(w + lay.off_low1);
    c->n_H = p->n_H;
    c->Ht_d = (const double2 *)(w + lay.off_Ht);
    c->Ut_d = (double2 *)(w + lay.off_Ut);
    c->coef = w + lay.off_coef;
    c->stage = (double2 *)(w + lay.off_stage);
    c->pairs = (double2 *)(w + lay.off_pairs);
    c->sink = (RhoSink *)(w + lay.off_sink);
    c->plan = (double2 *)(w + lay.off_plan);
    if (filtered) {
        c->filtered = true;
        c->theta = theta;
        c->fcap = fcap;
        for (int b = 0; b < 2; ++b) {
            c->fkeys[b] = (unsigned long long *)(w + lay.off_fkeys[b]);
            c->fvals[b] = w + lay.off_fvals[b];
        }
        c->fmask = (unsigned short *)(w + lay.off_fmask);
        c->fbofs = (unsigned long long *)(w + lay.off_fbofs);
        c->fctr = (unsigned long long *)(w + lay.off_fctr);
        c->fpart = (double2 *)(w + lay.off_fpart);
        c->fplan = (double2 *)(w + lay.off_fplan);
        c->fplan_entries = lay.fplan_entries;
        c->graph_failed = true;   // the steps read their sizes from device memory; nothing to capture
    }

    c->s_h.assign(p->s, p->s + M);
    // L = 1: the oldest-point tables carry K, whose rows are not shared
    if (N == 16 && L >= 2 && !filtered && !cls16_disabled())
        c->cls_ok = pack_classes16(c->s_h, &c->cls_out, &c->cls_rep, &c->cls_selb);
    c->H_h.assign(p->H, p->H + 2 * M * M);
    if (p->n_H > 0) c->Ht_h.assign(p->H_t, p->H_t + (size_t)2 * M * M * p->n_H);
    c->rho0_h.assign(p->rho0, p->rho0 + 2 * N);
    {
        // the path sum maps to its conjugate under the mirror only if rho0 does
        bool herm = true;
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b)
                herm = herm && p->rho0[2 * (a * M + b)] == p->rho0[2 * (b * M + a)] &&
                       p->rho0[2 * (a * M + b) + 1] == -p->rho0[2 * (b * M + a) + 1];
        if (triple_ok(N, L) && !filtered) {
            for (int pass = 0; pass < 2; ++pass)
                for (int h = 0; h < lay.split3.grid; ++h)
                    if (pass == 0 ? h < mirror4(h) : h == mirror4(h)) c->blk3_h.push_back(h);
            for (int low = 0; low < lay.split3.R * lay.split3.Q; ++low)
                if (mirror4(low) > low) c->low3_h.push_back(low);
            c->mirror_ok = herm;
        }
        if (fused_ok(N, L) && !filtered) {
            for (int pass = 0; pass < 2; ++pass)
                for (int h = 0; h < lay.split2.grid; ++h)
                    if (pass == 0 ? h < mirror4(h) : h == mirror4(h)) c->blk2_h.push_back(h);
            for (int low = 0; low < lay.split2.R * lay.split2.Q; ++low)
                if (mirror4(low) > low) c->low2_h.push_back(low);
        }
        if (single_mirror_ok(N, L, lay.main_split) && !filtered) {
            for (int pass = 0; pass < 2; ++pass)
                for (int h = 0; h < lay.main_split.grid; ++h)
                    if (pass == 0 ? h < mirror_n(N, h) : h == mirror_n(N, h)) c->blk1_h.push_back(h);
            if (N == 9)
                for (int low = 0; low < lay.main_split.R * lay.main_split.Q; ++low)
                    if (mirror9(low) > low) c->low1_h.push_back(low);
            c->mirror_ok = herm;
        }
        c->mirror = c->mirror_ok ? 1 : 0;
    }
    c->fuse = c->n_H > 0 || filtered ? 1 : fusion_width(N, L, c->prec);
    {
        // the persistent path: the tensor in LDS when both buffers fit a
        // block's LDS, else in the global buffers (still L2 resident)
        size_t ent = 1;
        checked_pow((size_t)N, L, &ent);
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_max = 64 * 1024;
        if (ent <= (size_t)kSmallMaxEntries && !filtered) {
            c->small = small_lds_bytes(N, c->prec, L, true) <= (size_t)lds_max ? 1
                       : small_lds_bytes(N, c->prec, L, false) <= (size_t)lds_max ? 2 : 0;
        }
    }
    c->pa_h = std::move(pa);
    c->ph_h = std::move(ph);
    c->pseg_h = std::move(pseg);
    if (p->bath.kind == QUAPI_BATH_TABLE) {
        c->tw_h.assign(p->bath.omega, p->bath.omega + p->bath.n_tab);
        c->tJ_h.assign(p->bath.J, p->bath.J + p->bath.n_tab);
    } else {
        c->tw_h.assign(1, 0.0);
        c->tJ_h.assign(1, 0.0);
    }
    gauss_legendre(kGL, c->glx_h, c->glw_h);

    auto up = [&](size_t off, const void *src, size_t bytes) {
        return hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(lay.off_s, c->s_h.data(), (size_t)M * 8);
    if (e == hipSuccess) e = up(lay.off_H, c->H_h.data(), (size_t)M * M * 16);
    if (e == hipSuccess && c->n_H > 0) e = up(lay.off_Ht, c->Ht_h.data(), c->Ht_h.size() * 8);
    if (e == hipSuccess) e = up(lay.off_rho0, c->rho0_h.data(), (size_t)N * 16);
    if (e == hipSuccess && !c->blk3_h.empty()) e = up(lay.off_blk3, c->blk3_h.data(), c->blk3_h.size() * sizeof(int));
    if (e == hipSuccess && (int)c->low3_h.size() != lay.n_low3) e = hipErrorInvalidValue;
    if (e == hipSuccess && !c->low3_h.empty()) e = up(lay.off_low3, c->low3_h.data(), c->low3_h.size() * sizeof(int));
    if (e == hipSuccess && !c->blk2_h.empty()) e = up(lay.off_blk2, c->blk2_h.data(), c->blk2_h.size() * sizeof(int));
    if (e == hipSuccess && (int)c->low2_h.size() != lay.n_low2) e = hipErrorInvalidValue;
    if (e == hipSuccess && !c->low2_h.empty()) e = up(lay.off_low2, c->low2_h.data(), c->low2_h.size() * sizeof(int));
    if (e == hipSuccess && !c->blk1_h.empty()) e = up(lay.off_blk1, c->blk1_h.data(), c->blk1_h.size() * sizeof(int));
    if (e == hipSuccess && (int)c->low1_h.size() != lay.n_low1) e = hipErrorInvalidValue;
    if (e == hipSuccess && !c->low1_h.empty()) e = up(lay.off_low1, c->low1_h.data(), c->low1_h.size() * sizeof(int));
    if (e == hipSuccess) e = up(lay.off_pa, c->pa_h.data(), c->pa_h.size() * 8);
    if (e == hipSuccess) e = up(lay.off_ph, c->ph_h.data(), c->ph_h.size() * 8);
    if (e == hipSuccess) e = up(lay.off_pseg, c->pseg_h.data(), c->pseg_h.size() * 4);
    if (e == hipSuccess) e = up(lay.off_tw, c->tw_h.data(), c->tw_h.size() * 8);
    if (e == hipSuccess) e = up(lay.off_tJ, c->tJ_h.data(), c->tJ_h.size() * 8);
    if (e == hipSuccess) e = up(lay.off_glx, c->glx_h.data(), kGL * 8);
    if (e == hipSuccess) e = up(lay.off_glw, c->glw_h.data(), kGL * 8);
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, QUAPI_ERR_DEVICE, "input upload failed: %s", hipGetErrorString(e));
    }

    hipEvent_t s0 = nullptr, s1 = nullptr;
    if (!one_stream) {
        (void)hipEventCreate(&s0);
        (void)hipEventCreate(&s1);
    }
    if (s0) (void)hipEventRecord(s0, c->stream);
    QuadArgs qa{};
    qa.kind = p->bath.kind;
    qa.xi = p->bath.xi;
    qa.omega_c = p->bath.omega_c;
    qa.kT = p->kT;
    qa.half_dt = 0.5 * p->dt;
    qa.pa = (const double *)(w + lay.off_pa);
    qa.ph = (const double *)(w + lay.off_ph);
    qa.pseg = (const int *)(w + lay.off_pseg);
    qa.n_panels = lay.n_panels;
    qa.tw = (const double *)(w + lay.off_tw);
    qa.tJ = (const double *)(w + lay.off_tJ);
    qa.n_tab = p->bath.kind == QUAPI_BATH_TABLE ? p->bath.n_tab : 0;
    qa.glx = (const double *)(w + lay.off_glx);
    qa.glw = (const double *)(w + lay.off_glw);
    e = launch_g_quad(qa, 2 * L + 3, c->g, c->stream);
    TablesArgs ta{};
    ta.M = M;
    ta.L = L;
    ta.dt = p->dt;
    ta.s = (const double *)(w + lay.off_s);
    ta.g = c->g;
    ta.U = c->U;
    ta.eta = c->eta;
    ta.bank = c->bank;
    ta.bank_f = c->bank_f;
    ta.k_trace_exact = c->prec == kPrecC64;            // FP32 arithmetic: keep the trace exact per step
    c->drive_ta = ta;
    // U = exp(-i H dt): for a driven system every interval's, once, in
    // parallel (step 1 uses the first); the tables kernel takes it from there
    if (c->n_H > 0) {
        if (e == hipSuccess) e = launch_u_stack(c->Ht_d, c->n_H, M, p->dt, c->Ut_d, c->stream);
        ta.U_given = c->Ut_d;
    } else {
        if (e == hipSuccess) e = launch_u_stack((const double2 *)(w + lay.off_H), 1, M, p->dt, c->U, c->stream);
        ta.U_given = c->U;
    }
    if (e == hipSuccess) e = launch_tables(ta, c->stream);
    if (e == hipSuccess && filtered)
        e = launch_filter_init(c->prec, c->rho0_d, c->bank, BankLayout{L}.self_end(), N, theta, fcap, c->fkeys[0],
                               c->fvals[0], c->fctr, (int *)(c->fctr + 2), c->stream);
    else if (e == hipSuccess)
        e = launch_init_tensor(N, c->prec, c->rho0_d, c->bank, BankLayout{L}.self_end(), c->A[0], c->stream);
    if (s1) (void)hipEventRecord(s1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        if (s0) (void)hipEventDestroy(s0);
        if (s1) (void)hipEventDestroy(s1);
        release(c);
        return fail(nullptr, QUAPI_ERR_DEVICE, "setup failed: %s", hipGetErrorString(e));
    }
    float ms = 0.0f;
    if (s0 && s1 && hipEventElapsedTime(&ms, s0, s1) == hipSuccess) c->setup_ms = ms;
    if (s0) (void)hipEventDestroy(s0);
    if (s1) (void)hipEventDestroy(s1);
    c->cur = 0;
    c->step = 0;
    *out = c;
    return QUAPI_OK;
}

}  // namespace

// ------------------------------------------------------------ static scratch
// The whole working set of quapi_propagate_static (both tensors, the factor
// tables, the rho reduction buffers): a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  In host code
// the array's name is not a device address: kernels and copies get the
// address hipGetSymbolAddress returns on the current device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu[kMaxStaticDevices];        // one static call at a time per device
void *g_static_ptr[kMaxStaticDevices] = {};       // the device address of `scratch`, per device
}  // namespace

namespace {
// The capacity limits of a filtered context: at least one entry, and at most
// 2^38 (a block's share of a step's outputs is counted in 32 bits).
constexpr size_t kFilterMaxCapacity = size_t(1) << 38;
std::string filter_args_error(double theta, size_t capacity) {
    if (!(theta >= 0.0) || !std::isfinite(theta)) return "theta must be finite and >= 0";
    if (capacity < 1 || capacity > kFilterMaxCapacity) return "capacity must be in 1 .. 2^38";
    return "";
}
}  // namespace

// ===================================================================== ABI
extern "C" {

size_t quapi_paper_pmc_bytes(int M, int dk_max) {
    if (M < 1 || dk_max < 0) return 0;
    size_t e;
    if (!checked_pow((size_t)M, 2 * (dk_max + 1), &e)) return 0;
    if (e > std::numeric_limits<size_t>::max() / 64) return 0;
    return 64 * e;
}

quapi_status quapi_footprint(const quapi_params *p, size_t *device_bytes) {
    const std::string msg = validate(p);
    if (!msg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", msg.c_str());
    if (!device_bytes) return fail(nullptr, QUAPI_ERR_INVALID, "device_bytes is NULL");
    *device_bytes = make_layout(*p, count_panels(*p)).total;
    return QUAPI_OK;
}

quapi_status quapi_create(const quapi_params *p, void *hip_stream, void *workspace, size_t ws_bytes,
                          quapi_ctx **out) {
    return create_ctx(p, hip_stream, workspace, ws_bytes, false, out);
}

quapi_status quapi_filtered_footprint(const quapi_params *p, size_t capacity, size_t *device_bytes) {
    const std::string msg = validate(p, kFilterMaxLog2);
    if (!msg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", msg.c_str());
    const std::string fmsg = filter_args_error(0.0, capacity);
    if (!fmsg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", fmsg.c_str());
    if (!device_bytes) return fail(nullptr, QUAPI_ERR_INVALID, "device_bytes is NULL");
    *device_bytes = make_layout(*p, count_panels(*p), capacity).total;
    return QUAPI_OK;
}

quapi_status quapi_create_filtered(const quapi_params *p, double theta, size_t capacity, void *hip_stream,
                                   quapi_ctx **out) {
    const std::string msg = validate(p, kFilterMaxLog2);
    if (!msg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", msg.c_str());
    const std::string fmsg = filter_args_error(theta, capacity);
    if (!fmsg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", fmsg.c_str());
    return create_ctx(p, hip_stream, nullptr, 0, false, out, theta, capacity);
}

quapi_status quapi_filter_stats(quapi_ctx *ctx, long long *entries, int *overflow) {
    if (!ctx || !entries || !overflow) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    if (!ctx->filtered) return fail(ctx, QUAPI_ERR_INVALID, "not a filtered context");
    BusyGuard g(ctx);
    if (!g.ok) return fail(ctx, QUAPI_ERR_STATE, "context in use by another call");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long ctr[3] = {};
    HIP_TRY(ctx, hipMemcpy(ctr, ctx->fctr, sizeof ctr, hipMemcpyDeviceToHost));
    *entries = (long long)ctr[ctx->cur];
    int ov = 0;
    std::memcpy(&ov, &ctr[2], sizeof ov);
    *overflow = ov;
    return QUAPI_OK;
}

quapi_status quapi_filter_read(quapi_ctx *ctx, size_t first, size_t count, long long *keys, double *vals) {
    if (!ctx || (count && (!keys || !vals))) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    if (!ctx->filtered) return fail(ctx, QUAPI_ERR_INVALID, "not a filtered context");
    BusyGuard g(ctx);
    if (!g.ok) return fail(ctx, QUAPI_ERR_STATE, "context in use by another call");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long n = 0;
    HIP_TRY(ctx, hipMemcpy(&n, ctx->fctr + ctx->cur, sizeof n, hipMemcpyDeviceToHost));
    if (first > n || count > n - first)
        return fail(ctx, QUAPI_ERR_INVALID, "range [%zu, %zu) exceeds the %llu kept entries", first, first + count, n);
    if (!count) return QUAPI_OK;
    HIP_TRY(ctx, hipMemcpy(keys, ctx->fkeys[ctx->cur] + first, count * 8, hipMemcpyDeviceToHost));
    if (ctx->prec == kPrecC128) {
        HIP_TRY(ctx, hipMemcpy(vals, (const char *)ctx->fvals[ctx->cur] + first * 16, count * 16,
                               hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * count);
        HIP_TRY(ctx, hipMemcpy(tmp.data(), (const char *)ctx->fvals[ctx->cur] + first * 8, count * 8,
                               hipMemcpyDeviceToHost));
        for (size_t i = 0; i < 2 * count; ++i) vals[i] = tmp[i];
    }
    return QUAPI_OK;
}

quapi_status quapi_propagate_static(const quapi_params *p, int n_steps, const int *sel, int n_sel,
                                    void *rho_out_dev, void *hip_stream) {
    const std::string msg = validate(p);
    if (!msg.empty()) return fail(nullptr, QUAPI_ERR_INVALID, "%s", msg.c_str());
    if (n_steps < 0) return fail(nullptr, QUAPI_ERR_INVALID, "n_steps must be >= 0");
    const size_t need = make_layout(*p, count_panels(*p)).total;
    if (need > kStaticScratchBytes)
        return fail(nullptr, QUAPI_ERR_INVALID,
                    "the working set needs %zu bytes; the static scratch holds %zu (use quapi_create)", need,
                    kStaticScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) return fail(nullptr, QUAPI_ERR_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev >= kMaxStaticDevices) return fail(nullptr, QUAPI_ERR_DEVICE, "device %d beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_static_mu[dev]);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, QUAPI_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_static_ptr[dev] = ptr;
    }
    quapi_ctx *c = nullptr;
    quapi_status st = create_ctx(p, hip_stream, g_static_ptr[dev], kStaticScratchBytes, true, &c);
    if (st != QUAPI_OK) return st;
    int n_out = 0;
    st = check_selection(c, n_steps, sel, n_sel, &n_out);
    if (st == QUAPI_OK && n_out > 0 && !rho_out_dev) st = fail(c, QUAPI_ERR_INVALID, "rho_out_dev is NULL");
    if (st == QUAPI_OK) st = propagate_impl(c, n_steps, sel, n_sel, (double2 *)rho_out_dev, nullptr);
    e = hipStreamSynchronize(c->stream);
    if (st == QUAPI_OK && e != hipSuccess)
        st = fail(c, QUAPI_ERR_DEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    release(c);
    return st;
}

quapi_status quapi_propagate(quapi_ctx *ctx, int n_steps, const int *sel, int n_sel, double *rho_out) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    BusyGuard g(ctx);
    if (!g.ok) return fail(ctx, QUAPI_ERR_STATE, "context is in use by another call");
    return propagate_impl(ctx, n_steps, sel, n_sel, nullptr, rho_out);
}

quapi_status quapi_propagate_async(quapi_ctx *ctx, int n_steps, const int *sel, int n_sel,
                                   void *rho_out_dev) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    BusyGuard g(ctx);
    if (!g.ok) return fail(ctx, QUAPI_ERR_STATE, "context is in use by another call");
    int n_out = 0;
    quapi_status st = check_selection(ctx, n_steps, sel, n_sel, &n_out);
    if (st != QUAPI_OK) return st;
    if (n_out > 0 && !rho_out_dev) return fail(ctx, QUAPI_ERR_INVALID, "rho_out_dev is NULL");
    return propagate_impl(ctx, n_steps, sel, n_sel, (double2 *)rho_out_dev, nullptr);
}

quapi_status quapi_persistent(const quapi_ctx *ctx, int *mode) {
    if (!ctx || !mode) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    *mode = small_on(ctx) ? ctx->small : 0;
    return QUAPI_OK;
}

quapi_status quapi_propagate_batch(quapi_ctx *const *ctxs, int n_ctx, const int *n_steps, const int *rho_mode,
                                   void *const *rho_out_dev) {
    if (n_ctx < 0 || (n_ctx > 0 && (!ctxs || !n_steps || !rho_mode || !rho_out_dev)))
        return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument or n_ctx < 0");
    if (n_ctx == 0) return QUAPI_OK;
    for (int k = 0; k < n_ctx; ++k) {
        const quapi_ctx *c = ctxs[k];
        if (!c) return fail(nullptr, QUAPI_ERR_INVALID, "ctxs[%d] is NULL", k);
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == c) return fail(nullptr, QUAPI_ERR_INVALID, "ctxs[%d] repeats ctxs[%d]", k, j);
        if (!small_on(c))
            return fail(nullptr, QUAPI_ERR_INVALID,
                        "ctxs[%d] is not on the persistent path (N^L above 2^14, a driven system, a pinned "
                        "launch width or mirror mode 2)", k);
        if (c->N != ctxs[0]->N || c->prec != ctxs[0]->prec)
            return fail(nullptr, QUAPI_ERR_INVALID, "ctxs[%d] differs from ctxs[0] in M or dtype", k);
        if (n_steps[k] < 0 || (long long)c->step + n_steps[k] > std::numeric_limits<int>::max())
            return fail(nullptr, QUAPI_ERR_INVALID, "n_steps[%d] = %d is negative or overflows the step counter", k,
                        n_steps[k]);
        if (rho_mode[k] < 0 || rho_mode[k] > 2)
            return fail(nullptr, QUAPI_ERR_INVALID, "rho_mode[%d] must be 0, 1 or 2", k);
        if (rho_mode[k] != 0 && n_steps[k] > 0 && !rho_out_dev[k])
            return fail(nullptr, QUAPI_ERR_INVALID, "rho_out_dev[%d] is NULL", k);
    }
    // hold every context for the call
    int held = 0;
    for (; held < n_ctx; ++held) {
        int z = 0;
        if (!ctxs[held]->busy.compare_exchange_strong(z, 1)) break;
    }
    struct Release {
        quapi_ctx *const *cs;
        int n;
        ~Release() {
            for (int k = 0; k < n; ++k) cs[k]->busy.store(0);
        }
    } release_all{ctxs, held};
    if (held < n_ctx) return fail(nullptr, QUAPI_ERR_STATE, "ctxs[%d] is in use by another call", held);
    quapi_ctx *c0 = ctxs[0];
    hipStream_t bs = c0->stream;
    // each context's earlier work (its stream, its side stream, a mirror half)
    // comes first; the launches run on the first context's stream
    for (int k = 0; k < n_ctx; ++k) {
        quapi_ctx *c = ctxs[k];
        quapi_status st = join_side(c);
        if (st == QUAPI_OK) st = ensure_full(c);
        if (st != QUAPI_OK) return st;
        if (k > 0) {
            HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
            HIP_TRY(c0, hipStreamWaitEvent(bs, c->ev_fork, 0));
        }
    }
    for (int mode = 1; mode <= 2; ++mode) {
        SmallBatchArgs b;
        int nb = 0, L_max = 1;
        auto launch = [&]() -> quapi_status {
            if (!nb) return QUAPI_OK;
            hipError_t e = launch_small(c0->N, c0->prec, mode == 1, b, nb, L_max, bs);
            if (e != hipSuccess) return fail(c0, QUAPI_ERR_DEVICE, "persistent batch launch: %s", hipGetErrorString(e));
            nb = 0;
            L_max = 1;
            return QUAPI_OK;
        };
        for (int k = 0; k < n_ctx; ++k) {
            quapi_ctx *c = ctxs[k];
            if (c->small != mode || n_steps[k] == 0) continue;
            b.c[nb++] = small_args(c, n_steps[k], rho_mode[k], (double2 *)rho_out_dev[k]);
            L_max = std::max(L_max, c->L);
            if (nb == kMaxSmallBatch)
                if (quapi_status st = launch(); st != QUAPI_OK) return st;
        }
        if (quapi_status st = launch(); st != QUAPI_OK) return st;
    }
    for (int k = 0; k < n_ctx; ++k) small_advance(ctxs[k], n_steps[k]);
    // later work on every other context's stream waits for the launches
    if (n_ctx > 1) {
        HIP_TRY(c0, hipEventRecord(c0->ev_join, bs));
        for (int k = 1; k < n_ctx; ++k) HIP_TRY(ctxs[k], hipStreamWaitEvent(ctxs[k]->stream, c0->ev_join, 0));
    }
    return QUAPI_OK;
}

quapi_status quapi_step_count(const quapi_ctx *ctx, int *step) {
    if (!ctx || !step) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    *step = ctx->step;
    return QUAPI_OK;
}

quapi_status quapi_fused_steps(const quapi_ctx *ctx, int *steps) {
    if (!ctx || !steps) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    *steps = ctx->fuse;
    return QUAPI_OK;
}

quapi_status quapi_set_fused_steps(quapi_ctx *ctx, int steps) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    if (ctx->filtered && steps > 1) return fail(ctx, QUAPI_ERR_INVALID, "a filtered context runs one step at a time");
    const int N = ctx->N, L = ctx->L;
    const bool pinned = steps != 0;
    if (steps == 0) steps = ctx->n_H > 0 || ctx->filtered ? 1 : fusion_width(N, L, ctx->prec);
    if (ctx->n_H > 0 && steps != 1)
        return fail(ctx, QUAPI_ERR_INVALID, "a driven context runs one step per launch");
    const bool ok = steps == 1 || (steps == 2 && fused_ok(N, L)) || (steps == 3 && triple_ok(N, L));
    if (!ok)
        return fail(ctx, QUAPI_ERR_INVALID, "%d fused steps unavailable at N = %d, L = %d (1 always; 2: N = 4, L >= 3; "
                    "3: N = 4, L >= 4)", steps, N, L);
    BusyGuard guard(ctx);
    if (!guard.ok) return fail(ctx, QUAPI_ERR_STATE, "context in use by another call");
    ctx->fuse = steps;
    ctx->fuse_pinned = pinned;
    return QUAPI_OK;
}

quapi_status quapi_mirror(const quapi_ctx *ctx, int *enabled) {
    if (!ctx || !enabled) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    *enabled = ctx->mirror;
    return QUAPI_OK;
}

quapi_status quapi_set_mirror(quapi_ctx *ctx, int enable) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    if (enable && !ctx->mirror_ok)
        return fail(ctx, QUAPI_ERR_INVALID, "mirror mode needs M = 2, 3 or 4, L >= 2 and an exactly Hermitian rho0");
    if (enable < 0 || enable > 2) return fail(ctx, QUAPI_ERR_INVALID, "enable must be 0, 1 or 2");
    BusyGuard guard(ctx);       // the graphs destroyed below must not be replayed meanwhile
    if (!guard.ok) return fail(ctx, QUAPI_ERR_STATE, "context in use by another call");
    if (enable == ctx->mirror) return QUAPI_OK;
    // the captured graphs hold the launches of the old mode
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &row : ctx->graph3)
        for (auto &g : row) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (auto &g : ctx->graph1) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto &row : ctx->graph2)
        for (auto &g : row) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    ctx->mirror = enable;
    return QUAPI_OK;
}

quapi_status quapi_get_setup(const quapi_ctx *ctx, int what, double *out, size_t out_len) {
    if (!ctx || !out) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    quapi_ctx *c = const_cast<quapi_ctx *>(ctx);
    const void *src = nullptr;
    size_t n = 0;
    switch (what) {
    case QUAPI_SETUP_G: src = c->g; n = 2 * c->L + 3; break;
    case QUAPI_SETUP_ETA: src = c->eta; n = 4 * c->L + 2; break;
    case QUAPI_SETUP_U: src = c->U; n = (size_t)c->M * c->M; break;
    case QUAPI_SETUP_K: src = c->bank + (size_t)BankLayout{c->L}.K() * c->N * c->N; n = (size_t)c->N * c->N; break;
    default: return fail(c, QUAPI_ERR_INVALID, "unknown setup item %d", what);
    }
    if (out_len < 2 * n) return fail(c, QUAPI_ERR_INVALID, "out_len %zu < %zu", out_len, 2 * n);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(out, src, n * 16, hipMemcpyDeviceToHost));
    return QUAPI_OK;
}

quapi_status quapi_tensor_size(const quapi_ctx *ctx, size_t *entries) {
    if (!ctx || !entries) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    if (ctx->filtered)
        return fail(const_cast<quapi_ctx *>(ctx), QUAPI_ERR_INVALID, "a filtered context: use quapi_filter_stats");
    const int axes = std::min(ctx->step + 1, ctx->L);
    *entries = (size_t)ipow_ll(ctx->N, axes);
    return QUAPI_OK;
}

quapi_status quapi_read_tensor(const quapi_ctx *ctx, size_t first, size_t count, double *out) {
    if (!ctx || (!out && count)) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    quapi_ctx *c = const_cast<quapi_ctx *>(ctx);
    if (c->filtered) return fail(c, QUAPI_ERR_INVALID, "a filtered context: use quapi_filter_read");
    BusyGuard g(c);                        // the step count and, in the completion pass, the tensor
    if (!g.ok) return fail(c, QUAPI_ERR_STATE, "context in use by another call");
    size_t entries = 0;
    quapi_tensor_size(ctx, &entries);
    if (first > entries || count > entries - first)
        return fail(c, QUAPI_ERR_INVALID, "range [%zu, %zu) exceeds the tensor of %zu entries", first,
                    first + count, entries);
    if (!count) return QUAPI_OK;
    if (quapi_status fs = ensure_full(c); fs != QUAPI_OK) return fs;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->prec == kPrecC128) {
        HIP_TRY(c, hipMemcpy(out, (const char *)c->A[c->cur] + first * 16, count * 16, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * count);
        HIP_TRY(c, hipMemcpy(tmp.data(), (const char *)c->A[c->cur] + first * 8, count * 8, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < 2 * count; ++i) out[i] = tmp[i];
    }
    return QUAPI_OK;
}

quapi_status quapi_restore(quapi_ctx *ctx, int step, const double *tensor, size_t count) {
    if (!ctx || !tensor) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    quapi_ctx *c = ctx;
    if (c->filtered) return fail(c, QUAPI_ERR_INVALID, "a filtered context cannot be restored from a dense tensor");
    if (step < 0) return fail(c, QUAPI_ERR_INVALID, "step must be >= 0");
    const size_t want = (size_t)ipow_ll(c->N, std::min(step + 1, c->L));
    if (count != want)
        return fail(c, QUAPI_ERR_INVALID, "count %zu is not N^min(step+1, L) = %zu", count, want);
    BusyGuard g(c);
    if (!g.ok) return fail(c, QUAPI_ERR_STATE, "context in use by another call");
    if (quapi_status js = join_side(c); js != QUAPI_OK) return js;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // on the context's stream, so that its next kernels see the copy
    std::vector<float> tmp;
    if (c->prec == kPrecC128) {
        HIP_TRY(c, hipMemcpyAsync(c->A[c->cur], tensor, count * 16, hipMemcpyHostToDevice, c->stream));
    } else {
        tmp.resize(2 * count);
        for (size_t i = 0; i < 2 * count; ++i) tmp[i] = (float)tensor[i];
        HIP_TRY(c, hipMemcpyAsync(c->A[c->cur], tmp.data(), count * 8, hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = step;
    c->half_cur = false;
    return QUAPI_OK;
}

quapi_status quapi_set_timing(quapi_ctx *ctx, int enable) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    ctx->timing = enable != 0;
    return QUAPI_OK;
}

quapi_status quapi_get_timing(quapi_ctx *ctx, quapi_timing *out) {
    if (!ctx || !out) return fail(nullptr, QUAPI_ERR_INVALID, "NULL argument");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->side));
    for (auto &r : ctx->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ctx->acc_ms[r.kind] += ms;
            ctx->acc_n[r.kind] += 1;
            ctx->acc_steps += r.steps;
            if (r.kind == 0) {
                ctx->acc_width_ms[r.width] += ms;
                ctx->acc_width_n[r.width] += 1;
            }
        }
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    out->setup_ms = ctx->setup_ms;
    out->step_ms = ctx->acc_ms[0];
    out->step_launches = ctx->acc_n[0];
    out->step_steps = ctx->acc_steps;
    out->grow_ms = ctx->acc_ms[1];
    out->grow_launches = ctx->acc_n[1];
    out->finalize_ms = ctx->acc_ms[2];
    out->finalize_launches = ctx->acc_n[2];
    for (int k = 0; k < 4; ++k) {
        out->width_ms[k] = ctx->acc_width_ms[k];
        out->width_launches[k] = ctx->acc_width_n[k];
        ctx->acc_width_ms[k] = 0.0;
        ctx->acc_width_n[k] = 0;
    }
    for (int k = 0; k < 3; ++k) {
        ctx->acc_ms[k] = 0.0;
        ctx->acc_n[k] = 0;
    }
    ctx->acc_steps = 0;
    return QUAPI_OK;
}

quapi_status quapi_destroy(quapi_ctx *ctx) {
    if (!ctx) return fail(nullptr, QUAPI_ERR_INVALID, "ctx is NULL");
    if (ctx->busy.load() != 0) return fail(ctx, QUAPI_ERR_STATE, "context is in use by another call");
    release(ctx);
    return QUAPI_OK;
}

const char *quapi_last_error(const quapi_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
