// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace quapi {

constexpr int kMaxM = 4;
constexpr int kMaxN = kMaxM * kMaxM;
constexpr int kMaxL = 30;
constexpr int kBlock = 256;              // threads per block of every propagation kernel
constexpr int kGL = 16;                  // Gauss-Legendre nodes per quadrature panel
constexpr int kLdsLimit = 64 * 1024;     // LDS bytes a step block may use
// gfx950 has 160 KB of LDS per compute unit; the three-step kernel with FP32
// arithmetic keeps its rho sums there (about 73 KB per block, two blocks per CU)
constexpr int kLdsLimitStep3 = 80 * 1024;

// Tensor precision (values of quapi_dtype): storage / arithmetic.
constexpr int kPrecC128 = 0;             // complex128 / FP64
constexpr int kPrecC64 = 1;              // complex64 / FP32
constexpr int kPrecC64F64 = 2;           // complex64 / FP64

// Influence/propagator table bank.  Every table is N x N complex128, row o
// (later point) and column p (earlier point), stored at bank[t * N*N + o*N + p].
struct BankLayout {
    int L;
    __host__ __device__ int K() const { return 0; }
    __host__ __device__ int lag(int D) const { return D; }               // D = 1..L
    __host__ __device__ int init(int k) const { return L + k; }          // k = 1..L
    __host__ __device__ int fin(int D) const { return 2 * L + D; }       // D = 1..L
    __host__ __device__ int fin_init(int n) const { return 3 * L + n; }  // n = 1..L
    __host__ __device__ int self_int() const { return 4 * L + 1; }       // row o: F_self_interior(o)
    __host__ __device__ int self_end() const { return 4 * L + 2; }       // row o: F_self_end(o)
    __host__ __device__ int k_lag1() const { return 4 * L + 3; }         // K * F_lag[1]
    __host__ __device__ int k_init1() const { return 4 * L + 4; }        // K * F_init[1]
    __host__ __device__ int k_fin1() const { return 4 * L + 5; }         // K * F_fin[1]
    __host__ __device__ int k_fin_init1() const { return 4 * L + 6; }    // K * F_fin_init[1]
    // Oldest-point tables of a full-window step, with the new point's self
    // factor folded in (and K too when L = 1, where the oldest point is n-1).
    __host__ __device__ int old_main() const { return 4 * L + 7; }       // n > L, interior
    __host__ __device__ int old_first() const { return 4 * L + 8; }      // n = L, oldest is point 0
    __host__ __device__ int oldf_main() const { return 4 * L + 9; }      // n > L, final classes
    __host__ __device__ int oldf_first() const { return 4 * L + 10; }    // n = L, final classes
    __host__ __device__ int count() const { return 4 * L + 11; }
};

// One propagation step: A_out[m + m_count*o] = P(o,m) * sum_i Old[o][i] A_in[i + I*m].
struct StepArgs {
    const void *a_in;
    void *a_out;
    const double2 *bank;
    const void *bank_c;         // the bank in the compute precision (N >= 9 reads it by scalar loads)
    // Full-window steps: factor products over the thread / sweep / block digits,
    // precomputed once per context (FP64, [N][R], [N][Q], [N][grid]).  NULL:
    // the kernel multiplies the bank tables of the digits itself (growth steps).
    const double2 *t_lo, *t_lof, *t_mid, *t_midf, *t_hi, *t_hif;
    double2 *partials;          // [grid][N] block partial sums of rho (with_rho)
    long long m_count;          // N^n_digits
    int n_digits;               // digits of m
    int d_lo, d_mid;            // digits owned by the thread / swept by the block loop
    int R, Q, grid;             // N^d_lo, N^d_mid, N^(n_digits - d_lo - d_mid)
    int old_tab, oldf_tab;      // bank indices of the oldest-point tables
    int16_t tab[kMaxL];         // bank index of the interior table for digit j
    int16_t tabf[kMaxL];        // bank index of the final-point table for digit j
    // Mirror mode of the N = 4, 9 and 16 single steps (as for the three-step
    // kernel): mode 1 the high-digit values blk_hi[..] below their mirror
    // (n_canon of them), mode 2 those equal to it in `parts` blocks of q_span
    // sweep rows (items below their mirror), mode 3 the same values, the items
    // that are their own mirror; rho partials at row part_base + block.  At
    // N = 9 the mode-1 launch also runs, after its n_canon blocks, `parts`
    // blocks per value equal to its mirror over q_span items of low_list (the
    // n_low indices qm * R + r below their mirror), and mode 2 does not run.
    // Mode 0: every block.
    const int *blk_hi;
    const int *low_list;
    int n_blk, n_canon, parts, q_span, part_base, mode, n_low;
    // N = 16 full-window steps (L >= 2) with the new points grouped by their
    // oldest-point rows (cls_on): the row of o is F_self(o) times the
    // influence row of the oldest point, which depends on o = (a, b) only
    // through s_a - s_b; outputs with equal s_a - s_b share one contraction
    // with the influence table cls_tab (interior) / clsf_tab (final point),
    // and the self factors (tables cls_self, cls_selff) scale the outputs.
    // Lane group g of the MFMA form owns the outputs cls_out >> 4(4g + q)
    // (q = 0..3, 4 bits each), which take the contraction of class slot
    // (cls_selb >> (4g + q)) & 1; slot c of group g is the row of output
    // cls_rep >> 4(2g + c).
    int cls_on, cls_tab, clsf_tab, cls_self, cls_selff;
    unsigned long long cls_out;
    unsigned cls_rep, cls_selb;
};

// Two consecutive full-window steps n, n+1 (n > L, N = 4) in one pass:
// A_out[m + m_count*(o + N*o')] from the N^2 contiguous inputs A_in[i + N*i' + N^2*m],
// m the digits of points n-L+2 .. n-1 (m_count = N^(L-2)); A_n stays in registers.
struct Step2Args {
    const void *a_in;
    void *a_out;
    const double2 *bank;
    // factor products over the digits of m, per table set: 0 interior step n,
    // 1 interior step n+1, 2 final step n, 3 final step n+1 ([N][R], [N][Q], [N][grid])
    const double2 *t_lo[4], *t_mid[4], *t_hi[4];
    double2 *partials[2];       // block partials of rho(t_n), rho(t_{n+1}) [grid][N]
    long long m_count;
    int R, Q, grid;
    const void *coef;           // kCoefCount complex entries in the compute precision
    // Mirror mode, as for the three-step kernel (Step3Args): modes 1 (with
    // the listed items of the diagonal values as its tail) and 3 over the
    // high-digit values blk_hi[..]; rho partials at part_base + block.
    const int *blk_hi;
    const int *low_list;
    int n_blk, n_canon, parts, q_span, part_base, mode, n_low;
};

// Coefficients of the fused step in the compute precision, grouped by the new
// point o of step n so that one o reads one contiguous stretch of kCoefPerO:
//   OA[o][i'][i]   an[o][i'] old[o][i]    (step-n entry y(o, i') from x(i, i'))
//   W[o][i + N i'] anf[o][i'] oldf[o][i]  (rho(t_n) weight of x(i, i'))
//   DO[o][o'][i']  dT[o][o'] old[o'][i']  (step-(n+1) entry (o, o') from y(o, i'))
//   V[o][o'][i']   df[o'][o] oldf[o'][i'] (rho(t_{n+1}) weight of y(o, i'))
// old: oldest point seen from the new point (both steps); an: point n-L+1 seen
// from o (step n); dT[o][o']: point n (= o) seen from o' (step n+1, K folded in).
constexpr int kCoefOA = 0, kCoefW = 16, kCoefDO = 32, kCoefV = 48, kCoefPerO = 64, kCoefCount = 4 * kCoefPerO;
struct CoefArgs {
    const double2 *bank;
    // bank indices: oldest point (interior / final; both steps), point n-L+1 for
    // step n (interior / final), point n for step n+1 (interior / final, K folded)
    int old_tab, oldf_tab, an_tab, anf_tab, d_tab, df_tab;
    int prec;
    void *out;
};

// Three consecutive full-window steps n, n+1, n+2 (n > L, N = 4, L >= 4) in
// one pass: A_out[m + m_count*(o + N*o' + N^2*o'')] from the N^3 contiguous
// inputs A_in[i + N*i' + N^2*i'' + N^3*m], m the digits of points
// n-L+3 .. n-1 (m_count = N^(L-3)); the step-n and step-(n+1) tensors stay in
// registers.
struct Step3Args {
    const void *a_in;
    void *a_out;
    // factor products over the digits of m, per table set: 0, 1, 2 interior
    // steps n, n+1, n+2; 3, 4, 5 final point of those steps ([N][R], [N][Q], [N][grid])
    const double2 *t_lo[6], *t_mid[6], *t_hi[6];
    double2 *partials[3];       // block partials of rho(t_n), rho(t_{n+1}), rho(t_{n+2})
    long long m_count;
    int R, Q, grid;
    const void *coef;           // kC3Count complex entries in the compute precision
    // Mirror mode (half of the tensor), two launches over high-digit values
    // blk_hi[..] (n_canon values below their mirror, then those equal to it,
    // all digits diagonal): mode 1 one block per value below its mirror
    // (every item below its mirror), then `parts` blocks per value equal to
    // it, each running q_span items of low_list (the n_low item indices
    // qm * R + r below their mirror, the same list for every such value):
    // n_blk = n_canon + values * parts; mode 3 (blk_hi from the equal
    // values) one block per value equal to its mirror, running the items
    // that are their own mirror.  rho partials go to row part_base + block.
    // Mode 0 runs every block of the grid.
    const int *blk_hi;
    const int *low_list;
    int n_blk, n_canon, parts, q_span, part_base, mode, n_low;
};

// The mirror of an entry (N = 4, M = 2): every digit o = (a, b) -> (b, a),
// i.e. 1 <-> 2, which swaps the two bits of each base-4 digit.  The path sum
// maps to its complex conjugate under it (K, every influence factor and a
// Hermitian rho(0) do), so A[mirror(x)] = conj(A[x]) for every entry x.
__host__ __device__ constexpr long long mirror4(long long x) {
    return ((x & 0x5555555555555555LL) << 1) | ((x >> 1) & 0x5555555555555555LL);
}
// The same for N = 16 (M = 4): digit o = 4a + b -> 4b + a swaps the two bit
// pairs of each base-16 digit.
__host__ __device__ constexpr long long mirror16(long long x) {
    return ((x & 0x3333333333333333LL) << 2) | ((x >> 2) & 0x3333333333333333LL);
}
// N = 9 (M = 3): digit o = 3a + b -> 3b + a, digit by digit.
__host__ __device__ inline long long mirror9(long long x) {
    long long out = 0, w = 1;
    while (x > 0) {
        const int d = (int)(x % 9);
        out += (long long)(3 * (d % 3) + d / 3) * w;
        x /= 9;
        w *= 9;
    }
    return out;
}
__host__ __device__ inline long long mirror_n(int N, long long x) {
    return N == 4 ? mirror4(x) : N == 16 ? mirror16(x) : N == 9 ? mirror9(x) : x;
}

// Coefficients of the three-step kernel (compute precision), the four of one
// group of a stage contiguous (indexed by the stage's new point last):
//   old[o][i], oldf[o][i]       oldest point seen from the new point (every step)
//   AF[i''][i'][o]  an(o, i') F(o, i'')     step n: points n-L+1 (lag L-1), n-L+2 (lag L-2)
//   GH[i''][o][o']  G(o', o) H(o', i'')     step n+1: point n (lag 1, K), n-L+2 (lag L-1)
//   PQ[o'][o][o'']  P(o'', o') Q(o'', o)    step n+2: point n+1 (lag 1, K), n (lag 2)
// and the final-point versions (suffix f) for rho.
constexpr int kC3Old = 0, kC3Oldf = 16, kC3AF = 32, kC3AFf = 96, kC3GH = 160, kC3GHf = 224, kC3PQ = 288,
              kC3PQf = 352, kC3Count = 416;
struct Coef3Args {
    const double2 *bank;
    int old_tab, oldf_tab, an_tab, anf_tab, f_tab, ff_tab, g_tab, gf_tab, h_tab, hf_tab, p_tab, pf_tab,
        q_tab, qf_tab;
    int prec;
    void *out;
};

// Factor products of the full-window digit split (see StepArgs::t_lo ...).
struct PlanArgs {
    const double2 *bank;
    int N, d_lo, d_mid, n_digits, R, Q, grid;
    int16_t tab[kMaxL], tabf[kMaxL];
    double2 *t_lo, *t_lof, *t_mid, *t_midf, *t_hi, *t_hif;
};

struct QuadArgs {
    int kind;                   // 0 Ohmic, 1 table
    double xi, omega_c, kT, half_dt;
    const double *pa, *ph;      // panel left ends and widths
    const int *pseg;            // table segment of each panel (-1 for Ohmic)
    int n_panels;
    const double *tw, *tJ;      // table nodes and values
    int n_tab;
    const double *glx, *glw;    // Gauss-Legendre nodes/weights on [-1, 1]
};

struct TablesArgs {
    int M, L;
    double dt;
    const double *s;
    const double2 *g;           // G(j dt/2), j = 0..2L+2
    double2 *U;                 // out: M x M
    double2 *eta;               // out: 4L+2 classes
    double2 *bank;              // out: BankLayout{L}.count() tables
    float2 *bank_f;             // out (if not NULL): the same tables rounded to complex64
    int k_trace_exact;          // K rows (a, a) chosen on the FP32 grid with exact column sums
    int k_only;                 // rewrite only the tables that carry K (driven H: per step); eta, U untouched
    const double2 *U_given;     // U (M x M) from launch_u_stack
};

// Kernel launchers (quapi_kernels.hip).  They return the launch status.
hipError_t launch_g_quad(const QuadArgs &a, int n_t, double2 *g, hipStream_t st);
hipError_t launch_tables(const TablesArgs &a, hipStream_t st);
// U_k = exp(-i H_t[k] dt) for k < n_H (M x M each), a thread each.
hipError_t launch_u_stack(const double2 *H_t, int n_H, int M, double dt, double2 *U_t, hipStream_t st);
hipError_t launch_init_tensor(int N, int prec, const double2 *rho0, const double2 *bank,
                              int self_end_tab, void *a0, hipStream_t st);
hipError_t launch_step(int N, int prec, bool with_rho, bool grow, const StepArgs &a, int grid,
                       hipStream_t st);
// Where finalized rho values go: rho of the k-th finalize after a reset is
// written to base + k*N.  Device-resident, so graph replays need no new arguments.
struct RhoSink {
    double2 *base;
    unsigned long long count;
};

// Sums the block partials of rho into the sink's next slot: two launches on
// st, using pairs (kRhoSlices * N * 2 complex) as scratch.
constexpr int kRhoSlices = 256;
hipError_t launch_rho_finalize(int N, const double2 *partials, int n_blocks, double2 *pairs, RhoSink *sink,
                               hipStream_t st);
// sink = {base, 0}, as a kernel (no memset node) so that it is capture-safe.
hipError_t launch_set_sink(RhoSink *sink, double2 *base, hipStream_t st);
hipError_t launch_plan_tables(const PlanArgs &a, hipStream_t st);
size_t step_lds_bytes(int N, int prec, bool with_rho, bool grow, int R, int Q);
hipError_t launch_step2(int prec, bool with_rho, const Step2Args &a, hipStream_t st);
hipError_t launch_step2_coef(const CoefArgs &a, hipStream_t st);
hipError_t launch_step3(int prec, bool with_rho, const Step3Args &a, hipStream_t st);
// Persistent propagation of small tensors (quapi_small.hip): one block per
// context runs every step of a call.  The tensor is in a0 at entry and ends
// in a0 after an even number of steps, a1 after an odd one.
constexpr int kSmallBlock = 256;
constexpr int kMaxSmallBatch = 32;                   // contexts per launch (kernel-argument size)
// N^L of a context on the persistent path: up to here one workgroup per
// step beats the multi-block kernels (M = 2, L = 7: 13 against 23 us per
// step with rho; at 2^16 entries it is slower, 40 against 23 us)
constexpr long long kSmallMaxEntries = 1LL << 14;
struct SmallCtxArgs {
    const double2 *bank;
    void *a0, *a1;              // the context's two tensor buffers
    double2 *rho_out;           // rho of the selected steps, N complex each, in step order
    int L;
    int step0;                  // global step reached before the launch
    int n_steps;
    int rho_mode;               // 0 none, 1 every step, 2 the last step of the launch
};
struct SmallBatchArgs {
    SmallCtxArgs c[kMaxSmallBatch];
};
// LDS bytes of a block (in_lds: the two tensor buffers in LDS too).
size_t small_lds_bytes(int N, int prec, int L, bool in_lds);
// n_ctx blocks, block k running b.c[k]; L_max sizes the dynamic LDS.
hipError_t launch_small(int N, int prec, bool in_lds, const SmallBatchArgs &b, int n_ctx, int L_max,
                        hipStream_t st);
// Fill every entry above its mirror (N = 4, 9 or 16) with the conjugate of the mirror.
hipError_t launch_mirror_complete(int N, int prec, void *a, long long entries, hipStream_t st);
hipError_t launch_step3_coef(const Coef3Args &a, hipStream_t st);
size_t step3_lds_bytes(int prec, bool with_rho, int R, int Q);
size_t step2_lds_bytes(int prec, bool with_rho, int R, int Q);

// Filtered propagation (quapi_filter.hip): the kept tensor entries as sorted
// (key, value) pairs.  Fixed grids; the entry count is read from device memory.
constexpr int kFilterBlock = 256;
constexpr int kFilterStepBlocks = 2048;      // blocks of the count and write passes (rho partial rows)
// Factor-product tables of a step's digits, in levels (filter_levels of them,
// filter_level_size x N entries each), every entry the FP64 pair (interior,
// final classes).
struct FilterPlanArgs {
    const double2 *bank;
    int N, nd, n_lv;
    int16_t tab[kMaxL], tabf[kMaxL];
    double2 *t;
};
struct FilterStepArgs {
    const double2 *bank;
    const unsigned long long *count_in;      // entries of the input
    const unsigned long long *keys_in;
    const void *vals_in;
    unsigned long long *keys_out;
    void *vals_out;
    unsigned short *masks;      // [entries] keep bits of a segment's N outputs, at its head entry
    unsigned long long *bofs;   // [N][kFilterStepBlocks] kept outputs per (o, block), then their offsets
    double2 *partials;          // [kFilterStepBlocks][N] block partial sums of rho (count pass)
    const double2 *t;           // factor-product levels, (interior, final) pairs
    unsigned long long capacity;
    unsigned long long stride_new;   // N^(L-1) (full window) or N^n (growth step n)
    double theta;
    int full, n_lv;
    int old_tab, oldf_tab;      // oldest-point tables (full window) or self factors (growth, column 0)
};
size_t filter_step_lds_bytes(int N, bool rho);      // dynamic LDS of the count pass with rho
int filter_levels(int N, int n_digits);
size_t filter_plan_entries(int N, int n_digits);
hipError_t launch_filter_plan(const FilterPlanArgs &a, hipStream_t st);
// count = true: keep masks, per-(o, block) counts and (rho) partials; false: the write pass.
hipError_t launch_filter_step(int N, int prec, const FilterStepArgs &a, bool count, bool rho, hipStream_t st);
hipError_t launch_filter_offsets(int N, unsigned long long *bofs, unsigned long long capacity,
                                 unsigned long long *count_out, int *overflow, hipStream_t st);
hipError_t launch_filter_init(int prec, const double2 *rho0, const double2 *bank, int self_end_tab, int N,
                              double theta, unsigned long long capacity, unsigned long long *keys, void *vals,
                              unsigned long long *count, int *overflow, hipStream_t st);

}  // namespace quapi
