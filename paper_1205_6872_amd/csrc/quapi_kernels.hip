// HIP kernels for gfx950: Feynman-integral setup (lineshape quadrature,
// eta classes, propagator and influence tables) and the tensor-propagator
// step with fused rho extraction.
//
// Method: Dattani 2012, Sec. II (bath response function, exact path-sum
// equation, discretized influence functional, eta definitions); the tensor
// step is the tensor-propagator scheme the Introduction attributes to Makri
// and Makarov.  Unlike the paper's program, the N^(L+1) propagator array is
// never materialized: each step recomputes the factor product of an output
// entry from N x N tables, hoisting the product over the index digits that
// are constant across a block, a loop sweep, or a thread.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

// ------------------------------------------------ compensated summation
// Neumaier's variant of Kahan summation: s + c carries the running sum.
__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}
// (s1, c1) += (s2, c2) with the rounding error of s1 + s2 kept (Knuth's two-sum).
__device__ __forceinline__ void two_sum_combine(double &s1, double &c1, double s2, double c2) {
    const double s = s1 + s2;
    const double bp = s - s1;
    const double e = (s1 - (s - bp)) + (s2 - bp);
    s1 = s;
    c1 = c1 + c2 + e;
}
// Block-wide compensated reduction of (sum, compensation) pairs for a real
// and an imaginary part, in a fixed tree order; the totals land in thread 0's
// arguments.  All B threads of the block must call it.
template <int B>
__device__ void block_reduce_pairs(double &sr, double &cr, double &si, double &ci) {
    __shared__ double s_v[4][B];
    const int t = threadIdx.x;
    s_v[0][t] = sr;
    s_v[1][t] = cr;
    s_v[2][t] = si;
    s_v[3][t] = ci;
    __syncthreads();
    for (int w = B / 2; w > 0; w >>= 1) {
        if (t < w) {
            two_sum_combine(s_v[0][t], s_v[1][t], s_v[0][t + w], s_v[1][t + w]);
            two_sum_combine(s_v[2][t], s_v[3][t], s_v[2][t + w], s_v[3][t + w]);
        }
        __syncthreads();
    }
    sr = s_v[0][0];
    cr = s_v[1][0];
    si = s_v[2][0];
    ci = s_v[3][0];
    __syncthreads();
}
__device__ double2 block_sum_compensated(double sr, double cr, double si, double ci) {
    block_reduce_pairs<kBlock>(sr, cr, si, ci);
    return make_double2(sr + cr, si + ci);
}

// --------------------------------------------------- lineshape quadrature
// sin(u) - u without cancellation: Taylor series for |u| < 1 (terms through
// u^21; the first omitted term is below 1e-21 of the result), direct otherwise.
__device__ double sin_minus_id(double u) {
    if (fabs(u) >= 1.0) return sin(u) - u;
    const double u2 = u * u;
    double p = 1.0 / 51090942171709440000.0;    // +1/21!
    p = fma(p, u2, -1.0 / 121645100408832000.0); // -1/19!
    p = fma(p, u2, 1.0 / 355687428096000.0);     // +1/17!
    p = fma(p, u2, -1.0 / 1307674368000.0);      // -1/15!
    p = fma(p, u2, 1.0 / 6227020800.0);          // +1/13!
    p = fma(p, u2, -1.0 / 39916800.0);           // -1/11!
    p = fma(p, u2, 1.0 / 362880.0);              // +1/9!
    p = fma(p, u2, -1.0 / 5040.0);               // -1/7!
    p = fma(p, u2, 1.0 / 120.0);                 // +1/5!
    p = fma(p, u2, -1.0 / 6.0);                  // -1/3!
    return u * u2 * p;
}

// G(t_j) = (1/pi) Int_0^inf J(w)/w^2 [coth(w/2kT)(1 - cos wt) + i (sin wt - wt)] dw,
// t_j = j dt/2, by composite Gauss-Legendre over host-planned panels.  One
// block per t_j; compensated sums, fixed reduction order.
__global__ void __launch_bounds__(kBlock) g_quad_kernel(const QuadArgs a, double2 *g) {
    const int j = blockIdx.x;
    const double t = j * a.half_dt;
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    if (j > 0) {
        const int total = a.n_panels * kGL;
        for (int idx = threadIdx.x; idx < total; idx += kBlock) {
            const int p = idx / kGL, q = idx % kGL;
            const double half_h = 0.5 * a.ph[p];
            const double w = a.pa[p] + half_h * (1.0 + a.glx[q]);
            const double wq = half_h * a.glw[q];
            double jw;  // J(w) / w
            if (a.kind == 0) {
                jw = 0.5 * M_PI * a.xi * exp(-w / a.omega_c);
            } else {
                const int sg = a.pseg[p];
                const double w1 = a.tw[sg], J1 = a.tJ[sg];
                if (sg == 0) {
                    jw = J1 / w1;  // J linear through (0, 0) on the first segment
                } else {
                    const double w0 = a.tw[sg - 1], J0 = a.tJ[sg - 1];
                    jw = (J0 + (J1 - J0) * ((w - w0) / (w1 - w0))) / w;
                }
            }
            const double sh = sin(0.5 * w * t);
            double re = 2.0 * sh * sh / w;  // (1 - cos wt) / w
            if (a.kT > 0.0) re /= tanh(w / (2.0 * a.kT));
            const double im = sin_minus_id(w * t) / w;
            const double f = wq * jw * (1.0 / M_PI);
            neumaier(sr, cr, f * re);
            neumaier(si, ci, f * im);
        }
    }
    const double2 r = block_sum_compensated(sr, cr, si, ci);
    if (threadIdx.x == 0) g[j] = r;
}

// ------------------------------------------------------------ setup tables
// Influence factor F_eta(o, p) = exp(-(s_a - s_b)(eta s_c - conj(eta) s_d))
// for the later point o = (a, b) and the earlier point p = (c, d).
__device__ double2 influence(const double *s, int M, int o, int p, double2 eta) {
    const int a = o / M, b = o % M, c = p / M, d = p % M;
    const double del = s[a] - s[b];
    const double zr = -del * eta.x * (s[c] - s[d]);
    const double zi = -del * eta.y * (s[c] + s[d]);
    double sn, cs;
    sincos(zi, &sn, &cs);
    const double e = exp(zr);
    return make_double2(e * cs, e * sn);
}

// U = exp(-i H dt) by scaling and squaring of the Taylor series (degree 20 on
// a matrix of 1-norm <= 1/4, then repeated squaring).  One thread; M <= 4.
__device__ void expm_minus_i_h_dt(const double2 *H, int M, double dt, double2 *U) {
    double2 A[kMaxM * kMaxM], T[kMaxM * kMaxM], term[kMaxM * kMaxM], tmp[kMaxM * kMaxM];
    const int MM = M * M;
    double norm = 0.0;
    for (int i = 0; i < MM; ++i) A[i] = make_double2(H[i].y * dt, -H[i].x * dt);  // -i H dt
    for (int c = 0; c < M; ++c) {
        double col = 0.0;
        for (int r = 0; r < M; ++r) col += hypot(A[r * M + c].x, A[r * M + c].y);
        norm = fmax(norm, col);
    }
    int sq = 0;
    while (norm > 0.25) {
        norm *= 0.5;
        ++sq;
    }
    const double scale = ldexp(1.0, -sq);
    for (int i = 0; i < MM; ++i) {
        A[i].x *= scale;
        A[i].y *= scale;
        T[i] = term[i] = make_double2((i / M) == (i % M) ? 1.0 : 0.0, 0.0);
    }
    for (int k = 1; k <= 20; ++k) {
        const double inv = 1.0 / k;
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) {
                double2 acc = make_double2(0.0, 0.0);
                for (int x = 0; x < M; ++x) cmac(acc, term[r * M + x], A[x * M + c]);
                tmp[r * M + c] = make_double2(acc.x * inv, acc.y * inv);
            }
        for (int i = 0; i < MM; ++i) {
            term[i] = tmp[i];
            T[i].x += term[i].x;
            T[i].y += term[i].y;
        }
    }
    for (int k = 0; k < sq; ++k) {
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) {
                double2 acc = make_double2(0.0, 0.0);
                for (int x = 0; x < M; ++x) cmac(acc, T[r * M + x], T[x * M + c]);
                tmp[r * M + c] = acc;
            }
        for (int i = 0; i < MM; ++i) T[i] = tmp[i];
    }
    for (int i = 0; i < MM; ++i) U[i] = T[i];
}

// Trace-exact FP32 representatives of the propagator's diagonal rows.  The
// trace of rho is kept by the propagation because every influence factor of a
// diagonal point o = (a, a) is 1 and, by unitarity of U, the K entries of the
// diagonal rows sum to delta_cd over a for every column p = (c, d).  Rounding
// each entry to FP32 on its own breaks that sum by a fixed amount that then
// acts at every step (a linear trace drift).  Here, for each column and each
// of the real and imaginary parts, the entries other than the largest one are
// rounded to the FP32 spacing of the largest, and the largest is set to the
// target minus their sum; all of them are then exact FP32 values whose sum is
// exactly the target (up to the largest leaving its binade).  Change per entry:
// at most half an FP32 spacing of the column's largest entry.
__device__ void trace_exact_column(const double2 *U, int M, int c, int d, double2 *out) {
    double2 v[kMaxM];
    for (int q = 0; q < M; ++q) {
        const double2 u2 = U[q * M + d];
        v[q] = cmul(U[q * M + c], make_double2(u2.x, -u2.y));
    }
    for (int part = 0; part < 2; ++part) {
        const double target = (part == 0 && c == d) ? 1.0 : 0.0;
        int big = 0;
        for (int q = 1; q < M; ++q)
            if (fabs(part ? v[q].y : v[q].x) > fabs(part ? v[big].y : v[big].x)) big = q;
        const double vb = fabs(part ? v[big].y : v[big].x);
        double w[kMaxM];
        if (vb == 0.0) {
            for (int q = 0; q < M; ++q) w[q] = 0.0;
        } else {
            const double grid = ldexp(1.0, ilogb(vb) - 23);   // FP32 spacing in the binade of vb
            double rest = 0.0;
            for (int q = 0; q < M; ++q) {
                if (q == big) continue;
                w[q] = rint((part ? v[q].y : v[q].x) / grid) * grid;
                rest += w[q];
            }
            w[big] = target - rest;
        }
        for (int q = 0; q < M; ++q) {
            if (part) out[q].y = w[q];
            else out[q].x = w[q];
        }
    }
}

__global__ void __launch_bounds__(kBlock) tables_kernel(const TablesArgs a) {
    __shared__ double2 sU[kMaxM * kMaxM];
    __shared__ double2 sEta[4 * kMaxL + 2];
    __shared__ double sS[kMaxM];
    __shared__ double2 sKd[kMaxM * kMaxM * kMaxM];    // [a][p]: K[(a, a)][p], trace-exact
    const int M = a.M, N = M * M, NN = N * N, L = a.L;
    const int t = threadIdx.x;
    if (t < M * M) sU[t] = a.U_given[t];
    if (t < M) sS[t] = a.s[t];
    // eta classes from g_j = G(j dt/2) (second differences of G over the
    // intervals [0, dt/2], [k dt - dt/2, k dt + dt/2] and [n dt - dt/2, n dt])
    const double2 *g = a.g;
    for (int c = t; c < 4 * L + 2; c += kBlock) {
        double2 v;
        if (c == 0) {
            v = g[2];                                    // interior self pair
        } else if (c == 1) {
            v = g[1];                                    // initial / final self pair
        } else {
            const int cls = (c - 2) / L, D = (c - 2) % L + 1;
            if (cls == 0) {                              // interior pair, lag D
                v = make_double2(g[2 * D + 2].x - 2.0 * g[2 * D].x + g[2 * D - 2].x,
                                 g[2 * D + 2].y - 2.0 * g[2 * D].y + g[2 * D - 2].y);
            } else if (cls == 1 || cls == 2) {           // interior k=D with point 0; final with lag D
                v = make_double2(g[2 * D + 1].x - g[2 * D].x - g[2 * D - 1].x + g[2 * D - 2].x,
                                 g[2 * D + 1].y - g[2 * D].y - g[2 * D - 1].y + g[2 * D - 2].y);
            } else {                                     // final point n=D with point 0
                v = make_double2(g[2 * D].x - 2.0 * g[2 * D - 1].x + g[2 * D - 2].x,
                                 g[2 * D].y - 2.0 * g[2 * D - 1].y + g[2 * D - 2].y);
            }
        }
        sEta[c] = v;
        if (!a.k_only) a.eta[c] = v;
    }
    __syncthreads();
    if (t < M * M && !a.k_only) a.U[t] = sU[t];
    if (a.k_trace_exact && t < N) {
        double2 col[kMaxM];
        trace_exact_column(sU, M, t / M, t % M, col);
        for (int q = 0; q < M; ++q) sKd[q * N + t] = col[q];
    }
    __syncthreads();
    const BankLayout B{L};
    const double2 e_self_int = sEta[0], e_self_end = sEta[1];
    auto lag = [&](int D) { return sEta[1 + D]; };
    auto init = [&](int k) { return sEta[1 + L + k]; };
    auto fin = [&](int D) { return sEta[1 + 2 * L + D]; };
    auto fin_init = [&](int n) { return sEta[1 + 3 * L + n]; };
    const int n_tab = B.count();
    // the tables that carry K: K itself, K folded into the lag-1 classes, and
    // the oldest-point tables when L = 1 (their oldest point is the previous one)
    auto carries_k = [&](int tb) {
        return tb == B.K() || tb == B.k_lag1() || tb == B.k_init1() || tb == B.k_fin1() ||
               tb == B.k_fin_init1() || (L == 1 && tb >= B.old_main() && tb <= B.oldf_first());
    };
    for (int idx = t; idx < n_tab * NN; idx += kBlock) {
        const int tb = idx / NN, o = (idx / N) % N, p = idx % N;
        if (a.k_only && !carries_k(tb)) continue;
        const int oa = o / M, ob = o % M, pc = p / M, pd = p % M;
        const double2 Kop = [&] {
            if (a.k_trace_exact && oa == ob) return sKd[oa * N + p];
            const double2 u1 = sU[oa * M + pc], u2 = sU[ob * M + pd];
            return cmul(u1, make_double2(u2.x, -u2.y));   // U[a][c] conj(U[b][d])
        }();
        const double2 one = make_double2(1.0, 0.0);
        double2 v;
        if (tb == B.K()) v = Kop;
        else if (tb <= L) v = influence(sS, M, o, p, lag(tb));
        else if (tb <= 2 * L) v = influence(sS, M, o, p, init(tb - L));
        else if (tb <= 3 * L) v = influence(sS, M, o, p, fin(tb - 2 * L));
        else if (tb <= 4 * L) v = influence(sS, M, o, p, fin_init(tb - 3 * L));
        else if (tb == B.self_int()) v = influence(sS, M, o, o, e_self_int);
        else if (tb == B.self_end()) v = influence(sS, M, o, o, e_self_end);
        else if (tb == B.k_lag1()) v = cmul(Kop, influence(sS, M, o, p, lag(1)));
        else if (tb == B.k_init1()) v = cmul(Kop, influence(sS, M, o, p, init(1)));
        else if (tb == B.k_fin1()) v = cmul(Kop, influence(sS, M, o, p, fin(1)));
        else if (tb == B.k_fin_init1()) v = cmul(Kop, influence(sS, M, o, p, fin_init(1)));
        else {
            const bool final_cls = (tb == B.oldf_main() || tb == B.oldf_first());
            const bool first = (tb == B.old_first() || tb == B.oldf_first());
            const double2 self = influence(sS, M, o, o, final_cls ? e_self_end : e_self_int);
            const double2 e = final_cls ? (first ? fin_init(L) : fin(L)) : (first ? init(L) : lag(L));
            v = cmul(self, influence(sS, M, o, p, e));
            v = cmul(v, L == 1 ? Kop : one);
        }
        a.bank[idx] = v;
        if (a.bank_f) a.bank_f[idx] = make_float2((float)v.x, (float)v.y);
    }
}

template <typename C>
__global__ void init_tensor_kernel(const double2 *rho0, const double2 *self_end, C *a0, int N) {
    const int o = threadIdx.x;
    if (o < N) a0[o] = from_d2<C>(cmul(rho0[o], self_end[o * N]));
}

// ------------------------------------------------------- propagation step
// LDS layout of a step block (host and device agree through this function).
struct StepLds {
    unsigned old, oldf, tq, tqf, plo, plof, phi, red, total;
};
__host__ __device__ inline StepLds step_lds_layout(int N, int csize, bool rho, int I, int R, int Q,
                                                   bool plo_reg) {
    StepLds l;
    unsigned off = 0;
    l.old = lds_take(off, plo_reg ? N * I * csize : 0);
    l.oldf = lds_take(off, (plo_reg && rho) ? N * I * csize : 0);
    l.tq = lds_take(off, N * Q * csize);
    l.tqf = lds_take(off, rho ? N * Q * csize : 0);
    l.plo = lds_take(off, plo_reg ? 0 : N * R * csize);
    l.plof = lds_take(off, (plo_reg || !rho) ? 0 : N * R * 16);
    l.phi = lds_take(off, 2 * N * 16);
    l.red = lds_take(off, rho ? (kBlock / 64) * N * 16 : 0);
    l.total = off;
    return l;
}

// Product over nd digits of v (base N, least significant first) of the bank
// tables tab[j0 + j], row o.
template <int N>
__device__ double2 digit_product(const double2 *__restrict__ bank, const int16_t *tab, int j0, int nd,
                                 long long v, int o, double2 p) {
    for (int j = 0; j < nd; ++j) {
        const int dg = (int)(v % N);
        v /= N;
        p = cmul(p, bank[(size_t)tab[j0 + j] * (N * N) + o * N + dg]);
    }
    return p;
}

// One propagation step.  Output entry (m, o), o the new point's index and m the
// digits of the kept window points:
//   A_out[m + m_count*o] = P(o, m) * sum_{i<I} Old[o][i] * A_in[i + I*m]
// with P(o, m) = prod_j Tab_j[o][digit_j(m)].  I = N sums out the oldest point
// (full window); I = 1 is a growth step (window not yet full).  With RHO the
// same loaded values also give rho(t_n)[o] = sum_m Pfin(o,m) sum_i OldFin[o][i] A_in[i + I*m]
// (final-point classes), reduced per block into partials[blockIdx][o] and
// summed across blocks by rho_finalize_kernel.
//
// Digits of m: the low d_lo digits are fixed per thread (product in
// registers or LDS), the next d_mid digits are swept by the thread's loop
// (products tabulated in LDS per block), the rest are the block index
// (product computed once per block).  Consecutive threads own consecutive m,
// so each thread reads I contiguous values and every o-plane store is
// coalesced.  For N <= 4 each thread keeps two items in flight.
//
// S is the storage scalar of the tensor and T the arithmetic scalar: double /
// double (complex128), float / float (complex64 tier), float / double
// (complex64 storage, each loaded value widened and every product in FP64).
//
// MODE 1, 2, 3 (mirror mode, full-window steps at N = 4 and 9): as in the
// N = 16 MFMA step, with the mirror of digit o = Ma + b -> Mb + a: mode 1 the
// blocks whose high digits are below their mirror; mode 2 those with all
// high digits diagonal, the items below their mirror; mode 3 the items whose
// digits are all diagonal (threads whose low digits are diagonal, sweep rows
// whose digits are), which read their input slots above the mirror from the
// mirrored slot, conjugated.  Outputs above their mirror are stored as the
// conjugate at the mirrored address; each block adds the mirrored items' rho
// terms as S[o] + conj(S[mirror(o)]) (modes 1, 2).
template <int N>
struct MirrorDigits {
    static constexpr int M = N == 4 ? 2 : N == 9 ? 3 : 4;
    static __host__ __device__ constexpr int digit(int d) { return M * (d % M) + d / M; }
    static __device__ long long index(long long x) { return N == 4 ? mirror4(x) : mirror9(x); }
    // the mirror of a small index (few digits), in 32-bit arithmetic
    static __device__ int index_small(int x) {
        if (N == 4) return (int)mirror4(x);
        int out = 0, w = 1;
        for (; x > 0; x /= N, w *= N) out += digit(x % N) * w;
        return out;
    }
    static __device__ bool diagonal_only(int v) {          // every digit a (M + 1)
        for (; v > 0; v /= N)
            if (v % N % (M + 1) != 0) return false;
        return true;
    }
    static __device__ int diagonal(int x) {                // base-M digit a -> base-N digit a (M + 1)
        int out = 0, w = 1;
        for (; x > 0; x /= M, w *= N) out += (M + 1) * (x % M) * w;
        return out;
    }
};
template <int N, typename S, typename T, bool RHO, bool GROW, int MODE = 0>
__global__ void __launch_bounds__(kBlock) step_kernel(const StepArgs a) {
    static_assert(MODE == 0 || ((N == 4 || N == 9) && !GROW), "mirror mode: full-window N = 4, 9 steps");
    using MD = MirrorDigits<N == 9 ? 9 : 4>;
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    constexpr int I = GROW ? 1 : N;
    // FP32 arithmetic, full-window N = 4, 9: the diagonal rows' sums compensated
    constexpr bool TRACE_ROWS = sizeof(T) == 4 && !GROW && (N == 4 || N == 9);
    constexpr bool PLO_REG = (N <= 4);
    constexpr bool OLD_REG = (N <= 4);
    constexpr int ILP = (N <= 4) ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int R = a.R, Q = a.Q;
    const StepLds lay = step_lds_layout(N, (int)sizeof(C), RHO, I, R, Q, PLO_REG);
    C *s_old = (C *)(smem + lay.old);
    C *s_oldf = (C *)(smem + lay.oldf);
    C *s_tq = (C *)(smem + lay.tq);
    C *s_tqf = (C *)(smem + lay.tqf);
    C *s_plo = (C *)(smem + lay.plo);
    double2 *s_plof = (double2 *)(smem + lay.plof);
    double2 *s_phi = (double2 *)(smem + lay.phi);
    double2 *s_red = (double2 *)(smem + lay.red);

    const int t = threadIdx.x;
    const int cR = kBlock / R;       // sweep stride in units of R
    const int active = cR * R;       // threads that own items
    const double2 *__restrict__ bank = a.bank;
    // N = 9, mode 1: blocks below n_canon run the canonical high-digit values,
    // the rest the listed items of the values equal to their mirror
    constexpr bool kListed = N == 9 && MODE == 1;
    const bool listed = kListed && (int)blockIdx.x >= a.n_canon;
    const int lblk = listed ? (int)blockIdx.x - a.n_canon : 0;
    const long long blk = MODE == 0   ? (long long)blockIdx.x
                          : listed    ? (long long)a.blk_hi[a.n_canon + lblk / a.parts]
                          : MODE == 2 ? (long long)a.blk_hi[blockIdx.x / a.parts]
                                      : (long long)a.blk_hi[blockIdx.x];     // high digits
    const double2 one = make_double2(1.0, 0.0);
    const bool planned = a.t_lo != nullptr;
    const int j_hi = a.d_lo + a.d_mid;

    // Block constants (FP64): high-digit products and the oldest-point tables.
    if (t < N) {
        double2 ph, phf = one;
        if (planned) {
            ph = a.t_hi[(size_t)t * a.grid + blk];
            if (RHO) phf = a.t_hif[(size_t)t * a.grid + blk];
        } else {
            ph = digit_product<N>(bank, a.tab, j_hi, a.n_digits - j_hi, blk, t, one);
            if (RHO) phf = digit_product<N>(bank, a.tabf, j_hi, a.n_digits - j_hi, blk, t, one);
        }
        s_phi[t] = ph;
        s_phi[N + t] = phf;
    }
    for (int idx = t; OLD_REG && idx < N * I; idx += kBlock) {
        const int o = idx / I, i = idx % I;
        s_old[idx] = from_d2<C>(bank[(size_t)a.old_tab * (N * N) + o * N + i]);
        if (RHO) s_oldf[idx] = from_d2<C>(bank[(size_t)a.oldf_tab * (N * N) + o * N + i]);
    }
    // N >= 9: the oldest-point tables are read per use by scalar loads from
    // the bank in the compute precision (wave-uniform operands of the FMAs).
    const T *old_c = (const T *)a.bank_c + 2 * (size_t)a.old_tab * (N * N);
    const T *oldf_c = (const T *)a.bank_c + 2 * (size_t)a.oldf_tab * (N * N);
    if (!PLO_REG) {
        for (int idx = t; idx < N * R; idx += kBlock) {
            const int o = idx / R, v = idx % R;
            s_plo[idx] = from_d2<C>(planned ? a.t_lo[idx] : digit_product<N>(bank, a.tab, 0, a.d_lo, v, o, one));
            if (RHO) s_plof[idx] = planned ? a.t_lof[idx] : digit_product<N>(bank, a.tabf, 0, a.d_lo, v, o, one);
        }
    }
    __syncthreads();
    // Mid-digit products times the block's high-digit product, cast once to C.
    for (int idx = t; idx < N * Q; idx += kBlock) {
        const int o = idx / Q, v = idx % Q;
        const double2 mid = planned ? a.t_mid[idx] : digit_product<N>(bank, a.tab, a.d_lo, a.d_mid, v, o, one);
        s_tq[idx] = from_d2<C>(cmul(s_phi[o], mid));
        if (RHO) {
            const double2 midf = planned ? a.t_midf[idx] : digit_product<N>(bank, a.tabf, a.d_lo, a.d_mid, v, o, one);
            s_tqf[idx] = from_d2<C>(cmul(s_phi[N + o], midf));
        }
    }
    // Low-digit products of this thread's fixed digits.
    const int r = t % R;
    C plo[PLO_REG ? N : 1];
    double2 plof[PLO_REG ? N : 1];
    if (PLO_REG) {
#pragma unroll
        for (int o = 0; o < N; ++o) {
            plo[o] = from_d2<C>(planned ? a.t_lo[o * R + r] : digit_product<N>(bank, a.tab, 0, a.d_lo, r, o, one));
            plof[o] = RHO ? (planned ? a.t_lof[o * R + r] : digit_product<N>(bank, a.tabf, 0, a.d_lo, r, o, one)) : one;
        }
    }
    __syncthreads();
    C old_r[OLD_REG ? N * I : 1];
    C oldf_r[(OLD_REG && RHO) ? N * I : 1];
    if (OLD_REG) {
#pragma unroll
        for (int k = 0; k < N * I; ++k) {
            old_r[k] = s_old[k];
            if (RHO) oldf_r[k] = s_oldf[k];
        }
    }

    double2 acc[RHO ? N : 1];
#pragma unroll
    for (int o = 0; o < (RHO ? N : 1); ++o) acc[o] = make_double2(0.0, 0.0);

    if (t < active) {
        const long long m0 = blk * (long long)R * Q;
        const CS *__restrict__ ain = (const CS *)a.a_in;
        CS *__restrict__ aout = (CS *)a.a_out;
        const long long mc = a.m_count;
        // the mirror acts digit by digit, and m = (blk, qm, r) splits into whole
        // digits, so mirror(m) = mirror(blk) R Q + mirror(qm) R + mirror(r):
        // the block and thread parts once, the sweep part per item in 32-bit
        // arithmetic, instead of a 64-bit digit loop per item (N = 9)
        const long long mbh = MODE == 0 ? 0 : MD::index(blk) * (long long)R * Q;
        const int r_mir = MODE == 0 ? 0 : MD::index_small(r);
        auto mirror_of = [&](int qm, int rr) {
            return mbh + (long long)MD::index_small(qm) * R + (listed ? MD::index_small(rr) : r_mir);
        };
        // sweep rows: all (mode 0, 1), a part (mode 2), or in mode 3 those with
        // all digits diagonal, for threads whose low digits are diagonal; a
        // listed block (N = 9) walks its part of the list of the items below
        // their mirror (qm * R + r, the same for every diagonal high value),
        // one item per active thread
        const int part = listed ? lblk % a.parts : MODE == 2 ? (int)(blockIdx.x % a.parts) : 0;
        const bool thread_runs = MODE != 3 || MD::diagonal_only(r);
        int n_diag_rows = 1;
        if (MODE == 3)
            for (int q = Q; q > 1; q /= N) n_diag_rows *= MD::M;
        const int i0 = listed ? part * a.q_span + t : (MODE == 2 ? part * a.q_span : 0) + t / R;
        const int i1 = !thread_runs ? 0
                       : MODE == 3  ? n_diag_rows
                       : listed     ? min(a.n_low, (part + 1) * a.q_span)
                       : MODE == 2  ? min(Q, (part + 1) * a.q_span)
                                    : Q;
        const int istride = listed ? active : cR;
        static_assert(!kListed || ILP == 1, "listed items: one item per thread and pass");
        for (int qm0 = i0; qm0 < i1; qm0 += ILP * istride) {
            // For N >= 9 the N*N table reads must stay in the loop: hoisted as
            // loop invariants they would need more registers than a thread has.
            if (!OLD_REG) asm volatile("" ::: "memory");
            C x[ILP][I];
            bool has[ILP];
            const int low = listed ? a.low_list[qm0] : 0;       // listed: one item (ILP = 1)
            const int rr = listed ? low % R : r;
#pragma unroll
            for (int u = 0; u < ILP; ++u) {      // issue every load first
                const int it = qm0 + u * istride;
                const int qm = MODE == 3 ? MD::diagonal(it) : listed ? low / R : it;
                const long long m = m0 + (long long)qm * R + rr;
                has[u] = it < i1 && (MODE != 2 || m < mirror_of(qm, rr));
                if (has[u]) {
#pragma unroll
                    for (int i = 0; i < I; ++i) {
                        // a self-mirror item holds valid values only at the slots
                        // not above their mirror
                        constexpr bool fix = MODE == 3;
                        const int ib = MODE == 3 ? MD::digit(i) : i;
                        x[u][i] = conv<C>(ain[(long long)I * m + (fix && ib < i ? ib : i)]);
                        if (fix && ib < i) x[u][i].y = -x[u][i].y;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < ILP; ++u) {
                if (!has[u]) continue;
                const int it = qm0 + u * istride;
                const int qm = MODE == 3 ? MD::diagonal(it) : listed ? low / R : it;
                const long long m = m0 + (long long)qm * R + rr;
                const long long mb = MODE == 0 ? m : mirror_of(qm, rr);
#pragma unroll
                for (int o = 0; o < N; ++o) {
                    if (!OLD_REG) asm volatile("" ::: "memory");   // table reads of this o only
                    const C p = cmul(PLO_REG ? plo[o] : s_plo[o * R + rr], s_tq[o * Q + qm]);
                    C v;
                    if (TRACE_ROWS && o % (MD::M + 1) == 0 && a.n_digits > 0) {
                        // a diagonal point with L >= 2: its oldest-point row is
                        // ones and p is K[o, m_last]; the sum stays unrounded
                        // until the product (these rows carry the trace)
                        TraceSum<C> ts;
                        ts.init(x[u][0]);
#pragma unroll
                        for (int i = 1; i < I; ++i) ts.add(x[u][i]);
                        v = ts.times_right(p);
                    } else {
                        C s = {};
#pragma unroll
                        for (int i = 0; i < I; ++i)
                            cmac(s, OLD_REG ? old_r[o * I + i] : coef_ld(old_c, o * N + i), x[u][i]);
                        v = cmul(s, p);
                    }
                    if (MODE == 0 || MD::digit(o) >= o) {
                        aout[m + mc * o] = conv<CS>(v);
                    } else if (MODE != 3) {
                        C vc = v;
                        vc.y = -vc.y;
                        aout[mb + mc * MD::digit(o)] = conv<CS>(vc);
                    }
                    if (RHO) {
                        if (!OLD_REG) asm volatile("" ::: "memory");
                        C sf = {};
#pragma unroll
                        for (int i = 0; i < I; ++i)
                            cmac(sf, OLD_REG ? oldf_r[o * I + i] : coef_ld(oldf_c, o * N + i), x[u][i]);
                        double2 v = to_d2(cmul(sf, s_tqf[o * Q + qm]));
                        // a listed item has its own low digits: their factor per item
                        if (kListed && listed) v = cmul(v, s_plof[o * R + rr]);
                        acc[o].x += v.x;
                        acc[o].y += v.y;
                    }
                }
            }
        }
    }
    if (RHO) {
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int o = 0; o < N; ++o) {
            double2 v = make_double2(0.0, 0.0);
            if (t < active) v = listed ? acc[o] : cmul(acc[o], PLO_REG ? plof[o] : s_plof[o * R + r]);
            for (int off = 32; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
            }
            if (lane == 0) s_red[wave * N + o] = v;
        }
        __syncthreads();
        if (t < N) {
            double2 s = make_double2(0.0, 0.0);
            for (int w = 0; w < kBlock / 64; ++w) {
                s.x += s_red[w * N + t].x;
                s.y += s_red[w * N + t].y;
            }
            if (MODE == 1 || MODE == 2) {               // the mirrored items' terms
                const int tb = MD::digit(t);
                for (int w = 0; w < kBlock / 64; ++w) {
                    s.x += s_red[w * N + tb].x;
                    s.y -= s_red[w * N + tb].y;
                }
            }
            a.partials[((size_t)a.part_base + (MODE == 0 ? blk : (long long)blockIdx.x)) * N + t] = s;
        }
    }
}

// rho(t_n)[o] = sum over the step's block partials, compensated, in a fixed
// order, in two launches on the side stream (each launch boundary makes the
// previous writes visible without device-scope fences):
//   rho_slice_kernel   kSlices blocks; block b sums rows [b*rows/kSlices,
//                      (b+1)*rows/kSlices) -- thread t takes rows t, t+kBlock, ...
//                      with Neumaier sums, then a fixed two-sum tree -- and
//                      writes a (sum, compensation) pair per o;
//   rho_final_kernel   one block combines the kSlices pairs in a fixed tree and
//                      writes rho to sink->base + sink->count * N, then advances
//                      sink->count (so a captured graph can replay it unchanged).
constexpr int kSlices = kRhoSlices;
template <int N>
__global__ void __launch_bounds__(kBlock) rho_slice_kernel(const double2 *__restrict__ partials, int rows,
                                                            double2 *__restrict__ pairs) {
    const int t = threadIdx.x;
    const int b = blockIdx.x;
    const long long r0 = (long long)rows * b / kSlices, r1 = (long long)rows * (b + 1) / kSlices;
    if constexpr (N >= 9) {
        // one point o per thread and kBlock / N row lanes: a row's N values
        // are read by N neighbouring threads, and each thread keeps one pair
        // of compensated sums; the lanes of a point are then combined in
        // lane order by one thread
        constexpr int RL = kBlock / N;
        __shared__ double s_p[4][kBlock];
        const int o = t % N, lane_r = t / N;
        double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
        if (lane_r < RL) {
            for (long long r = r0 + lane_r; r < r1; r += RL) {
                const double2 v = partials[(size_t)r * N + o];
                neumaier(sr, cr, v.x);
                neumaier(si, ci, v.y);
            }
        }
        s_p[0][t] = sr;
        s_p[1][t] = cr;
        s_p[2][t] = si;
        s_p[3][t] = ci;
        __syncthreads();
        if (t < N) {
            for (int k = 1; k < RL; ++k) {
                const int u = k * N + t;
                two_sum_combine(sr, cr, s_p[0][u], s_p[1][u]);
                two_sum_combine(si, ci, s_p[2][u], s_p[3][u]);
            }
            pairs[((size_t)b * N + t) * 2] = make_double2(sr, si);
            pairs[((size_t)b * N + t) * 2 + 1] = make_double2(cr, ci);
        }
        return;
    }
    constexpr int U = N >= 16 ? 1 : 16 / N;   // rows in flight per thread
    double sr[N], cr[N], si[N], ci[N];
#pragma unroll
    for (int o = 0; o < N; ++o) sr[o] = cr[o] = si[o] = ci[o] = 0.0;
    long long r = r0 + t;
    for (; r + (long long)(U - 1) * kBlock < r1; r += (long long)U * kBlock) {
        double2 v[U][N];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int o = 0; o < N; ++o) v[u][o] = partials[(size_t)(r + (long long)u * kBlock) * N + o];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int o = 0; o < N; ++o) {
                neumaier(sr[o], cr[o], v[u][o].x);
                neumaier(si[o], ci[o], v[u][o].y);
            }
    }
    for (; r < r1; r += kBlock) {
#pragma unroll
        for (int o = 0; o < N; ++o) {
            const double2 v = partials[(size_t)r * N + o];
            neumaier(sr[o], cr[o], v.x);
            neumaier(si[o], ci[o], v.y);
        }
    }
#pragma unroll
    for (int o = 0; o < N; ++o) {
        double a0 = sr[o], a1 = cr[o], a2 = si[o], a3 = ci[o];
        block_reduce_pairs<kBlock>(a0, a1, a2, a3);
        if (t == 0) {
            pairs[((size_t)b * N + o) * 2] = make_double2(a0, a2);
            pairs[((size_t)b * N + o) * 2 + 1] = make_double2(a1, a3);
        }
    }
}

template <int N>
__global__ void __launch_bounds__(kSlices) rho_final_kernel(const double2 *__restrict__ pairs, RhoSink *sink) {
    const int t = threadIdx.x;
    double2 *out = nullptr;
    unsigned long long count = 0;
    if (t == 0) {
        count = sink->count;
        out = sink->base + count * N;
    }
#pragma unroll
    for (int o = 0; o < N; ++o) {
        const double2 sv = pairs[((size_t)t * N + o) * 2], cv = pairs[((size_t)t * N + o) * 2 + 1];
        double a0 = sv.x, a1 = cv.x, a2 = sv.y, a3 = cv.y;
        block_reduce_pairs<kSlices>(a0, a1, a2, a3);
        if (t == 0) out[o] = make_double2(a0 + a1, a2 + a3);
    }
    if (t == 0) sink->count = count + 1;
}

__global__ void set_sink_kernel(RhoSink *sink, double2 *base) {
    if (threadIdx.x == 0) {
        sink->base = base;
        sink->count = 0;
    }
}

// Factor products of the full-window digit split: t_lo[o][v] over digits
// 0..d_lo-1, t_mid[o][v] over d_lo..d_lo+d_mid-1, t_hi[o][v] over the rest,
// interior (tab) and final-point (tabf) classes.  Step-independent for n > L.
__global__ void __launch_bounds__(kBlock) plan_tables_kernel(const PlanArgs a) {
    const int N = a.N;
    const long long n_lo = (long long)N * a.R, n_mid = (long long)N * a.Q, n_hi = (long long)N * a.grid;
    const long long total = n_lo + n_mid + n_hi;
    const double2 one = make_double2(1.0, 0.0);
    for (long long idx = (long long)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * kBlock) {
        long long k, v;
        int o, j0, nd, width;
        double2 *out, *outf;
        if (idx < n_lo) {
            k = idx; width = a.R; j0 = 0; nd = a.d_lo; out = a.t_lo; outf = a.t_lof;
        } else if (idx < n_lo + n_mid) {
            k = idx - n_lo; width = a.Q; j0 = a.d_lo; nd = a.d_mid; out = a.t_mid; outf = a.t_midf;
        } else {
            k = idx - n_lo - n_mid; width = a.grid; j0 = a.d_lo + a.d_mid; nd = a.n_digits - j0;
            out = a.t_hi; outf = a.t_hif;
        }
        o = (int)(k / width);
        v = k % width;
        double2 p = one, pf = one;
        for (int j = 0; j < nd; ++j) {
            const int dg = (int)(v % N);
            v /= N;
            p = cmul(p, a.bank[(size_t)a.tab[j0 + j] * (N * N) + o * N + dg]);
            pf = cmul(pf, a.bank[(size_t)a.tabf[j0 + j] * (N * N) + o * N + dg]);
        }
        out[k] = p;
        outf[k] = pf;
    }
}

// ------------------------------------ full-window step on MFMA (N = 16)
// For N = 16 the contraction over the oldest point is a 16 x 16 complex matrix
// (32 x 16 with the final-point table for rho) applied to every item's 16
// inputs: a real GEMM with 64 rows (Re / Im of each output, interior and final
// tables), K = 32 (the item's 32 real words in memory order) and one column per
// item.  A wave runs it on 16 items at a time with 16x16x4 MFMAs (FP32 for the
// complex64 tier, FP64 otherwise): the coefficients are per-lane A fragments
// kept in registers for the whole block (in LDS, read per item group, in the
// rho form, which has twice as many), the inputs are B fragments loaded
// straight from HBM, and each lane's accumulators hold 4 outputs of one item.
// Class form (cls_on): the oldest-point row of o is F_self(o) times an
// influence row that depends on o only through s_a - s_b, so outputs of equal
// s_a - s_b share one contraction; the rows are then the distinct influence
// rows a lane group needs, two per table (class slots 0, 1), in half the
// blocks (one interior, one final point), and the self factors move into the
// per-output multipliers.
//
// MFMA 16x16x4 lane layout (wave64): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k; D[i][j] in lane j + 16(i / 4), element i % 4 for f32, and in lane
// j + 16(i % 4), element i / 4 for f64.  The K index of MFMA step s held by
// lane group g = lane / 16 is word 8g + s of the item, so a lane loads 8
// consecutive words (32 B at complex64, 64 B at complex128).
// Rows of row block b (tables: blocks 0, 1 interior, 2, 3 final point) are
// numbered so that lane group g receives, as D elements v = 0..3, the real and
// imaginary parts of outputs o = 8(b % 2) + 2g + v / 2.  Lane j + 16g therefore
// holds outputs o = 2g, 2g+1 (block 0), 8+2g, 9+2g (block 1) of item j, and the
// same four with the final-point table in blocks 2, 3.
//
// MODE 1, 2, 3 (mirror mode, as in the three-step kernel): an entry and its
// mirror (every digit o = 4a + b -> 4b + a) are conjugates, so only the items
// not above their mirror run, each output entry above its mirror is stored as
// the conjugate at the mirrored address, and an item that is its own mirror
// (every digit diagonal) reads its input slots above their mirror from the
// mirrored slot, conjugated.  Mode 1 runs the blocks whose high digits are
// below their mirror; mode 2 those with all high digits diagonal, the items
// below their mirror; mode 3 the items that are their own mirror.  The MFMA
// runs on the whole wave, so a lane whose item does not run feeds zeros and
// stores nothing.  rho: a lane holds outputs of one lane group only, so the
// mirrored item's terms, conj(S[mirror(o)]), are added to each block's sums
// S[o] (modes 1, 2), whose items are never their own mirror.
__device__ __forceinline__ int mirror_digit16(int o) { return ((o & 3) << 2) | (o >> 2); }
template <typename C>
__device__ __forceinline__ C cconj16(C v) {
    v.y = -v.y;
    return v;
}
// Sweep index with all base-16 digits diagonal: base-4 digit d -> 5 d.
__device__ __forceinline__ int diagonal_digits16(int x, int nd) {
    int out = 0;
    for (int k = 0; k < nd; ++k) out += (5 * ((x >> (2 * k)) & 3)) << (4 * k);
    return out;
}
struct Step16Lds {
    unsigned tq, tqf, red, afr, total;
};
// afr_lds: the A fragments in LDS (the rho form without classes)
__host__ __device__ inline Step16Lds step16_lds_layout(int csize, bool rho, int Q, bool afr_lds) {
    Step16Lds l;
    unsigned off = 0;
    l.tq = lds_take(off, 16 * Q * csize);
    l.tqf = lds_take(off, rho ? 16 * Q * csize : 0);
    l.red = lds_take(off, rho ? (kBlock / 64) * 16 * 16 : 0);
    l.afr = lds_take(off, afr_lds ? 4 * 8 * 64 * (csize / 2) : 0);     // A fragments [4][8][lane]
    l.total = off;
    return l;
}

template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
    static constexpr bool kElemMajor = false;       // D row i: group i / 4, element i % 4
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma16<double> {
    static constexpr bool kElemMajor = true;        // D row i: group i % 4, element i / 4
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename S, typename T, bool RHO, int MODE, bool CLS>
__global__ void __launch_bounds__(kBlock, (RHO && MODE <= 1) ? 3 : 1) step16_mfma_kernel(const StepArgs a) {
    constexpr int N = 16, NB = CLS ? (RHO ? 2 : 1) : (RHO ? 4 : 2);
    // A-fragment blocks held in registers; the rest are read from LDS per use
    constexpr int kRegBlocks = !RHO ? NB : !CLS ? 0 : sizeof(T) == 8 ? 1 : NB;
    constexpr bool kAfrLds = kRegBlocks < NB;
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    using V4 = typename Mfma16<T>::v4;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Q = a.Q;                                  // R = 16: one item per lane column
    const Step16Lds lay = step16_lds_layout((int)sizeof(C), RHO, Q, kAfrLds);
    C *s_tq = (C *)(smem + lay.tq);                      // [N][Q] mid x high products
    C *s_tqf = (C *)(smem + lay.tqf);
    double2 *s_red = (double2 *)(smem + lay.red);        // [waves][N]
    T *s_afr = (T *)(smem + lay.afr);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int j = lane & 15, g = lane >> 4;
    const long long blk = MODE == 0   ? (long long)blockIdx.x
                          : MODE == 2 ? (long long)a.blk_hi[blockIdx.x / a.parts]
                                      : (long long)a.blk_hi[blockIdx.x];     // high digits

    for (int idx = t; idx < N * Q; idx += kBlock) {
        const int o = idx / Q;
        s_tq[idx] = from_d2<C>(cmul(a.t_hi[(size_t)o * a.grid + blk], a.t_mid[idx]));
        if (RHO) s_tqf[idx] = from_d2<C>(cmul(a.t_hif[(size_t)o * a.grid + blk], a.t_midf[idx]));
    }
    // A fragments: row 16b + j, word 8g + s; in the rho form those of the
    // final-point table in LDS, read per use, to keep the registers down (all
    // blocks there without classes; the FP32 class form keeps all in registers)
    T afr[kRegBlocks > 0 ? kRegBlocks : 1][8];
    {
        const C *bc = (const C *)a.bank_c;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            // A row j of block b lands in D lane group gd as element vd
            const int gd = Mfma16<T>::kElemMajor ? (j & 3) : (j >> 2);
            const int vd = Mfma16<T>::kElemMajor ? (j >> 2) : (j & 3);
            const int im_row = vd & 1;
            int tb, o;
            if (CLS) {
                // block 0 interior, block 1 final point; class slot vd / 2
                tb = b == 1 ? a.clsf_tab : a.cls_tab;
                o = (int)((a.cls_rep >> (4 * (2 * gd + (vd >> 1)))) & 15u);
            } else {
                tb = b >= 2 ? a.oldf_tab : a.old_tab;
                o = 8 * (b & 1) + 2 * gd + (vd >> 1);
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int w = 8 * g + s, i = w / 2, im_word = w & 1;
                const C c = bc[(size_t)tb * (N * N) + o * N + i];
                // Re z = cr xr - ci xi ; Im z = ci xr + cr xi
                const T v = im_row ? (im_word ? c.x : c.y) : (im_word ? -c.y : c.x);
                if (b < kRegBlocks) afr[b < kRegBlocks ? b : 0][s] = v;
                else if (wave == 0) s_afr[(b * 8 + s) * 64 + lane] = v;
            }
        }
    }
    // per-lane digit-0 products (item j) of its four outputs (with the self
    // factors in the class form)
    // (class form: the host orders each group's outputs so that q = 0, 1
    // take class slot 0 and q = 3 slot 1; only q = 2 is looked up)
    int oo[4] = {2 * g, 2 * g + 1, 8 + 2 * g, 9 + 2 * g};
    bool slot1[4] = {false, false, false, true};
    if (CLS) {
#pragma unroll
        for (int q = 0; q < 4; ++q) oo[q] = (int)((a.cls_out >> (4 * (4 * g + q))) & 15ull);
        slot1[2] = (a.cls_selb >> (4 * g + 2)) & 1u;
    }
    C plo[4];
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double2 lo = a.t_lo[oo[q] * 16 + j];
        if (CLS) lo = cmul(lo, a.bank[(size_t)a.cls_self * (N * N) + oo[q] * N + oo[q]]);
        plo[q] = from_d2<C>(lo);
        acc[q] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    const long long m0 = blk * 16LL * Q;
    const long long mc = a.m_count;
    const S *__restrict__ ain = (const S *)a.a_in;
    CS *__restrict__ aout = (CS *)a.a_out;
    // sweep rows: all (mode 0, 1), a part of them (mode 2), or those whose
    // digits are all diagonal (mode 3)
    const int dm = (31 - __clz(Q)) >> 2;
    const int part = MODE == 2 ? (int)(blockIdx.x % a.parts) : 0;
    const int i0 = (MODE == 2 ? part * a.q_span : 0) + wave;
    const int i1 = MODE == 3 ? (1 << (2 * dm)) : MODE == 2 ? min(Q, (part + 1) * a.q_span) : Q;
    // the item of sweep index it: its index m, its mirror, and whether it runs
    auto item = [&](int it, long long &m, long long &mb) {
        const int qm = MODE == 3 ? diagonal_digits16(it, dm) : it;
        m = m0 + 16LL * qm + j;
        mb = MODE == 0 ? m : mirror16(m);
        return MODE == 0 || MODE == 1 || (MODE == 2 ? m < mb : j % 5 == 0);
    };
    // a lane's 8 input words of the item of sweep index it (as stored;
    // mode 3 converts them, to conjugate the mirrored slots)
    using LW = typename std::conditional<MODE == 3, T, S>::type;
    auto load = [&](int it, LW *xw) {
        long long m, mb;
        const bool run = item(it, m, mb);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            if (MODE == 3) {
                // word 8g + s is part (w & 1) of slot i = w / 2; slots above
                // their mirror come from the mirrored slot, conjugated
                const int w = 8 * g + s, i = w >> 1, ib = mirror_digit16(i);
                const bool flip = ib < i;
                const LW v = run ? (LW)ain[32 * m + (flip ? 2 * ib + (w & 1) : w)] : LW(0);
                xw[s] = flip && (w & 1) ? -v : v;
            } else {
                xw[s] = (MODE != 2 || run) ? (LW)ain[32 * m + 8 * g + s] : LW(0);
            }
        }
    };
    // the inputs of the next PF item groups are loaded before this group's
    // products, so that their latency overlaps the MFMAs; the complex64
    // tiers, whose groups are half as many bytes, load two groups ahead
    constexpr int PF = (MODE == 3 || sizeof(S) == 8) ? 1 : 2;
    constexpr int kStride = kBlock / 64;
    // Group k of the wave's sweep sits in buffer k % (PF + 1); at FP64 the
    // loop is unrolled over the PF + 1 buffers so that no buffer is copied
    // (M = 4, L = 7, complex128 rho step 0.970 -> 0.924 ms).
    LW xb[PF + 1][8];
#pragma unroll
    for (int k = 0; k < PF; ++k)
        if (i0 + k * kStride < i1) load(i0 + k * kStride, xb[k]);
    auto group = [&](int it, const LW *xs) {
        T xw[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) xw[s] = (T)xs[s];
        const int qm = MODE == 3 ? diagonal_digits16(it, dm) : it;
        long long m, mb;
        const bool run = item(it, m, mb);
        V4 d[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) d[b] = V4{0, 0, 0, 0};
        if (kAfrLds) asm volatile("" ::: "memory");   // the LDS fragments are read here, per item group
#pragma unroll
        for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                d[b] = Mfma16<T>::run(b < kRegBlocks ? afr[b < kRegBlocks ? b : 0][s] : s_afr[(b * 8 + s) * 64 + lane],
                                      xw[s], d[b]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // the contraction of output q: block b, elements e, e + 1
            const int b = CLS ? 0 : q / 2, e = CLS ? 0 : 2 * (q % 2);
            C z;
            if (CLS) {
                z.x = slot1[q] ? d[0][2] : d[0][0];
                z.y = slot1[q] ? d[0][3] : d[0][1];
            } else {
                z.x = d[b][e];
                z.y = d[b][e + 1];
            }
            const C p = cmul(plo[q], s_tq[oo[q] * Q + qm]);
            const C v = cmul(p, z);
            // an output above its mirror goes to the mirrored address as its
            // conjugate; address and value are selected, so that every lane
            // issues one full-width store (branches split it in two)
            const int ob = mirror_digit16(oo[q]);
            const bool direct = MODE == 0 || ob >= oo[q];
            CS *const dst = direct ? aout + m + mc * oo[q] : aout + mb + mc * ob;
            const C val = direct ? v : cconj16(v);
            if (MODE == 0 || MODE == 1 || (run && (MODE == 2 || direct))) *dst = conv<CS>(val);
            if (RHO && run) {
                C zf;
                if (CLS) {
                    zf.x = slot1[q] ? d[NB - 1][2] : d[NB - 1][0];
                    zf.y = slot1[q] ? d[NB - 1][3] : d[NB - 1][1];
                } else {
                    zf.x = d[NB - 2 + b][e];
                    zf.y = d[NB - 2 + b][e + 1];
                }
                const double2 v = to_d2(cmul(s_tqf[oo[q] * Q + qm], zf));
                acc[q].x += v.x;
                acc[q].y += v.y;
            }
        }
    };
    if constexpr (sizeof(T) == 8) {
        for (int base = i0; base < i1; base += (PF + 1) * kStride) {
#pragma unroll
            for (int u = 0; u <= PF; ++u) {
                const int it = base + u * kStride;
                if (it >= i1) break;
                if (it + PF * kStride < i1) load(it + PF * kStride, xb[(u + PF) % (PF + 1)]);
                group(it, xb[u]);
            }
        }
    } else {
        // FP32: the buffers rotate instead (the unrolled form needs more
        // registers, a wave less per SIMD, and was slower: M = 4, L = 7,
        // complex64 rho step 0.524 -> 0.540-0.547 ms)
        for (int it = i0; it < i1; it += kStride) {
            if (it + PF * kStride < i1) load(it + PF * kStride, xb[PF]);
            group(it, xb[0]);
#pragma unroll
            for (int k = 0; k < PF; ++k)
#pragma unroll
                for (int s = 0; s < 8; ++s) xb[k][s] = xb[k + 1][s];
        }
    }
    if (RHO) {
        // sum over the 16 items of the lane group, then over the waves (the
        // digit-0 factors of the final-point table are read here, not held)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double2 plof = a.t_lof[oo[q] * 16 + j];
            if (CLS) plof = cmul(plof, a.bank[(size_t)a.cls_selff * (N * N) + oo[q] * N + oo[q]]);
            double2 v = cmul(acc[q], plof);
            for (int off = 8; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
            }
            if (j == 0) s_red[wave * N + oo[q]] = v;
        }
        __syncthreads();
        if (t < N) {
            double2 s = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
            const int tb = mirror_digit16(t);
            for (int w = 0; w < kBlock / 64; ++w) {
                s.x += s_red[w * N + t].x;
                s.y += s_red[w * N + t].y;
                sb.x += s_red[w * N + tb].x;
                sb.y += s_red[w * N + tb].y;
            }
            if (MODE == 1 || MODE == 2) {
                s.x += sb.x;
                s.y -= sb.y;
            }
            a.partials[((size_t)a.part_base + blockIdx.x) * N + t] = s;
        }
    }
}

template <typename S, typename T, bool RHO, bool CLS>
hipError_t launch_step16_c(const StepArgs &a, int grid, hipStream_t st) {
    using C = typename Cx<T>::type;
    const Step16Lds lay = step16_lds_layout((int)sizeof(C), RHO, a.Q, RHO && (!CLS || sizeof(T) == 8));
    const dim3 b(kBlock);
    switch (a.mode) {
    case 0: hipLaunchKernelGGL((step16_mfma_kernel<S, T, RHO, 0, CLS>), dim3(grid), b, lay.total, st, a); break;
    case 1: hipLaunchKernelGGL((step16_mfma_kernel<S, T, RHO, 1, CLS>), dim3(a.n_blk), b, lay.total, st, a); break;
    case 2: hipLaunchKernelGGL((step16_mfma_kernel<S, T, RHO, 2, CLS>), dim3(a.n_blk), b, lay.total, st, a); break;
    case 3: hipLaunchKernelGGL((step16_mfma_kernel<S, T, RHO, 3, CLS>), dim3(a.n_blk), b, lay.total, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, typename T, bool RHO>
hipError_t launch_step16_t(const StepArgs &a, int grid, hipStream_t st) {
    return a.cls_on ? launch_step16_c<S, T, RHO, true>(a, grid, st) : launch_step16_c<S, T, RHO, false>(a, grid, st);
}

// The MFMA form runs the full-window steps of N = 16 whose thread digit split
// gives 16 items per wave column (R = 16).
__host__ __device__ inline bool use_step16(int N, bool grow, int R) { return N == 16 && !grow && R == 16; }

template <int N, typename S, typename T, bool RHO, bool GROW>
hipError_t launch_step_t(const StepArgs &a, int grid, hipStream_t st) {
    using C = typename Cx<T>::type;
    const StepLds lay = step_lds_layout(N, (int)sizeof(C), RHO, GROW ? 1 : N, a.R, a.Q, N <= 4);
    const dim3 b(kBlock);
    if constexpr ((N == 4 || N == 9) && !GROW) {
        switch (a.mode) {
        case 0: break;
        case 1: hipLaunchKernelGGL((step_kernel<N, S, T, RHO, GROW, 1>), dim3(a.n_blk), b, lay.total, st, a); return hipGetLastError();
        case 2: hipLaunchKernelGGL((step_kernel<N, S, T, RHO, GROW, 2>), dim3(a.n_blk), b, lay.total, st, a); return hipGetLastError();
        case 3: hipLaunchKernelGGL((step_kernel<N, S, T, RHO, GROW, 3>), dim3(a.n_blk), b, lay.total, st, a); return hipGetLastError();
        default: return hipErrorInvalidValue;
        }
    } else {
        if (a.mode != 0) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((step_kernel<N, S, T, RHO, GROW>), dim3(grid), b, lay.total, st, a);
    return hipGetLastError();
}

template <int N, typename S, typename T>
hipError_t launch_step_n(bool rho, bool grow, const StepArgs &a, int grid, hipStream_t st) {
    if (rho)
        return grow ? launch_step_t<N, S, T, true, true>(a, grid, st) : launch_step_t<N, S, T, true, false>(a, grid, st);
    return grow ? launch_step_t<N, S, T, false, true>(a, grid, st) : launch_step_t<N, S, T, false, false>(a, grid, st);
}

template <typename S, typename T>
hipError_t launch_step_dt(int N, bool rho, bool grow, const StepArgs &a, int grid, hipStream_t st) {
    switch (N) {
    case 1: return launch_step_n<1, S, T>(rho, grow, a, grid, st);
    case 4: return launch_step_n<4, S, T>(rho, grow, a, grid, st);
    case 9: return launch_step_n<9, S, T>(rho, grow, a, grid, st);
    case 16: return launch_step_n<16, S, T>(rho, grow, a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t step_lds_bytes(int N, int prec, bool with_rho, bool grow, int R, int Q) {
    if (use_step16(N, grow, R)) return step16_lds_layout(prec == kPrecC64 ? 8 : 16, with_rho, Q, with_rho).total;
    return step_lds_layout(N, prec == kPrecC64 ? 8 : 16, with_rho, grow ? 1 : N, R, Q, N <= 4).total;
}

hipError_t launch_g_quad(const QuadArgs &a, int n_t, double2 *g, hipStream_t st) {
    hipLaunchKernelGGL(g_quad_kernel, dim3(n_t), dim3(kBlock), 0, st, a, g);
    return hipGetLastError();
}

// U = exp(-i H dt) for each of n_H Hamiltonians (one for a static system,
// one per time interval for a driven one), a thread each.
__global__ void __launch_bounds__(64) u_stack_kernel(const double2 *H_t, int n_H, int M, double dt, double2 *U_t) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k < n_H) expm_minus_i_h_dt(H_t + (size_t)k * M * M, M, dt, U_t + (size_t)k * M * M);
}

hipError_t launch_u_stack(const double2 *H_t, int n_H, int M, double dt, double2 *U_t, hipStream_t st) {
    if (n_H <= 0) return hipSuccess;
    hipLaunchKernelGGL(u_stack_kernel, dim3((n_H + 63) / 64), dim3(64), 0, st, H_t, n_H, M, dt, U_t);
    return hipGetLastError();
}

hipError_t launch_tables(const TablesArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(tables_kernel, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init_tensor(int N, int prec, const double2 *rho0, const double2 *bank,
                              int self_end_tab, void *a0, hipStream_t st) {
    const double2 *se = bank + (size_t)self_end_tab * N * N;
    if (prec != kPrecC128) hipLaunchKernelGGL(init_tensor_kernel<float2>, dim3(1), dim3(64), 0, st, rho0, se, (float2 *)a0, N);
    else hipLaunchKernelGGL(init_tensor_kernel<double2>, dim3(1), dim3(64), 0, st, rho0, se, (double2 *)a0, N);
    return hipGetLastError();
}

hipError_t launch_step(int N, int prec, bool with_rho, bool grow, const StepArgs &a, int grid,
                       hipStream_t st) {
    if (use_step16(N, grow, a.R)) {
        switch (prec) {
        case kPrecC128:
            return with_rho ? launch_step16_t<double, double, true>(a, grid, st)
                            : launch_step16_t<double, double, false>(a, grid, st);
        case kPrecC64:
            return with_rho ? launch_step16_t<float, float, true>(a, grid, st)
                            : launch_step16_t<float, float, false>(a, grid, st);
        case kPrecC64F64:
            return with_rho ? launch_step16_t<float, double, true>(a, grid, st)
                            : launch_step16_t<float, double, false>(a, grid, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (prec) {
    case kPrecC128: return launch_step_dt<double, double>(N, with_rho, grow, a, grid, st);
    case kPrecC64: return launch_step_dt<float, float>(N, with_rho, grow, a, grid, st);
    case kPrecC64F64: return launch_step_dt<float, double>(N, with_rho, grow, a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_set_sink(RhoSink *sink, double2 *base, hipStream_t st) {
    hipLaunchKernelGGL(set_sink_kernel, dim3(1), dim3(64), 0, st, sink, base);
    return hipGetLastError();
}

hipError_t launch_rho_finalize(int N, const double2 *partials, int n_blocks, double2 *pairs, RhoSink *sink,
                               hipStream_t st) {
    switch (N) {
#define QUAPI_FIN(NV)                                                                                  \
    case NV:                                                                                           \
        hipLaunchKernelGGL(rho_slice_kernel<NV>, dim3(kSlices), dim3(kBlock), 0, st, partials, n_blocks, pairs); \
        hipLaunchKernelGGL(rho_final_kernel<NV>, dim3(1), dim3(kSlices), 0, st, pairs, sink);          \
        break;
        QUAPI_FIN(1)
        QUAPI_FIN(4)
        QUAPI_FIN(9)
        QUAPI_FIN(16)
#undef QUAPI_FIN
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_plan_tables(const PlanArgs &a, hipStream_t st) {
    const long long total = (long long)a.N * (a.R + a.Q + a.grid);
    const int grid = (int)std::min<long long>(1024, (total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(plan_tables_kernel, dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace quapi
