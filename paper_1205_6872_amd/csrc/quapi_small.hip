// Persistent propagation of small tensors: one workgroup per context runs
// every step of a call in one launch, and one launch serves a batch of
// contexts (same N and precision; each block its own context, memory length
// and step range).
//
// Method: Dattani 2012, Sec. II (exact path-sum equation, discretized
// influence functional); the tensor-propagator recursion of the Introduction,
// with rho(t_n) from the final-point classes (Sec. IV 'allPoints' /
// 'justFinalPoint').  The same steps as the multi-block kernels -- growth
// while the window fills, then multiply by K and the new point's factors and
// sum out the oldest point -- but the whole step sequence stays inside one
// workgroup, so a step costs a barrier rather than three kernel launches.
// The tensor ping-pongs between two LDS buffers when both fit (N^L up to
// 4096 at complex128), else between the context's two global buffers, which
// stay in the L2 cache at these sizes.
#include <hip/hip_runtime.h>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

// threads per block: 16 waves where the registers allow (N <= 9), else 4
template <int N> struct SmallBlock {
    static constexpr int threads = N <= 9 ? 1024 : 256;
    static constexpr int waves = threads / 64;
};

__host__ __device__ inline long long ipow_s(int b, int e) {
    long long r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// LDS layout of one block: the two tensor buffers (in-LDS mode), the
// full-window factor products over the low and high digits of m, interior
// and final ([N][RL], [N][RH] each, compute precision), the oldest-point
// tables (first / main full-window step, interior / final: 4 x [N][N],
// compute precision), and the per-wave rho sums (two parities).
struct SmallLds {
    unsigned buf0, buf1, plo, phi, pflo, pfhi, old, red, total;
    int dlo, dhi, RL, RH;
};
__host__ __device__ inline SmallLds small_lds_layout(int N, int csize_store, int csize_comp, int L, bool in_lds) {
    const int waves = N <= 9 ? SmallBlock<4>::waves : SmallBlock<16>::waves;
    SmallLds l;
    const int nd = L - 1;
    l.dlo = nd / 2;
    l.dhi = nd - l.dlo;
    l.RL = (int)ipow_s(N, l.dlo);
    l.RH = (int)ipow_s(N, l.dhi);
    const unsigned E = (unsigned)ipow_s(N, L);
    unsigned off = 0;
    l.buf0 = lds_take(off, in_lds ? E * csize_store : 0);
    l.buf1 = lds_take(off, in_lds ? E * csize_store : 0);
    l.plo = lds_take(off, N * l.RL * csize_comp);
    l.phi = lds_take(off, N * l.RH * csize_comp);
    l.pflo = lds_take(off, N * l.RL * csize_comp);
    l.pfhi = lds_take(off, N * l.RH * csize_comp);
    l.old = lds_take(off, 4 * N * N * csize_comp);
    l.red = lds_take(off, 2 * waves * N * 16);
    l.total = off;
    return l;
}

// Sum over the 64 lanes of a wave of P values per lane (P a power of two <= 64),
// leaving lane l with the total of value o = l >> (6 - log2 P): a butterfly
// that halves the values each lane carries per round (the half it does not
// keep goes to its partner), then sums the one value left over the lanes that
// share it -- P - 1 + 6 - log2 P exchanges instead of 6 P.
template <int P, int HALF>
__device__ __forceinline__ void scatter_round(double2 (&v)[P], int lane, int d) {
    if constexpr (HALF >= 1) {
        const bool up = (lane & d) != 0;
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const double2 send = up ? v[j] : v[j + HALF];
            const double2 keep = up ? v[j + HALF] : v[j];
            v[j].x = keep.x + __shfl_xor(send.x, d, 64);
            v[j].y = keep.y + __shfl_xor(send.y, d, 64);
        }
        scatter_round<P, HALF / 2>(v, lane, d / 2);
    }
}
template <int P>
__device__ __forceinline__ double2 wave_sum_scatter(double2 (&v)[P], int lane) {
    scatter_round<P, P / 2>(v, lane, 32);
    double2 r = v[0];
    for (int d = 32 / P; d >= 1; d /= 2) {
        r.x += __shfl_xor(r.x, d, 64);
        r.y += __shfl_xor(r.y, d, 64);
    }
    return r;
}

// Product over the digits j0 .. j0+nd-1 of v (base N, least significant
// first, digit j of v is table tab(j0 + k)) of the bank tables, row o (FP64).
template <int N, typename TabOf>
__device__ double2 small_digit_product(const double2 *__restrict__ bank, TabOf tab, int j0, int nd, long long v,
                                       int o) {
    double2 p = make_double2(1.0, 0.0);
    for (int k = 0; k < nd; ++k) {
        const int dg = (int)(v % N);
        v /= N;
        p = cmul(p, bank[(size_t)tab(j0 + k) * (N * N) + o * N + dg]);
    }
    return p;
}

template <int N, typename S, typename T, bool IN_LDS>
__global__ void __launch_bounds__(SmallBlock<N>::threads) small_kernel(const SmallBatchArgs args) {
    constexpr int kSB = SmallBlock<N>::threads, kSW = SmallBlock<N>::waves;
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    constexpr int M = N == 1 ? 1 : N == 4 ? 2 : N == 9 ? 3 : 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallCtxArgs a = args.c[blockIdx.x];
    const int L = a.L;
    const BankLayout B{L};
    const SmallLds lay = small_lds_layout(N, (int)sizeof(CS), (int)sizeof(C), L, IN_LDS);
    C *s_plo = (C *)(smem + lay.plo);
    C *s_phi = (C *)(smem + lay.phi);
    C *s_pflo = (C *)(smem + lay.pflo);
    C *s_pfhi = (C *)(smem + lay.pfhi);
    C *s_old = (C *)(smem + lay.old);          // [4][N][N]: old_first, old_main, oldf_first, oldf_main
    double2 *s_red = (double2 *)(smem + lay.red);
    const double2 *__restrict__ bank = a.bank;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long long NM = ipow_s(N, L - 1);      // items of a full-window step

    CS *buf[2];
    if (IN_LDS) {
        buf[0] = (CS *)(smem + lay.buf0);
        buf[1] = (CS *)(smem + lay.buf1);
        const long long E0 = ipow_s(N, min(a.step0 + 1, L));
        const CS *src = (const CS *)a.a0;
        for (long long x = t; x < E0; x += kSB) buf[0][x] = src[x];
    } else {
        buf[0] = (CS *)a.a0;
        buf[1] = (CS *)a.a1;
    }
    // the oldest-point tables of every full-window step, and the factor
    // products over the digits of m (formed in FP64, rounded once)
    const int otab[4] = {B.old_first(), B.old_main(), B.oldf_first(), B.oldf_main()};
    for (int idx = t; idx < 4 * N * N; idx += kSB)
        s_old[idx] = from_d2<C>(bank[(size_t)otab[idx / (N * N)] * (N * N) + idx % (N * N)]);
    auto tab_int = [&](int j) { const int lag = L - 1 - j; return lag == 1 ? B.k_lag1() : B.lag(lag); };
    auto tab_fin = [&](int j) { const int lag = L - 1 - j; return lag == 1 ? B.k_fin1() : B.fin(lag); };
    for (int idx = t; idx < N * lay.RL; idx += kSB) {
        const int o = idx / lay.RL, v = idx % lay.RL;
        s_plo[idx] = from_d2<C>(small_digit_product<N>(bank, tab_int, 0, lay.dlo, v, o));
        s_pflo[idx] = from_d2<C>(small_digit_product<N>(bank, tab_fin, 0, lay.dlo, v, o));
    }
    for (int idx = t; idx < N * lay.RH; idx += kSB) {
        const int o = idx / lay.RH, v = idx % lay.RH;
        s_phi[idx] = from_d2<C>(small_digit_product<N>(bank, tab_int, lay.dlo, lay.dhi, v, o));
        s_pfhi[idx] = from_d2<C>(small_digit_product<N>(bank, tab_fin, lay.dlo, lay.dhi, v, o));
    }
    __syncthreads();

    int n_out = 0;
    for (int k = 0; k < a.n_steps; ++k) {
        const int n = a.step0 + 1 + k;
        const bool sel = a.rho_mode == 1 || (a.rho_mode == 2 && k == a.n_steps - 1);
        const CS *__restrict__ in = buf[k & 1];
        CS *__restrict__ out = buf[(k + 1) & 1];
        // waves that own items this step (the others add nothing to rho)
        const long long items = n < L ? ipow_s(N, n) : NM;
        const int nw = (int)min((long long)kSW, (items + 63) / 64);
        double2 acc[N];
#pragma unroll
        for (int o = 0; o < N; ++o) acc[o] = make_double2(0.0, 0.0);
        if (n < L) {
            // growth: points 0 .. n-1 in, n+1 points out; out[x + E_in o] = x F(o, x)
            const long long E_in = ipow_s(N, n);
            auto tab_g = [&](int j) {
                if (j == 0) return n == 1 ? B.k_init1() : B.init(n);
                const int lag = n - j;
                return lag == 1 ? B.k_lag1() : B.lag(lag);
            };
            auto tab_gf = [&](int j) {
                if (j == 0) return n == 1 ? B.k_fin_init1() : B.fin_init(n);
                const int lag = n - j;
                return lag == 1 ? B.k_fin1() : B.fin(lag);
            };
            for (long long x = t; x < E_in; x += kSB) {
                const C xv = conv<C>(in[x]);
                const double2 xd = to_d2(xv);
#pragma unroll
                for (int o = 0; o < N; ++o) {
                    const double2 f = cmul(small_digit_product<N>(bank, tab_g, 0, n, x, o),
                                           bank[(size_t)B.self_int() * (N * N) + o * N]);
                    out[x + E_in * o] = conv<CS>(cmul(xv, from_d2<C>(f)));
                    if (sel) {
                        const double2 ff = cmul(small_digit_product<N>(bank, tab_gf, 0, n, x, o),
                                                bank[(size_t)B.self_end() * (N * N) + o * N]);
                        const double2 v = cmul(xd, ff);
                        acc[o].x += v.x;
                        acc[o].y += v.y;
                    }
                }
            }
        } else {
            // full window: out[m + NM o] = P(o, m) sum_i old[o][i] in[i + N m]
            const C *old = s_old + (n == L ? 0 : 1) * N * N;
            const C *oldf = s_old + (n == L ? 2 : 3) * N * N;
            for (long long m = t; m < NM; m += kSB) {
                C x[N];
#pragma unroll
                for (int i = 0; i < N; ++i) x[i] = conv<C>(in[i + N * m]);
                const int ml = (int)(m % lay.RL), mh = (int)(m / lay.RL);
#pragma unroll
                for (int o = 0; o < N; ++o) {
                    const C p = cmul(s_plo[o * lay.RL + ml], s_phi[o * lay.RH + mh]);
                    C v;
                    if (sizeof(T) == 4 && N > 1 && o % (M + 1) == 0 && L >= 2) {
                        // a diagonal point: its oldest-point row is ones and p is
                        // K[o, m_last]; the sum stays unrounded until the product
                        TraceSum<C> ts;
                        ts.init(x[0]);
#pragma unroll
                        for (int i = 1; i < N; ++i) ts.add(x[i]);
                        v = ts.times_right(p);
                    } else {
                        C s = {};
#pragma unroll
                        for (int i = 0; i < N; ++i) cmac(s, old[o * N + i], x[i]);
                        v = cmul(s, p);
                    }
                    out[m + NM * o] = conv<CS>(v);
                    if (sel) {
                        C sf = {};
#pragma unroll
                        for (int i = 0; i < N; ++i) cmac(sf, oldf[o * N + i], x[i]);
                        const C pf = cmul(s_pflo[o * lay.RL + ml], s_pfhi[o * lay.RH + mh]);
                        const double2 w = to_d2(cmul(sf, pf));
                        acc[o].x += w.x;
                        acc[o].y += w.y;
                    }
                }
            }
        }
        if (sel && wave < nw) {
            constexpr int P = N == 1 ? 1 : N <= 4 ? 4 : 16;      // N rounded up to a power of two
            constexpr int lg = P == 1 ? 0 : P == 4 ? 2 : 4;
            double2 v[P];
#pragma unroll
            for (int o = 0; o < P; ++o) v[o] = o < N ? acc[o] : make_double2(0.0, 0.0);
            const double2 r = wave_sum_scatter<P>(v, lane);
            const int o = lane >> (6 - lg);
            double2 *red = s_red + (k & 1) * kSW * N;
            if ((lane & ((64 >> lg) - 1)) == 0 && o < N) red[wave * N + o] = r;
        }
        __syncthreads();          // the new tensor and the wave sums are complete
        if (sel) {
            const double2 *red = s_red + (k & 1) * kSW * N;
            if (t < N) {
                double2 s = make_double2(0.0, 0.0);
                for (int w = 0; w < nw; ++w) {
                    s.x += red[w * N + t].x;
                    s.y += red[w * N + t].y;
                }
                a.rho_out[(size_t)n_out * N + t] = s;
            }
            ++n_out;
        }
    }
    if (IN_LDS) {
        // the last tensor goes to the buffer a step-by-step run would have
        // left it in: a0 after an even number of steps, a1 after an odd one
        const int last = a.step0 + a.n_steps;
        const long long E = ipow_s(N, min(last + 1, L));
        CS *dst = (CS *)((a.n_steps & 1) ? a.a1 : a.a0);
        const CS *src = buf[a.n_steps & 1];
        for (long long x = t; x < E; x += kSB) dst[x] = src[x];
    }
}

template <int N, typename S, typename T>
hipError_t launch_small_t(bool in_lds, const SmallBatchArgs &b, int n_ctx, int L_max, hipStream_t st) {
    const SmallLds lay = small_lds_layout(N, (int)sizeof(typename Cx<S>::type), (int)sizeof(typename Cx<T>::type),
                                          L_max, in_lds);
    if (in_lds)
        hipLaunchKernelGGL((small_kernel<N, S, T, true>), dim3(n_ctx), dim3(SmallBlock<N>::threads), lay.total, st, b);
    else
        hipLaunchKernelGGL((small_kernel<N, S, T, false>), dim3(n_ctx), dim3(SmallBlock<N>::threads), lay.total, st,
                           b);
    return hipGetLastError();
}

template <int N>
hipError_t launch_small_n(int prec, bool in_lds, const SmallBatchArgs &b, int n_ctx, int L_max, hipStream_t st) {
    switch (prec) {
    case kPrecC128: return launch_small_t<N, double, double>(in_lds, b, n_ctx, L_max, st);
    case kPrecC64: return launch_small_t<N, float, float>(in_lds, b, n_ctx, L_max, st);
    case kPrecC64F64: return launch_small_t<N, float, double>(in_lds, b, n_ctx, L_max, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t small_lds_bytes(int N, int prec, int L, bool in_lds) {
    const int cs = prec == kPrecC128 ? 16 : 8;
    const int cc = prec == kPrecC64 ? 8 : 16;
    return small_lds_layout(N, cs, cc, L, in_lds).total;
}

hipError_t launch_small(int N, int prec, bool in_lds, const SmallBatchArgs &b, int n_ctx, int L_max,
                        hipStream_t st) {
    if (n_ctx < 1 || n_ctx > kMaxSmallBatch) return hipErrorInvalidValue;
    switch (N) {
    case 1: return launch_small_n<1>(prec, in_lds, b, n_ctx, L_max, st);
    case 4: return launch_small_n<4>(prec, in_lds, b, n_ctx, L_max, st);
    case 9: return launch_small_n<9>(prec, in_lds, b, n_ctx, L_max, st);
    case 16: return launch_small_n<16>(prec, in_lds, b, n_ctx, L_max, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace quapi
