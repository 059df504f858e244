// Two full-window propagation steps per pass over the tensor (M = 2, N = 4):
// the fused step kernel, its coefficient kernel and their launchers.
//
// Method: Dattani 2012, Sec. II (exact path-sum equation and discretized
// influence functional); the tensor-propagator step of the Introduction,
// applied twice with the intermediate tensor kept in registers.
#include <hip/hip_runtime.h>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

// ------------------------------------------------- fused two-step (N = 4)
struct Step2Lds {
    unsigned tq, plo, phi, red, total;
};
__host__ __device__ inline Step2Lds step2_lds_layout(int csize, bool rho, int R, int Q) {
    constexpr int N = 4;
    const int ns = rho ? 4 : 2;
    Step2Lds l;
    unsigned off = 0;
    l.tq = lds_take(off, ns * N * Q * csize);
    l.plo = lds_take(off, ns * N * R * csize);
    l.phi = lds_take(off, ns * N * 16);
    l.red = lds_take(off, rho ? 2 * (kBlock / 64) * N * 16 : 0);
    l.total = off;
    return l;
}

// The fused-step coefficients (layout at kCoefOA ..), computed in FP64 and
// rounded once to the compute precision.
template <typename T>
__global__ void step2_coef_kernel(const CoefArgs a) {
    constexpr int N = 4, NN = 16;
    using C = typename Cx<T>::type;
    const int k = threadIdx.x;
    if (k >= kCoefCount) return;
    const double2 *old = a.bank + (size_t)a.old_tab * NN, *oldf = a.bank + (size_t)a.oldf_tab * NN;
    const double2 *an = a.bank + (size_t)a.an_tab * NN, *anf = a.bank + (size_t)a.anf_tab * NN;
    const double2 *d = a.bank + (size_t)a.d_tab * NN, *df = a.bank + (size_t)a.df_tab * NN;
    const int o = k / kCoefPerO, part = k % kCoefPerO / NN, e = k % NN, hi = e / N, lo = e % N;
    double2 v;
    if (part * NN == kCoefOA) v = cmul(an[o * N + hi], old[o * N + lo]);             // i' = hi, i = lo
    else if (part * NN == kCoefW) v = cmul(anf[o * N + hi], oldf[o * N + lo]);       // i' = hi, i = lo
    else if (part * NN == kCoefDO) v = cmul(d[hi * N + o], old[hi * N + lo]);        // o' = hi, i' = lo
    else v = cmul(df[hi * N + o], oldf[hi * N + lo]);                               // o' = hi, i' = lo
    ((C *)a.out)[k] = conv<C>(v);
}

// Steps n and n+1 (both full-window, n > L) in one pass over the tensor.
// Each item m (points n-L+2 .. n-1) reads the N^2 contiguous entries of the
// oldest two points (i = point n-L, i' = point n-L+1) and writes the N^2
// entries of the two new points (o = point n, o' = point n+1):
//   y(o, i')   = A_n(o, i') Bn(o, m) sum_i Old(o, i) x(i, i')          (A_n entry)
//   out(o, o') = D(o', o) Cn1(o', m) sum_i' Old(o', i') y(o, i')        (A_{n+1} entry)
// A_n(o, i') is the step-n factor of point n-L+1 and D(o', o) the step-(n+1)
// factor of point n (K folded in); Bn, Cn1 are the products over the digits of m.
// With RHO, rho(t_n) comes from x with the final-point classes of step n, and
// rho(t_{n+1}) from y with those of step n+1; both are reduced per block.
// The coefficients that do not depend on m are read per use through scalar
// loads; the m-dependent digit products come from LDS.
//
// MODE 1, 3: mirror mode, as in the three-step kernel (an entry and its
// mirror, every digit 2a + b -> 2b + a, are conjugates): mode 1 the blocks
// whose high digits are below their mirror and then, as the tail of the same
// launch, blocks of the high-digit values equal to it, which take the items
// below their mirror from a list, one per thread (as a launch of its own
// with the other items skipped this part took 0.058 ms of a 1.88 ms pass at
// L = 15); mode 3 the items that are their own mirror, whose input slots
// above the mirror are read from the mirrored slot, conjugated.  Outputs
// above their mirror go, conjugated, to the mirrored address; each block
// adds the mirrored items' rho terms as S[o] + conj(S[mirror(o)]) (mode 1).
__device__ __forceinline__ constexpr int mirror_digit4(int d) { return d == 1 ? 2 : d == 2 ? 1 : d; }
__device__ __forceinline__ int diagonal_digits4(unsigned x) {    // bit k -> digit k = 3
    int out = 0;
    for (int k = 0; x > 0; ++k, x >>= 1) out += (int)(x & 1u) * 3 << (2 * k);
    return out;
}
__device__ __forceinline__ bool diagonal_digits_only4(int v) {
    for (; v > 0; v >>= 2)
        if ((v & 3) == 1 || (v & 3) == 2) return false;
    return true;
}
template <typename S, typename T, bool RHO, int MODE>
__global__ void __launch_bounds__(kBlock) step2_kernel(const Step2Args a) {
    constexpr int N = 4, NN = 16;
    constexpr int NS = RHO ? 4 : 2;
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int R = a.R, Q = a.Q;
    const Step2Lds lay = step2_lds_layout((int)sizeof(C), RHO, R, Q);
    C *s_tq = (C *)(smem + lay.tq);            // [NS][N][Q]
    C *s_plo = (C *)(smem + lay.plo);          // [NS][N][R]
    double2 *s_phi = (double2 *)(smem + lay.phi);
    double2 *s_red = (double2 *)(smem + lay.red);
    const T *coef = (const T *)a.coef;

    const int t = threadIdx.x;
    const int cR = kBlock / R, active = cR * R;
    // mode 1: blocks below n_canon run the canonical high-digit values, the
    // rest the listed items of the values equal to their mirror (block-uniform)
    const bool listed = MODE == 1 && (int)blockIdx.x >= a.n_canon;
    const int lblk = listed ? (int)blockIdx.x - a.n_canon : 0;
    const long long blk = MODE == 0 ? (long long)blockIdx.x
                          : listed  ? (long long)a.blk_hi[a.n_canon + lblk / a.parts]
                                    : (long long)a.blk_hi[blockIdx.x];     // high digits
    if (t < NS * N) {
        const int s = t / N, o = t % N;
        s_phi[t] = a.t_hi[s][(size_t)o * a.grid + blk];
    }
    for (int idx = t; idx < NS * N * R; idx += kBlock) {
        const int s = idx / (N * R), k = idx % (N * R);
        s_plo[idx] = from_d2<C>(a.t_lo[s][k]);
    }
    __syncthreads();
    for (int idx = t; idx < NS * N * Q; idx += kBlock) {
        const int s = idx / (N * Q), k = idx % (N * Q), o = k / Q;
        s_tq[idx] = from_d2<C>(cmul(s_phi[s * N + o], a.t_mid[s][k]));
    }
    __syncthreads();

    double2 accn[RHO ? N : 1], accn1[RHO ? N : 1];
#pragma unroll
    for (int o = 0; o < (RHO ? N : 1); ++o) accn[o] = accn1[o] = make_double2(0.0, 0.0);
    const int r = t % R;
    if (t < active) {
        const long long m0 = blk * (long long)R * Q;
        const CS *__restrict__ ain = (const CS *)a.a_in;
        CS *__restrict__ aout = (CS *)a.a_out;
        const long long mc = a.m_count;
        // sweep rows: all (mode 0, 1), the listed items (q_span of them per
        // block, one per thread), or in mode 3 those whose digits are all
        // diagonal, for threads whose low digits are
        const int part = listed ? lblk % a.parts : 0;
        const bool thread_runs = MODE != 3 || diagonal_digits_only4(r);
        const int dm = (31 - __clz(Q)) >> 1;
        const int i0 = listed ? part * a.q_span + t : t / R;
        const int i1 = !thread_runs ? 0 : MODE == 3 ? (1 << dm) : listed ? min(a.n_low, (part + 1) * a.q_span) : Q;
        const int istep = listed ? kBlock : cR;
        for (int it = i0; it < i1; it += istep) {
            asm volatile("" ::: "memory");
            const int low = listed ? a.low_list[it] : 0;
            const int qm = MODE == 3 ? diagonal_digits4((unsigned)it) : listed ? low / R : it;
            // opaque per item: the factor reads from LDS stay in the loop
            // instead of being hoisted into registers for the whole block
            int rl = listed ? low & (R - 1) : r;
            asm volatile("" : "+v"(rl));
            const long long m = m0 + (long long)qm * R + rl;
            const long long mb = MODE == 0 ? m : mirror4(m);
            constexpr bool selfm = MODE == 3;
            C x[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                const int kb = (int)mirror4(k);
                x[k] = conv<C>(ain[(long long)NN * m + (selfm && kb < k ? kb : k)]);
                if (selfm && kb < k) x[k].y = -x[k].y;
            }
            C cn1[N], totf[RHO ? N : 1];
#pragma unroll
            for (int op = 0; op < N; ++op) {
                cn1[op] = cmul(s_plo[(1 * N + op) * R + rl], s_tq[(1 * N + op) * Q + qm]);
                if (RHO) totf[op] = C{};
            }
            // Diagonal points o = (a, a) (o = 0 and 3) carry no influence: every
            // factor exp(-(s_a - s_b)(...)) of a later point o is exactly one
            // there.  So OA and W (old-point tables times the lag L-1 >= 2
            // factor, no K) are ones in the rows o = 0, 3, and DO, V (K folded
            // in) do not depend on i' in the rows o' = 0, 3: those rows reduce
            // to plain sums over the summed point, shared by both diagonal rows.
            // (With FP32 arithmetic these shared sums stay unrounded until their
            // products, TraceSum: the diagonal rows carry the trace.)
            TraceSum<C> sx[N];
            C totd = {};
#pragma unroll
            for (int ip = 0; ip < N; ++ip) {
                sx[ip].init(x[N * ip]);
#pragma unroll
                for (int i = 1; i < N; ++i) sx[ip].add(x[i + N * ip]);
            }
            if (RHO) {
                totd = x[0];
#pragma unroll
                for (int k = 1; k < NN; ++k) totd = cadd(totd, x[k]);
            }
            // Per new point o of step n: the step-n entries y(o, i') (and the
            // rho(t_n) term), then every step-(n+1) entry that reads them.  The
            // diagonal points go first, so the shared sums are dead after them.
#pragma unroll
            for (int oo = 0; oo < N; ++oo) {
                const int o = oo == 0 ? 0 : oo == 1 ? 3 : oo - 1;
                asm volatile("" ::: "memory");  // coefficient reads of this o only
                const T *co = coef + 2 * kCoefPerO * o;
                const bool dg = o == 0 || o == 3;
                const C bn = cmul(s_plo[(0 * N + o) * R + rl], s_tq[(0 * N + o) * Q + qm]);
                C y[N];
#pragma unroll
                for (int ip = 0; ip < N; ++ip) {
                    if (dg) {
                        y[ip] = sx[ip].times(bn);
                    } else {
                        C sum = {};
#pragma unroll
                        for (int i = 0; i < N; ++i) cmac(sum, coef_ld(co, kCoefOA + ip * N + i), x[i + N * ip]);
                        y[ip] = cmul(bn, sum);
                    }
                }
                if (RHO) {
                    C tot = totd;
                    if (!dg) {
                        tot = C{};
#pragma unroll
                        for (int k = 0; k < NN; ++k) cmac(tot, coef_ld(co, kCoefW + k), x[k]);
                    }
                    const C bnf = cmul(s_plo[(2 * N + o) * R + rl], s_tq[(2 * N + o) * Q + qm]);
                    const double2 v = to_d2(cmul(bnf, tot));
                    accn[o].x += v.x;
                    accn[o].y += v.y;
                }
                TraceSum<C> ysum;
                ysum.init(y[0]);
#pragma unroll
                for (int ip = 1; ip < N; ++ip) ysum.add(y[ip]);
#pragma unroll
                for (int op = 0; op < N; ++op) {
                    asm volatile("" ::: "memory");
                    const bool dgp = op == 0 || op == 3;
                    C sum = {};
                    if (dgp) {
                        sum = ysum.times(coef_ld(co, kCoefDO + op * N));
                    } else {
#pragma unroll
                        for (int ip = 0; ip < N; ++ip) cmac(sum, coef_ld(co, kCoefDO + op * N + ip), y[ip]);
                    }
                    const C v = cmul(cn1[op], sum);
                    const int c2 = o + N * op, c2b = mirror_digit4(o) + N * mirror_digit4(op);
                    if (MODE == 0 || c2b >= c2) {
                        aout[m + mc * c2] = conv<CS>(v);
                    } else if (!selfm) {
                        C vc = v;
                        vc.y = -vc.y;
                        aout[mb + mc * c2b] = conv<CS>(vc);
                    }
                    if (RHO) {
                        if (dgp) {
                            cmac(totf[op], coef_ld(co, kCoefV + op * N), ysum.rounded());
                        } else {
#pragma unroll
                            for (int ip = 0; ip < N; ++ip) cmac(totf[op], coef_ld(co, kCoefV + op * N + ip), y[ip]);
                        }
                    }
                }
            }
            if (RHO) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int op = 0; op < N; ++op) {
                    const C cf1 = cmul(s_plo[(3 * N + op) * R + rl], s_tq[(3 * N + op) * Q + qm]);
                    const double2 v = to_d2(cmul(cf1, totf[op]));
                    accn1[op].x += v.x;
                    accn1[op].y += v.y;
                }
            }
        }
    }
    if (RHO) {
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int o = 0; o < N; ++o) {
            double2 v = accn[o], w = accn1[o];
            for (int off = 32; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
                w.x += __shfl_xor(w.x, off, 64);
                w.y += __shfl_xor(w.y, off, 64);
            }
            if (lane == 0) {
                s_red[wave * N + o] = v;
                s_red[(kBlock / 64 + wave) * N + o] = w;
            }
        }
        __syncthreads();
        if (t < 2 * N) {
            const int which = t / N, o = t % N, ob = mirror_digit4(o);
            double2 s = make_double2(0.0, 0.0);
            for (int w = 0; w < kBlock / 64; ++w) {
                s.x += s_red[(which * (kBlock / 64) + w) * N + o].x;
                s.y += s_red[(which * (kBlock / 64) + w) * N + o].y;
            }
            if (MODE == 1) {                        // the mirrored items' terms
                for (int w = 0; w < kBlock / 64; ++w) {
                    s.x += s_red[(which * (kBlock / 64) + w) * N + ob].x;
                    s.y -= s_red[(which * (kBlock / 64) + w) * N + ob].y;
                }
            }
            a.partials[which][((size_t)a.part_base + (MODE == 0 ? blk : (long long)blockIdx.x)) * N + o] = s;
        }
    }
}

template <typename S, typename T, bool RHO>
hipError_t launch_step2_t(const Step2Args &a, hipStream_t st) {
    using C = typename Cx<T>::type;
    const Step2Lds lay = step2_lds_layout((int)sizeof(C), RHO, a.R, a.Q);
    const dim3 b(kBlock);
    switch (a.mode) {
    case 0: hipLaunchKernelGGL((step2_kernel<S, T, RHO, 0>), dim3(a.grid), b, lay.total, st, a); break;
    case 1: hipLaunchKernelGGL((step2_kernel<S, T, RHO, 1>), dim3(a.n_blk), b, lay.total, st, a); break;
    case 3: hipLaunchKernelGGL((step2_kernel<S, T, RHO, 3>), dim3(a.n_blk), b, lay.total, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

size_t step2_lds_bytes(int prec, bool with_rho, int R, int Q) {
    return step2_lds_layout(prec == kPrecC64 ? 8 : 16, with_rho, R, Q).total;
}

hipError_t launch_step2(int prec, bool with_rho, const Step2Args &a, hipStream_t st) {
    switch (prec) {
    case kPrecC128:
        return with_rho ? launch_step2_t<double, double, true>(a, st) : launch_step2_t<double, double, false>(a, st);
    case kPrecC64:
        return with_rho ? launch_step2_t<float, float, true>(a, st) : launch_step2_t<float, float, false>(a, st);
    case kPrecC64F64:
        return with_rho ? launch_step2_t<float, double, true>(a, st) : launch_step2_t<float, double, false>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2_coef(const CoefArgs &a, hipStream_t st) {
    if (a.prec == kPrecC64) hipLaunchKernelGGL(step2_coef_kernel<float>, dim3(1), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(step2_coef_kernel<double>, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace quapi
