// Three full-window propagation steps per pass over the tensor (M = 2, N = 4):
// the three-step kernel, its coefficient kernel and their launchers.
//
// Method: Dattani 2012, Sec. II (exact path-sum equation and discretized
// influence functional); the tensor-propagator step of the Introduction,
// applied three times with the two intermediate tensors kept in registers.
// Each pass reads and writes the tensor once, so a step moves a third of the
// bytes of a single step.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

// With FP32 arithmetic (csize 8) and rho, each thread's FP64 rho sums live
// in LDS (acc: [3][N][kBlock]) instead of 48 registers, which lets the kernel
// fit two waves per SIMD.
struct Step3Lds {
    unsigned tq, plo, phi, red, acc, total;
};
__host__ __device__ inline Step3Lds step3_lds_layout(int csize, bool rho, int R, int Q) {
    constexpr int N = 4;
    const int ns = rho ? 6 : 3;
    Step3Lds l;
    unsigned off = 0;
    l.tq = lds_take(off, ns * N * Q * csize);
    l.plo = lds_take(off, ns * N * R * csize);
    l.phi = lds_take(off, ns * N * 16);
    l.red = lds_take(off, rho ? 3 * (kBlock / 64) * N * 16 : 0);
    l.acc = lds_take(off, rho && csize == 8 ? 3 * N * kBlock * 16 : 0);
    l.total = off;
    return l;
}

// The coefficient pointer passed through an opaque register move: loads
// through it are issued again after each call instead of being kept live in
// scalar registers across the whole item (the constant address space lets the
// compiler reuse them otherwise, and there are too many to keep).
template <typename T>
__device__ __forceinline__ const T *fresh(const T *p) {
    asm volatile("" : "+s"(p));
    return p;
}
// The same for a plane stride, so the 64 output-plane offsets are formed per
// group instead of all being kept (and spilled) for the whole item.
__device__ __forceinline__ long long fresh_stride(long long v) {
    asm volatile("" : "+s"(v));
    return v;
}

// The coefficients (layout at kC3Old ..), computed in FP64 and rounded once to
// the compute precision.
template <typename T>
__global__ void step3_coef_kernel(const Coef3Args a) {
    constexpr int N = 4, NN = 16;
    using C = typename Cx<T>::type;
    const int k = threadIdx.x;
    if (k >= kC3Count) return;
    auto tab = [&](int t, int row, int col) { return a.bank[(size_t)t * NN + row * N + col]; };
    double2 v;
    if (k < kC3Oldf) {
        v = tab(a.old_tab, k / N, k % N);
    } else if (k < kC3AF) {
        v = tab(a.oldf_tab, (k - kC3Oldf) / N, (k - kC3Oldf) % N);
    } else {
        const bool fin = ((k - kC3AF) / 64) % 2 == 1;
        const int part = (k - kC3AF) / 128, e = (k - kC3AF) % 64;
        // [x][y][z]: (x, y) is the group, z the new point of the stage
        const int x = e / NN, y = (e / N) % N, z = e % N;
        if (part == 0) {        // AF[i''][i'][o] = an(o, i') F(o, i'')
            v = cmul(tab(fin ? a.anf_tab : a.an_tab, z, y), tab(fin ? a.ff_tab : a.f_tab, z, x));
        } else if (part == 1) { // GH[i''][o][o'] = G(o', o) H(o', i'')
            v = cmul(tab(fin ? a.gf_tab : a.g_tab, z, y), tab(fin ? a.hf_tab : a.h_tab, z, x));
        } else {                // PQ[o'][o][o''] = P(o'', o') Q(o'', o)
            v = cmul(tab(fin ? a.pf_tab : a.p_tab, z, x), tab(fin ? a.qf_tab : a.q_tab, z, y));
        }
    }
    ((C *)a.out)[k] = conv<C>(v);
}

// Steps n, n+1, n+2 (all full-window, n > L) in one pass.  Each item m (points
// n-L+3 .. n-1) reads the N^3 contiguous entries of the oldest three points
// (i = n-L, i' = n-L+1, i'' = n-L+2) into w[i + N i' + N^2 i''] and writes the
// N^3 entries of the three new points (o = n, o' = n+1, o'' = n+2):
//   y(o, i', i'')  = B(o, m) AF(i'', i', o) sum_i old(o, i) x(i, i', i'')        (step n)
//   z(o, o', i'')  = C(o', m) GH(i'', o, o') sum_i' old(o', i') y(o, i', i'')    (step n+1)
//   out(o, o', o'') = D(o'', m) PQ(o', o, o'') sum_i'' old(o'', i'') z(o, o', i'') (step n+2)
// B, C, D are the products over the digits of m.  Each stage overwrites the
// four slots it reads, so w holds x, then y (slot o + N i' + N^2 i''), then z
// (slot o + N o' + N^2 i'').  With RHO, rho at each of the three steps comes
// from the values that stage reads, with the final-point classes.
//
// MODE 1, 3 (mirror mode): an entry and its mirror are conjugates, so
// only the items m not above their mirror mb are run, and of each output
// entry only the one not above its mirror is stored (the conjugate goes to
// the mirrored address).  Only those entries of the input need be valid: an
// item that is its own mirror (all digits diagonal) takes its other entries
// as the conjugates of theirs.  rho gets each item's terms and, for the
// mirrored item that is not run, their conjugates at the mirrored point.
// Mode 1 runs every item below its mirror: first the blocks whose high
// digits are below their mirror (all their items), then, as the tail of the
// same launch, the blocks of the high-digit values that are all diagonal,
// which walk the list of the items below their mirror (one per thread, so
// no lane idles: as a launch of its own with the other items skipped, this
// part took 0.17 ms of the 3.64 ms complex128 pass at L = 15; in the tail of
// the mode-1 launch it adds about 0.06 ms).  Mode 3, one block per diagonal
// high-digit value, runs the items that are their own mirror, from 2^28
// entries on a second stream, concurrently with the tail of mode 1.  Each
// mode knows at compile time which of the cases it handles.
__device__ __forceinline__ constexpr int mirror_digit(int d) { return d == 1 ? 2 : d == 2 ? 1 : d; }
// The item digits whose bits are those of x: bit i -> digit i = 3 (else 0).
__device__ __forceinline__ int diagonal_digits(unsigned x) {
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return (int)(3u * x);
}
template <typename C>
__device__ __forceinline__ C cconj(C v) {
    v.y = -v.y;
    return v;
}

template <typename S, typename T, bool RHO, int MODE>
__global__ void __launch_bounds__(kBlock, sizeof(T) == 4 ? 2 : 1) step3_kernel(const Step3Args a) {
    constexpr bool HALF = MODE != 0;
    constexpr bool ACC_LDS = RHO && sizeof(T) == 4;
    constexpr int N = 4, NNN = 64;
    constexpr int NS = RHO ? 6 : 3;
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int R = a.R, Q = a.Q;
    const Step3Lds lay = step3_lds_layout((int)sizeof(C), RHO, R, Q);
    C *s_tq = (C *)(smem + lay.tq);            // [NS][N][Q]
    C *s_plo = (C *)(smem + lay.plo);          // [NS][N][R]
    double2 *s_phi = (double2 *)(smem + lay.phi);
    double2 *s_red = (double2 *)(smem + lay.red);
    double2 *s_acc = (double2 *)(smem + lay.acc);
    const T *coef = (const T *)a.coef;

    const int t = threadIdx.x;
    const int cR = kBlock / R, active = cR * R;
    // high digits of m
    // mode 1: blocks below n_canon run the canonical high-digit values (every
    // item below its mirror), the rest the listed items of the values that
    // are their own mirror, `parts` blocks per value (block-uniform)
    const bool listed = MODE == 1 && (int)blockIdx.x >= a.n_canon;
    const int lblk = listed ? (int)blockIdx.x - a.n_canon : 0;
    const long long blk = MODE == 0 ? (long long)blockIdx.x
                          : listed  ? (long long)a.blk_hi[a.n_canon + lblk / a.parts]
                                    : (long long)a.blk_hi[blockIdx.x];
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

    double2 acc[(RHO && !ACC_LDS) ? 3 : 1][(RHO && !ACC_LDS) ? N : 1];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int o = 0; o < N; ++o) {
            if (ACC_LDS) s_acc[(s * N + o) * kBlock + t] = make_double2(0.0, 0.0);
            else if (RHO) acc[s][o] = make_double2(0.0, 0.0);
        }
    // this thread's rho sum of stage s and point o
    auto acc_at = [&](int s, int o) -> double2 & {
        return ACC_LDS ? s_acc[(s * N + o) * kBlock + t] : acc[ACC_LDS ? 0 : s][ACC_LDS ? 0 : o];
    };
    auto factor = [&](int set, int o, int r, int qm) {
        return cmul(s_plo[(set * N + o) * R + r], s_tq[(set * N + o) * Q + qm]);
    };
    // rho terms v[o] of one item; in mirror mode the mirrored item adds
    // conj(v[mirror(o)]) (o = 0, 3 are their own mirrors, 1 and 2 swap)
    auto add_rho = [&](int s, const double2 *v, bool both) {
        if (HALF && both) {
            acc_at(s, 0).x += 2.0 * v[0].x;
            acc_at(s, 1).x += v[1].x + v[2].x;
            acc_at(s, 1).y += v[1].y - v[2].y;
            acc_at(s, 2).x += v[2].x + v[1].x;
            acc_at(s, 2).y += v[2].y - v[1].y;
            acc_at(s, 3).x += 2.0 * v[3].x;
        } else {
#pragma unroll
            for (int o = 0; o < N; ++o) {
                acc_at(s, o).x += v[o].x;
                acc_at(s, o).y += v[o].y;
            }
        }
    };
    if (t < active) {
        const long long m0 = blk * (long long)R * Q;
        const CS *__restrict__ ain = (const CS *)a.a_in;
        CS *__restrict__ aout = (CS *)a.a_out;
        const long long mc = a.m_count;
        // iterations: sweep rows qm (thread digits r = t % R), a part of
        // them in mode 2; in mode 3 the items with all digits diagonal, whose
        // bits give the low and the sweep digits
        const int dl = (31 - __clz(R)) >> 1, dm = (31 - __clz(Q)) >> 1;
        // a listed block walks the list of the items below their mirror (the
        // same for every high-digit value that is its own mirror), q_span of
        // them per block, one per thread: every lane has an item
        const int part = listed ? lblk % a.parts : 0;
        const int i0 = MODE == 3 ? t : listed ? part * a.q_span + t : t / R;
        const int i1 = MODE == 3 ? (1 << (dl + dm)) : listed ? min(a.n_low, (part + 1) * a.q_span) : Q;
        const int istep = MODE == 3 || listed ? kBlock : cR;
        for (int it = i0; it < i1; it += istep) {
            asm volatile("" ::: "memory");
            const int low = listed ? a.low_list[it] : 0;
            int r = MODE == 3 ? diagonal_digits((unsigned)it & ((1u << dl) - 1)) : listed ? low & (R - 1) : t % R;
            // opaque per item: the factor reads from LDS below stay in the loop
            // instead of being hoisted (and, short of registers, spilled)
            asm volatile("" : "+v"(r));
            const int qm = MODE == 3 ? diagonal_digits((unsigned)it >> dl) : listed ? low / R : it;
            const long long m = m0 + (long long)qm * R + r;
            const long long mb = HALF ? mirror4(m) : m;
            constexpr bool selfm = MODE == 3;
            // an item that is its own mirror holds valid values only at the
            // slots not above their mirror: the others are their mirrors' conjugates
            C w[NNN];
#pragma unroll
            for (int k = 0; k < NNN; ++k) {
                const int kb = (int)mirror4(k);
                w[k] = conv<C>(ain[(long long)NNN * m + (selfm && kb < k ? kb : k)]);
                if (selfm && kb < k) w[k].y = -w[k].y;
            }

            // Each stage runs two passes over its 16 groups of four slots: first
            // the rho terms (the final-point table old_f resident in scalar
            // registers), then the step itself (table old resident), which
            // overwrites the slots.  Per group only the four group coefficients
            // are fetched again.
            //
            // Diagonal points o = (a, a) (o = 0 and 3) carry no influence: every
            // factor exp(-(s_a - s_b)(...)) of a later point o is exactly one
            // there.  So the old / old_f rows of o = 0, 3 and the step-n group
            // factors AF of o = 0, 3 (lags L-1 and L-2 >= 2, no K) are ones, and
            // their sums over the summed point are one plain sum shared by both
            // rows -- the same additions in the same order as the general form
            // (with FP32 arithmetic kept unrounded until their products,
            // TraceSum: these rows carry the trace).
            // ---- step n: groups g = i' + N i'', slots 4g .. 4g+3
            {
                if (RHO) {
                    const T *co = fresh(coef);
                    C tf[N] = {};           // tf[0]: both diagonal points
#pragma unroll
                    for (int g = 0; g < N * N; ++g) {
                        const T *cg = fresh(coef);
                        C sd = w[N * g];
#pragma unroll
                        for (int i = 1; i < N; ++i) sd = cadd(sd, w[N * g + i]);
                        tf[0] = cadd(tf[0], sd);
#pragma unroll
                        for (int o = 1; o <= 2; ++o) {
                            C sf = {};
#pragma unroll
                            for (int i = 0; i < N; ++i) cmac(sf, coef_ld(co, kC3Oldf + o * N + i), w[N * g + i]);
                            cmac(tf[o], coef_ld(cg, kC3AFf + g * N + o), sf);
                        }
                    }
                    double2 v[N];
#pragma unroll
                    for (int o = 0; o < N; ++o) v[o] = to_d2(cmul(factor(3, o, r, qm), tf[o == 3 ? 0 : o]));
                    add_rho(0, v, !selfm);
                }
                asm volatile("" ::: "memory");
                const T *co = fresh(coef);
                C bn[N];
#pragma unroll
                for (int o = 0; o < N; ++o) bn[o] = factor(0, o, r, qm);
#pragma unroll
                for (int g = 0; g < N * N; ++g) {
                    const T *cg = fresh(coef);
                    C xs[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) xs[i] = w[N * g + i];
                    {
                        TraceSum<C> sd;
                        sd.init(xs[0]);
#pragma unroll
                        for (int i = 1; i < N; ++i) sd.add(xs[i]);
                        w[N * g] = sd.times(bn[0]);
                        w[N * g + 3] = sd.times(bn[3]);
                    }
#pragma unroll
                    for (int o = 1; o <= 2; ++o) {
                        C s = {};
#pragma unroll
                        for (int i = 0; i < N; ++i) cmac(s, coef_ld(co, kC3Old + o * N + i), xs[i]);
                        w[N * g + o] = cmul(bn[o], cmul(coef_ld(cg, kC3AF + g * N + o), s));
                    }
                }
            }
            // ---- step n+1: groups (o, i''), slots o + N i' + N^2 i'' over i'
            {
                asm volatile("" ::: "memory");
                if (RHO) {
                    const T *co = fresh(coef);
                    C tf[N] = {};
#pragma unroll
                    for (int ipp = 0; ipp < N; ++ipp) {
#pragma unroll
                        for (int o = 0; o < N; ++o) {
                            const T *cg = fresh(coef);
                            C sd = w[o + N * N * ipp];
#pragma unroll
                            for (int ip = 1; ip < N; ++ip) sd = cadd(sd, w[o + N * ip + N * N * ipp]);
#pragma unroll
                            for (int op = 0; op < N; ++op) {
                                C sf = sd;
                                if (op == 1 || op == 2) {
                                    sf = C{};
#pragma unroll
                                    for (int ip = 0; ip < N; ++ip)
                                        cmac(sf, coef_ld(co, kC3Oldf + op * N + ip), w[o + N * ip + N * N * ipp]);
                                }
                                cmac(tf[op], coef_ld(cg, kC3GHf + (ipp * N + o) * N + op), sf);
                            }
                        }
                    }
                    double2 v[N];
#pragma unroll
                    for (int op = 0; op < N; ++op) v[op] = to_d2(cmul(factor(4, op, r, qm), tf[op]));
                    add_rho(1, v, !selfm);
                }
                asm volatile("" ::: "memory");
                const T *co = fresh(coef);
                C cn[N];
#pragma unroll
                for (int op = 0; op < N; ++op) cn[op] = factor(1, op, r, qm);
#pragma unroll
                for (int ipp = 0; ipp < N; ++ipp) {
#pragma unroll
                    for (int o = 0; o < N; ++o) {
                        const T *cg = fresh(coef);
                        C ys[N];
#pragma unroll
                        for (int ip = 0; ip < N; ++ip) ys[ip] = w[o + N * ip + N * N * ipp];
                        {
                            TraceSum<C> sd;
                            sd.init(ys[0]);
#pragma unroll
                            for (int ip = 1; ip < N; ++ip) sd.add(ys[ip]);
#pragma unroll
                            for (int op = 0; op < N; op += 3)
                                w[o + N * op + N * N * ipp] =
                                    cmul(cn[op], sd.times(coef_ld(cg, kC3GH + (ipp * N + o) * N + op)));
                        }
#pragma unroll
                        for (int op = 1; op <= 2; ++op) {
                            C s = {};
#pragma unroll
                            for (int ip = 0; ip < N; ++ip) cmac(s, coef_ld(co, kC3Old + op * N + ip), ys[ip]);
                            w[o + N * op + N * N * ipp] =
                                cmul(cn[op], cmul(coef_ld(cg, kC3GH + (ipp * N + o) * N + op), s));
                        }
                    }
                }
            }
            // ---- step n+2: groups (o, o'), slots o + N o' + N^2 i'' over i''; store
            {
                asm volatile("" ::: "memory");
                if (RHO) {
                    const T *co = fresh(coef);
                    C tf[N] = {};
#pragma unroll
                    for (int op = 0; op < N; ++op) {
#pragma unroll
                        for (int o = 0; o < N; ++o) {
                            const T *cg = fresh(coef);
                            C sd = w[o + N * op];
#pragma unroll
                            for (int ipp = 1; ipp < N; ++ipp) sd = cadd(sd, w[o + N * op + N * N * ipp]);
#pragma unroll
                            for (int opp = 0; opp < N; ++opp) {
                                C sf = sd;
                                if (opp == 1 || opp == 2) {
                                    sf = C{};
#pragma unroll
                                    for (int ipp = 0; ipp < N; ++ipp)
                                        cmac(sf, coef_ld(co, kC3Oldf + opp * N + ipp), w[o + N * op + N * N * ipp]);
                                }
                                cmac(tf[opp], coef_ld(cg, kC3PQf + (op * N + o) * N + opp), sf);
                            }
                        }
                    }
                    double2 v[N];
#pragma unroll
                    for (int opp = 0; opp < N; ++opp) v[opp] = to_d2(cmul(factor(5, opp, r, qm), tf[opp]));
                    add_rho(2, v, !selfm);
                }
                asm volatile("" ::: "memory");
                const T *co = fresh(coef);
                C dn[N];
#pragma unroll
                for (int opp = 0; opp < N; ++opp) dn[opp] = factor(2, opp, r, qm);
#pragma unroll
                for (int op = 0; op < N; ++op) {
#pragma unroll
                    for (int o = 0; o < N; ++o) {
                        const T *cg = fresh(coef);
                        const long long st = fresh_stride(mc);
                        CS *const po = aout + m + st * (o + N * op);
                        CS *const pb = aout + mb + st * (mirror_digit(o) + N * mirror_digit(op));
                        C zs[N];
#pragma unroll
                        for (int ipp = 0; ipp < N; ++ipp) zs[ipp] = w[o + N * op + N * N * ipp];
                        auto store = [&](int opp, C u) {
                            const C v = cmul(dn[opp], u);
                            const int c3 = o + N * op + N * N * opp;
                            if (!HALF || (int)mirror4(c3) >= c3) po[st * N * N * opp] = conv<CS>(v);
                            else if (!selfm) pb[st * N * N * mirror_digit(opp)] = conv<CS>(cconj(v));
                        };
                        {
                            TraceSum<C> sd;
                            sd.init(zs[0]);
#pragma unroll
                            for (int ipp = 1; ipp < N; ++ipp) sd.add(zs[ipp]);
#pragma unroll
                            for (int opp = 0; opp < N; opp += 3)
                                store(opp, sd.times(coef_ld(cg, kC3PQ + (op * N + o) * N + opp)));
                        }
#pragma unroll
                        for (int opp = 1; opp <= 2; ++opp) {
                            C s = {};
#pragma unroll
                            for (int ipp = 0; ipp < N; ++ipp) cmac(s, coef_ld(co, kC3Old + opp * N + ipp), zs[ipp]);
                            store(opp, cmul(coef_ld(cg, kC3PQ + (op * N + o) * N + opp), s));
                        }
                    }
                }
            }
        }
    }
    if (RHO) {
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
#pragma unroll
            for (int o = 0; o < N; ++o) {
                double2 v = acc_at(s, o);
                for (int off = 32; off > 0; off >>= 1) {
                    v.x += __shfl_xor(v.x, off, 64);
                    v.y += __shfl_xor(v.y, off, 64);
                }
                if (lane == 0) s_red[(s * (kBlock / 64) + wave) * N + o] = v;
            }
        }
        __syncthreads();
        if (t < 3 * N) {
            const int s = t / N, o = t % N;
            double2 sum = make_double2(0.0, 0.0);
            for (int w = 0; w < kBlock / 64; ++w) {
                sum.x += s_red[(s * (kBlock / 64) + w) * N + o].x;
                sum.y += s_red[(s * (kBlock / 64) + w) * N + o].y;
            }
            a.partials[s][((size_t)a.part_base + blockIdx.x) * N + o] = sum;
        }
    }
}

template <typename S, typename T, bool RHO>
hipError_t launch_step3_t(const Step3Args &a, hipStream_t st) {
    using C = typename Cx<T>::type;
    const Step3Lds lay = step3_lds_layout((int)sizeof(C), RHO, a.R, a.Q);
    if (a.mode == 1)
        hipLaunchKernelGGL((step3_kernel<S, T, RHO, 1>), dim3(a.n_blk), dim3(kBlock), lay.total, st, a);
    else if (a.mode == 3)
        hipLaunchKernelGGL((step3_kernel<S, T, RHO, 3>), dim3(a.n_blk), dim3(kBlock), lay.total, st, a);
    else
        hipLaunchKernelGGL((step3_kernel<S, T, RHO, 0>), dim3(a.grid), dim3(kBlock), lay.total, st, a);
    return hipGetLastError();
}

// One thread per entry x: entries above their mirror take the conjugate of it.
template <int N, typename CS>
__global__ void __launch_bounds__(kBlock) mirror_complete_kernel(CS *__restrict__ a, long long entries) {
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < entries;
         x += (long long)gridDim.x * kBlock) {
        const long long xb = N == 4 ? mirror4(x) : N == 16 ? mirror16(x) : mirror9(x);
        if (xb < x) a[x] = cconj(a[xb]);
    }
}

}  // namespace

size_t step3_lds_bytes(int prec, bool with_rho, int R, int Q) {
    return step3_lds_layout(prec == kPrecC64 ? 8 : 16, with_rho, R, Q).total;
}

hipError_t launch_step3(int prec, bool with_rho, const Step3Args &a, hipStream_t st) {
    switch (prec) {
    case kPrecC128:
        return with_rho ? launch_step3_t<double, double, true>(a, st) : launch_step3_t<double, double, false>(a, st);
    case kPrecC64:
        return with_rho ? launch_step3_t<float, float, true>(a, st) : launch_step3_t<float, float, false>(a, st);
    case kPrecC64F64:
        return with_rho ? launch_step3_t<float, double, true>(a, st) : launch_step3_t<float, double, false>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mirror_complete(int N, int prec, void *a, long long entries, hipStream_t st) {
    const long long blocks = std::min<long long>((entries + kBlock - 1) / kBlock, 1 << 20);
    if (blocks < 1) return hipSuccess;
    if (N != 4 && N != 9 && N != 16) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), b(kBlock);
    if (prec == kPrecC128) {
        double2 *p = (double2 *)a;
        if (N == 4) hipLaunchKernelGGL((mirror_complete_kernel<4, double2>), g, b, 0, st, p, entries);
        else if (N == 9) hipLaunchKernelGGL((mirror_complete_kernel<9, double2>), g, b, 0, st, p, entries);
        else hipLaunchKernelGGL((mirror_complete_kernel<16, double2>), g, b, 0, st, p, entries);
    } else {
        float2 *p = (float2 *)a;
        if (N == 4) hipLaunchKernelGGL((mirror_complete_kernel<4, float2>), g, b, 0, st, p, entries);
        else if (N == 9) hipLaunchKernelGGL((mirror_complete_kernel<9, float2>), g, b, 0, st, p, entries);
        else hipLaunchKernelGGL((mirror_complete_kernel<16, float2>), g, b, 0, st, p, entries);
    }
    return hipGetLastError();
}

hipError_t launch_step3_coef(const Coef3Args &a, hipStream_t st) {
    if (a.prec == kPrecC64) hipLaunchKernelGGL(step3_coef_kernel<float>, dim3(1), dim3(512), 0, st, a);
    else hipLaunchKernelGGL(step3_coef_kernel<double>, dim3(1), dim3(512), 0, st, a);
    return hipGetLastError();
}

}  // namespace quapi
