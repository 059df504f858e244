// Filtered propagation: the augmented tensor stored sparsely, every entry
// whose magnitude is not above a threshold theta dropped as soon as it is
// formed (Sim's on-the-fly filtering of the tensor propagator, which the
// paper names in its Introduction as the way to cut the tensor's memory).
//
// The kept entries are (key, value) pairs sorted by key, the flat tensor
// index (oldest point fastest).  A step works segment by segment, a segment
// being the kept entries that share every digit but the oldest:
//   full window (n >= L): out(o, m) = P(o, m) sum_{i kept} Old[o][i] A[i + N m],
//                         new key m + N^(L-1) o;
//   growth (n < L):       out(o, x) = P(o, x) Self[o] A[x], new key x + N^n o,
//                         every entry its own segment;
// P the product of the factor tables over the digits (Sec. II: the bare
// propagator and the discretized influence functional), Old the oldest
// point's table with the new point's self factor folded in.  An output is
// kept when |out| > theta.  Because the new point is the most significant
// digit, writing the kept outputs in the order (o, segment) leaves them
// sorted by the new key: no sort is needed.
//
// A step is three launches (and the rho finalize when rho is selected):
//   count   block b walks its contiguous range of input entries in tiles,
//           finds the segment heads of a tile (ballots), gathers them in
//           LDS, and gives one thread per segment: it forms the N outputs,
//           stores their keep bits as a mask at the segment's head entry,
//           counts the kept outputs per o for the block, and adds the
//           segment's rho(t_n) terms (final-point classes);
//   offsets one block turns the N x blocks counts into exclusive offsets
//           in (o, block) order, and sets the new entry count (at most the
//           capacity) and the overflow flag;
//   write   the same walk; each segment's mask gives, with ballots and the
//           block's running offset per o, the place of every kept output,
//           which is formed again and stored.
// Both walks cost one read of the keys and values; the write pass stores the
// kept outputs once.  The grids are fixed and read the entry count from
// device memory, so a run needs no host synchronization; integer counts and
// fixed-order partial sums make it deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

constexpr int kFB = kFilterBlock;        // threads per block
constexpr int kWaves = kFB / 64;
constexpr int kSpan = 4;                 // entries per thread and tile
constexpr int kTile = kFB * kSpan;       // entries per tile

// ------------------------------------------------------------ factor tables
// The factor product over the digits of m is split into levels: level 0 the
// lowest D0 digits, level l >= 1 the next D digits each, with
// T_l[v][o] = prod over the digits of v of the tables of those digits at o, so
// that P(o, m) = prod_l T_l[digits of m in level l][o] (FP64), and the same
// for the final-point classes.  An entry holds both (p, pf), and the N values
// of o for one (l, v) are contiguous.  Level 0 is small enough for LDS: the
// lowest digits differ from segment to segment, the higher ones change slowly
// along the sorted keys, so their lookups from global memory mostly hit the
// same cache lines.  S0 = N^D0 and S = N^D are compile-time constants.
template <int N> struct FilterLevel {
    static constexpr int D0 = N == 4 ? 3 : N == 1 ? kMaxL : 1;
    static constexpr int S0 = N == 4 ? 64 : N;
    static constexpr int S = N == 4 ? 4096 : N == 9 ? 729 : N == 16 ? 4096 : 1;
    static constexpr int kMax = 7;       // levels of the largest tensor (N^L <= 2^62)
};

__host__ __device__ inline int filter_level0_digits(int N) { return N == 4 ? 3 : N == 1 ? kMaxL : 1; }
__host__ __device__ inline int filter_level0_size(int N) { return N == 4 ? 64 : N; }
__host__ __device__ inline int filter_level_digits(int N) { return N == 4 ? 6 : N == 1 ? kMaxL : 3; }
__host__ __device__ inline int filter_level_size(int N) {
    return N == 4 ? 4096 : N == 9 ? 729 : N == 16 ? 4096 : 1;
}

__global__ void __launch_bounds__(kFB) filter_plan_kernel(const FilterPlanArgs a) {
    const int N = a.N, S0 = filter_level0_size(N), S = filter_level_size(N);
    const int D0 = filter_level0_digits(N), D = filter_level_digits(N);
    const long long total = (long long)N * (S0 + (long long)(a.n_lv - 1) * S);
    const double2 one = make_double2(1.0, 0.0);
    for (long long idx = (long long)blockIdx.x * kFB + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * kFB) {
        const int o = (int)(idx % N);
        const long long e = idx / N;
        int l, v;
        if (e < S0) {
            l = 0;
            v = (int)e;
        } else {
            l = 1 + (int)((e - S0) / S);
            v = (int)((e - S0) % S);
        }
        const int j0 = l == 0 ? 0 : D0 + (l - 1) * D, j1 = l == 0 ? D0 : j0 + D;
        double2 p = one, pf = one;
        for (int j = j0; j < a.nd && j < j1; ++j) {
            const int dg = v % N;
            v /= N;
            p = cmul(p, a.bank[(size_t)a.tab[j] * (N * N) + o * N + dg]);
            pf = cmul(pf, a.bank[(size_t)a.tabf[j] * (N * N) + o * N + dg]);
        }
        a.t[2 * idx] = p;
        a.t[2 * idx + 1] = pf;
    }
}

// ------------------------------------------------------------------- step
// The digits a segment shares: all but the oldest (full window), or all.
template <int N>
__device__ __forceinline__ unsigned long long seg_of(unsigned long long key, bool full) {
    return full ? key / N : key;
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) { return (1ull << lane) - 1ull; }

// The count (COUNT) or write pass of one step; see the top of the file.
// Dynamic LDS (RHO): each thread's rho sums, [o][thread].
template <int N, typename S, typename T, bool COUNT, bool RHO>
__global__ void __launch_bounds__(kFB) filter_step_kernel(const FilterStepArgs a) {
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    using LV = FilterLevel<N>;
    static_assert(N <= 16, "keep masks are 16 bits");
    // the outputs of a segment run unrolled at N <= 4 (their loads overlap);
    // at N = 9, 16 one at a time (unrolled, they spill)
    constexpr int kOutUnroll = 1;
    // N <= 4: the upper factor levels of a segment are multiplied for every o
    // at once, before the outputs, so that their loads are in flight together
    // (not in the FP64 count pass with rho, where the 2N held products cost a
    // wave per SIMD: M = 2, L = 15, theta = 1e-10, complex128 step 0.670 ->
    // 0.624 ms)
    constexpr bool kHoist = N <= 4 && !(COUNT && RHO && sizeof(T) == 8);
    // entries past a tile that a segment starting in it may reach
    constexpr int kExt = N - 1;
    // values staged with the keys (complex64 storage); complex128 values are
    // read per segment from global memory (their registers in flight cost
    // a wave per SIMD)
    constexpr bool kStageVals = sizeof(CS) <= 8;
    extern __shared__ __align__(16) unsigned char f_smem[];
    double2 *s_acc = (double2 *)f_smem;
    __shared__ C s_old[N * N], s_oldf[N * N];
    __shared__ double2 s_t0[2 * LV::S0 * N];           // level 0 of the factor tables
    __shared__ unsigned short s_heads[kTile];          // tile offsets of the tile's segment heads
    __shared__ unsigned s_hw[kSpan][kWaves];           // heads per sub-tile and wave
    __shared__ unsigned s_kw[kWaves][N];               // write pass: kept outputs per wave and o
    __shared__ unsigned long long s_run[N];            // write pass: the block's next place per o
    __shared__ unsigned s_cnt[N];                      // count pass: the block's kept outputs per o
    __shared__ double2 s_red[kWaves][RHO ? N : 1];
    // the staged tile: s_key[0] the key of the entry before it, s_key[1 + i]
    // and s_val[i] key and value of entry base + i (i < kTile + kExt; keys
    // past the last entry are ~0, which no segment matches), s_mask[i] its
    // keep mask (write pass)
    __shared__ unsigned long long s_key[kTile + kExt + 1];
    __shared__ CS s_val[kStageVals ? kTile + kExt : 1];
    __shared__ unsigned short s_mask[COUNT ? 1 : kTile];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const bool full = a.full != 0;
    const double2 *__restrict__ bank = a.bank;
    const unsigned long long *__restrict__ keys = a.keys_in;
    const CS *__restrict__ vin = (const CS *)a.vals_in;
    CS *__restrict__ vout = (CS *)a.vals_out;
    for (int idx = t; idx < N * N; idx += kFB) {
        s_old[idx] = from_d2<C>(bank[(size_t)a.old_tab * (N * N) + idx]);
        if (RHO) s_oldf[idx] = from_d2<C>(bank[(size_t)a.oldf_tab * (N * N) + idx]);
    }
    if (a.n_lv > 0)
        for (int idx = t; idx < 2 * LV::S0 * N; idx += kFB) s_t0[idx] = a.t[idx];
    if (RHO)
        for (int o = 0; o < N; ++o) s_acc[o * kFB + t] = make_double2(0.0, 0.0);
    if (t < N) {
        if (COUNT) s_cnt[t] = 0;
        else s_run[t] = a.bofs[(size_t)t * gridDim.x + blockIdx.x];
    }
    // |out| > theta as |out|^2 > theta^2 where theta^2 is a normal number
    const bool squared = a.theta >= 1e-150;
    const double theta2 = a.theta * a.theta;
    const unsigned long long n_in = *a.count_in;
    const unsigned long long chunk = (n_in + gridDim.x - 1) / gridDim.x;
    const unsigned long long lo = chunk * blockIdx.x;
    const unsigned long long hi = lo + chunk < n_in ? lo + chunk : n_in;

    // The next tile's keys, values (and masks) are loaded into registers
    // while the current tile, staged in LDS, is processed: one coalesced read
    // per tile, and no global load waits on another.
    unsigned long long pk[kSpan], pke = ~0ull, pprev = ~0ull;
    CS pv[kStageVals ? kSpan : 1], pve = CS{};
    unsigned short pm[kSpan];
    auto fetch = [&](unsigned long long b) {
#pragma unroll
        for (int u = 0; u < kSpan; ++u) {
            const unsigned long long k = b + (unsigned long long)u * kFB + t;
            const bool in = k < n_in;
            pk[u] = in ? keys[k] : ~0ull;
            if (kStageVals) pv[kStageVals ? u : 0] = in ? vin[k] : CS{};
            pm[u] = (!COUNT && k < hi) ? a.masks[k] : (unsigned short)0;
        }
        if (t < kExt) {
            const unsigned long long k = b + kTile + t;
            pke = k < n_in ? keys[k] : ~0ull;
            if (kStageVals) pve = k < n_in ? vin[k] : CS{};
        }
        if (t == kFB - 1) pprev = b > 0 ? keys[b - 1] : ~0ull;
    };
    // The digits above level 1 change slowly along the sorted keys: the
    // products of the levels >= 2 for the few values those digits take in
    // the block's range are formed once, in LDS (at most kHiCache values;
    // otherwise the segments multiply those levels from global memory).
    constexpr int kHiCache = 4;
    __shared__ double2 s_hi[kHiCache * N * 2];
    const unsigned long long hdiv = (unsigned long long)LV::S0 * LV::S;
    unsigned long long hv_lo = 0;
    int n_hi = 0;
    if (a.n_lv >= 3 && lo < hi) {
        hv_lo = seg_of<N>(keys[lo], full) / hdiv;
        const unsigned long long hv_hi = seg_of<N>(keys[hi - 1], full) / hdiv;
        if (hv_hi - hv_lo < (unsigned long long)kHiCache) n_hi = (int)(hv_hi - hv_lo) + 1;
    }
    for (int idx = t; idx < n_hi * N; idx += kFB) {
        const int o = idx % N;
        unsigned long long v = hv_lo + (unsigned long long)(idx / N);
        double2 p = make_double2(1.0, 0.0), pf = p;
        for (int l = 2; l < a.n_lv; ++l) {
            const double2 *q = a.t + 2 * (((size_t)LV::S0 + (size_t)(l - 1) * LV::S + v % LV::S) * N + o);
            v /= LV::S;
            p = cmul(p, q[0]);
            if (RHO) pf = cmul(pf, q[1]);
        }
        s_hi[2 * idx] = p;
        s_hi[2 * idx + 1] = pf;
    }
    if (lo < hi) fetch(lo);
    __syncthreads();
    // the oldest-point rows that are exactly one (the diagonal new points:
    // every influence factor of a point with s_a = s_b is one): their
    // contraction is a plain sum (interior and final-point tables alike)
    unsigned ones = 0, ones_f = 0;
    for (int o = 0; o < N; ++o) {
        bool r = true, rf = true;
        for (int i = 0; i < N; ++i) {
            r = r && s_old[o * N + i].x == T(1) && s_old[o * N + i].y == T(0);
            if (RHO) rf = rf && s_oldf[o * N + i].x == T(1) && s_oldf[o * N + i].y == T(0);
        }
        ones |= (unsigned)r << o;
        ones_f |= (unsigned)(RHO && rf) << o;
    }

    for (unsigned long long base = lo; base < hi; base += kTile) {
#pragma unroll
        for (int u = 0; u < kSpan; ++u) {
            s_key[1 + u * kFB + t] = pk[u];
            if (kStageVals) s_val[kStageVals ? u * kFB + t : 0] = pv[kStageVals ? u : 0];
            if (!COUNT) s_mask[u * kFB + t] = pm[u];
        }
        if (t < kExt) {
            s_key[1 + kTile + t] = pke;
            if (kStageVals) s_val[kStageVals ? kTile + t : 0] = pve;
        }
        if (t == kFB - 1) s_key[0] = pprev;
        if (base + kTile < hi) fetch(base + kTile);
        __syncthreads();
        // the segment heads of the tile, gathered in key order (sub-tile u, then lane)
        bool head[kSpan];
        unsigned long long bal[kSpan];
#pragma unroll
        for (int u = 0; u < kSpan; ++u) {
            const int i = u * kFB + t;
            head[u] = base + (unsigned long long)i < hi &&
                      seg_of<N>(s_key[i], full) != seg_of<N>(s_key[1 + i], full);
            bal[u] = __ballot(head[u]);
            if (lane == 0) s_hw[u][wave] = (unsigned)__popcll(bal[u]);
        }
        __syncthreads();
        unsigned n_heads = 0;
#pragma unroll
        for (int u = 0; u < kSpan; ++u) {
            unsigned before = n_heads;
            for (int w = 0; w < kWaves; ++w) {
                if (w < wave) before += s_hw[u][w];
                n_heads += s_hw[u][w];
            }
            if (head[u]) s_heads[before + __popcll(bal[u] & lanes_below(lane))] = (unsigned short)(u * kFB + t);
        }
        __syncthreads();

        // one thread per segment, in rounds of kFB segments
        for (unsigned r = 0; r < n_heads; r += kFB) {
            const bool active = r + t < n_heads;
            unsigned long long kh = 0, m = 0;
            C x[N];
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = C{};
            unsigned mask = 0;
            unsigned lv[LV::kMax];                     // level indices of m
            if (active) {
                const int h = s_heads[r + t];
                kh = base + (unsigned long long)h;
                m = seg_of<N>(s_key[1 + h], full);
                if (full) {
                    // the segment's values by oldest digit (the dropped ones are zero)
                    if constexpr (!kStageVals && N <= 4) {
                        // all N candidates requested at once; those of the next segments are ignored
                        CS vv[N];
#pragma unroll
                        for (int e = 0; e < N; ++e)
                            vv[e] = base + h + e < n_in ? vin[kh + e] : CS{};
#pragma unroll
                        for (int e = 0; e < N; ++e) {
                            const unsigned long long key = s_key[1 + h + e];
                            if (seg_of<N>(key, true) != m) continue;
                            const int i = (int)(key % N);
#pragma unroll
                            for (int ii = 0; ii < N; ++ii)
                                if (ii == i) x[ii] = conv<C>(vv[e]);
                        }
                    } else {
                        for (int e = 0; e < N; ++e) {
                            const unsigned long long key = s_key[1 + h + e];
                            if (seg_of<N>(key, true) != m) break;
                            const int i = (int)(key % N);
                            const C v = conv<C>(kStageVals ? s_val[kStageVals ? h + e : 0] : vin[kh + e]);
#pragma unroll
                            for (int ii = 0; ii < N; ++ii)
                                if (ii == i) x[ii] = v;
                        }
                    }
                } else {
                    x[0] = conv<C>(kStageVals ? s_val[kStageVals ? h : 0] : vin[kh]);
                }
                if (!COUNT) mask = s_mask[h];
            }
            {
                lv[0] = (unsigned)(m % LV::S0);
                unsigned long long v = m / LV::S0;
#pragma unroll
                for (int l = 1; l < LV::kMax; ++l) {
                    lv[l] = (unsigned)(v % LV::S);
                    v /= LV::S;
                }
            }
            if (!COUNT) {
                // places: the kept outputs of earlier waves and lanes of this round
#pragma unroll 1
                for (int o = 0; o < N; ++o) {
                    const unsigned long long b = __ballot((mask >> o) & 1u);
                    if (lane == 0) s_kw[wave][o] = (unsigned)__popcll(b);
                }
                __syncthreads();
            }
            // the segment's levels >= 2 from the block's LDS products (hc: their
            // row there, -1 when they are not cached)
            const unsigned long long hv = m / hdiv;
            const int hc = hv >= hv_lo && hv - hv_lo < (unsigned long long)n_hi ? (int)(hv - hv_lo) : -1;
            const int l_end = hc >= 0 ? 2 : LV::kMax;   // the global levels are 1 .. l_end - 1
            double2 up[kHoist ? N : 1], upf[kHoist ? N : 1];
            if constexpr (kHoist) {
#pragma unroll
                for (int o = 0; o < N; ++o) up[o] = upf[o] = make_double2(1.0, 0.0);
#pragma unroll
                for (int l = 1; l < LV::kMax; ++l) {
                    if (l < a.n_lv && l < l_end && active) {
                        const double2 *q = a.t + 2 * (((size_t)LV::S0 + (size_t)(l - 1) * LV::S + lv[l]) * N);
#pragma unroll
                        for (int o = 0; o < N; ++o) {
                            up[o] = cmul(up[o], q[2 * o]);
                            if (RHO) upf[o] = cmul(upf[o], q[2 * o + 1]);
                        }
                    }
                }
                if (hc >= 0 && active) {
#pragma unroll
                    for (int o = 0; o < N; ++o) {
                        up[o] = cmul(up[o], s_hi[2 * (hc * N + o)]);
                        if (RHO) upf[o] = cmul(upf[o], s_hi[2 * (hc * N + o) + 1]);
                    }
                }
            }
#pragma unroll kOutUnroll
            for (int o = 0; o < N; ++o) {
                const bool want = active && (COUNT || ((mask >> o) & 1u));
                unsigned long long place = 0;
                if (!COUNT) {
                    const unsigned long long b = __ballot((mask >> o) & 1u);
                    place = s_run[o] + __popcll(b & lanes_below(lane));
                    for (int w = 0; w < wave; ++w) place += s_kw[w][o];
                }
                if (want) {
                    double2 p = make_double2(1.0, 0.0), pf = p;
                    if (a.n_lv > 0) {
                        p = s_t0[2 * (lv[0] * N + o)];
                        if (RHO) pf = s_t0[2 * (lv[0] * N + o) + 1];
                    }
                    if constexpr (kHoist) {
                        double2 u = up[0], uf = upf[0];
#pragma unroll
                        for (int oo = 1; oo < N; ++oo)
                            if (oo == o) {
                                u = up[oo];
                                uf = upf[oo];
                            }
                        p = cmul(p, u);
                        if (RHO) pf = cmul(pf, uf);
                    } else {
#pragma unroll
                        for (int l = 1; l < LV::kMax; ++l) {
                            if (l < a.n_lv && l < l_end) {
                                const double2 *q =
                                    a.t + 2 * (((size_t)LV::S0 + (size_t)(l - 1) * LV::S + lv[l]) * N + o);
                                p = cmul(p, q[0]);
                                if (RHO) pf = cmul(pf, q[1]);
                            }
                        }
                        if (hc >= 0) {
                            p = cmul(p, s_hi[2 * (hc * N + o)]);
                            if (RHO) pf = cmul(pf, s_hi[2 * (hc * N + o) + 1]);
                        }
                    }
                    C sum = C{}, sumf = C{};
                    if (full) {
                        // the plain sum serves the rows of ones (uniform over the wave: o is)
                        C plain = C{};
                        if ((ones | ones_f) >> o & 1u) {
#pragma unroll
                            for (int i = 0; i < N; ++i) {
                                plain.x += x[i].x;
                                plain.y += x[i].y;
                            }
                        }
                        if (ones >> o & 1u) {
                            sum = plain;
                        } else {
#pragma unroll
                            for (int i = 0; i < N; ++i) cmac(sum, s_old[o * N + i], x[i]);
                        }
                        if (RHO) {
                            if (ones_f >> o & 1u) {
                                sumf = plain;
                            } else {
#pragma unroll
                                for (int i = 0; i < N; ++i) cmac(sumf, s_oldf[o * N + i], x[i]);
                            }
                        }
                    } else {
                        sum = cmul(s_old[o * N], x[0]);
                        if (RHO) sumf = cmul(s_oldf[o * N], x[0]);
                    }
                    const C out = cmul(from_d2<C>(p), sum);
                    if (COUNT) {
                        const double re = out.x, im = out.y, mag2 = fma(re, re, im * im);
                        if (squared ? mag2 > theta2 : sqrt(mag2) > a.theta) mask |= 1u << o;
                        if (RHO) {
                            const double2 w = cmul(pf, to_d2(sumf));
                            double2 &acc = s_acc[o * kFB + t];
                            acc.x += w.x;
                            acc.y += w.y;
                        }
                    } else if (place < a.capacity) {
                        a.keys_out[place] = m + a.stride_new * (unsigned long long)o;
                        vout[place] = conv<CS>(out);
                    }
                }
            }
            if (COUNT) {
                if (active) a.masks[kh] = (unsigned short)mask;
#pragma unroll 1
                for (int o = 0; o < N; ++o) {
                    const unsigned long long b = __ballot((mask >> o) & 1u);
                    if (lane == 0 && b) atomicAdd(&s_cnt[o], (unsigned)__popcll(b));
                }
            } else {
                __syncthreads();
                if (t < N) {
                    unsigned add = 0;
                    for (int w = 0; w < kWaves; ++w) add += s_kw[w][t];
                    s_run[t] += add;
                }
                __syncthreads();
            }
        }
        __syncthreads();                               // the tile's LDS is read before the next is staged
    }
    if (COUNT) {
        __syncthreads();
        if (t < N) a.bofs[(size_t)t * gridDim.x + blockIdx.x] = s_cnt[t];
        if (RHO) {
            for (int o = 0; o < N; ++o) {
                double2 v = s_acc[o * kFB + t];
                for (int off = 32; off > 0; off >>= 1) {
                    v.x += __shfl_xor(v.x, off, 64);
                    v.y += __shfl_xor(v.y, off, 64);
                }
                if (lane == 0) s_red[wave][o] = v;
            }
            __syncthreads();
            if (t < N) {
                double2 r = make_double2(0.0, 0.0);
                for (int w = 0; w < kWaves; ++w) {
                    r.x += s_red[w][t].x;
                    r.y += s_red[w][t].y;
                }
                a.partials[(size_t)blockIdx.x * N + t] = r;
            }
        }
    }
}

// Exclusive offsets of the n per-(o, block) counts in place (one block of
// kOffB threads, each owning a contiguous run of at most kOffMax counts,
// read once into registers), the total kept outputs, the new entry count (at
// most the capacity) and the sticky overflow flag.
constexpr int kOffB = 1024;
constexpr int kOffMax = 16 * kFilterStepBlocks / kOffB;
__global__ void __launch_bounds__(kOffB) filter_offsets_kernel(unsigned long long *bofs, int n,
                                                               unsigned long long capacity,
                                                               unsigned long long *count_out, int *overflow) {
    __shared__ unsigned long long s_w[kOffB / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (n + kOffB - 1) / kOffB;
    const int lo = std::min(n, t * per), hi = std::min(n, lo + per);
    unsigned long long v[kOffMax];
    unsigned long long mine = 0;
#pragma unroll
    for (int k = 0; k < kOffMax; ++k) {
        v[k] = lo + k < hi ? bofs[lo + k] : 0ull;
        mine += v[k];
    }
    unsigned long long x = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    unsigned long long run = x - mine, total = 0;
    for (int w = 0; w < kOffB / 64; ++w) {
        if (w < wave) run += s_w[w];
        total += s_w[w];
    }
#pragma unroll
    for (int k = 0; k < kOffMax; ++k) {
        if (lo + k < hi) bofs[lo + k] = run;
        run += v[k];
    }
    if (t == 0) {
        *count_out = total < capacity ? total : capacity;
        if (total > capacity) *overflow = 1;
    }
}

// The initial tensor: rho0[o] times the initial self factor (FP64), kept if
// its magnitude is above theta; one thread, N <= 16 entries.
template <typename CS>
__global__ void filter_init_kernel(const double2 *rho0, const double2 *bank, int self_end_tab, int N, double theta,
                                   unsigned long long capacity, unsigned long long *keys, void *vals,
                                   unsigned long long *count, int *overflow) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long k = 0;
    for (int o = 0; o < N; ++o) {
        const double2 v = cmul(rho0[o], bank[(size_t)self_end_tab * N * N + o * N]);
        if (sqrt(fma(v.x, v.x, v.y * v.y)) > theta) {
            if (k < capacity) {
                keys[k] = (unsigned long long)o;
                ((CS *)vals)[k] = conv<CS>(v);
            }
            ++k;
        }
    }
    *count = k < capacity ? k : capacity;
    *overflow = k > capacity ? 1 : 0;
}

template <int N, typename S, typename T>
hipError_t launch_filter_step_t(const FilterStepArgs &a, bool count, bool rho, hipStream_t st) {
    const dim3 g(kFilterStepBlocks), b(kFB);
    if (count && rho)
        hipLaunchKernelGGL((filter_step_kernel<N, S, T, true, true>), g, b, filter_step_lds_bytes(N, true), st, a);
    else if (count) hipLaunchKernelGGL((filter_step_kernel<N, S, T, true, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((filter_step_kernel<N, S, T, false, false>), g, b, 0, st, a);
    return hipGetLastError();
}

template <int N>
hipError_t launch_filter_step_n(int prec, const FilterStepArgs &a, bool count, bool rho, hipStream_t st) {
    switch (prec) {
    case kPrecC128: return launch_filter_step_t<N, double, double>(a, count, rho, st);
    case kPrecC64: return launch_filter_step_t<N, float, float>(a, count, rho, st);
    case kPrecC64F64: return launch_filter_step_t<N, float, double>(a, count, rho, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t filter_step_lds_bytes(int N, bool rho) { return rho ? (size_t)N * kFB * sizeof(double2) : 0; }

int filter_levels(int N, int n_digits) {
    if (n_digits <= 0) return 0;
    const int D0 = filter_level0_digits(N), D = filter_level_digits(N);
    return 1 + (std::max(n_digits - D0, 0) + D - 1) / D;
}

size_t filter_plan_entries(int N, int n_digits) {
    const int n_lv = filter_levels(N, n_digits);
    if (n_lv == 0) return 0;
    return (size_t)N * (filter_level0_size(N) + (size_t)(n_lv - 1) * filter_level_size(N));
}

hipError_t launch_filter_plan(const FilterPlanArgs &a, hipStream_t st) {
    const long long total = (long long)filter_plan_entries(a.N, a.nd);
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<long long>(1024, (total + kFB - 1) / kFB);
    hipLaunchKernelGGL(filter_plan_kernel, dim3(grid), dim3(kFB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_filter_step(int N, int prec, const FilterStepArgs &a, bool count, bool rho, hipStream_t st) {
    switch (N) {
    case 1: return launch_filter_step_n<1>(prec, a, count, rho, st);
    case 4: return launch_filter_step_n<4>(prec, a, count, rho, st);
    case 9: return launch_filter_step_n<9>(prec, a, count, rho, st);
    case 16: return launch_filter_step_n<16>(prec, a, count, rho, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_filter_offsets(int N, unsigned long long *bofs, unsigned long long capacity,
                                 unsigned long long *count_out, int *overflow, hipStream_t st) {
    if (N * kFilterStepBlocks > kOffB * kOffMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(filter_offsets_kernel, dim3(1), dim3(kOffB), 0, st, bofs, N * kFilterStepBlocks, capacity,
                       count_out, overflow);
    return hipGetLastError();
}

hipError_t launch_filter_init(int prec, const double2 *rho0, const double2 *bank, int self_end_tab, int N,
                              double theta, unsigned long long capacity, unsigned long long *keys, void *vals,
                              unsigned long long *count, int *overflow, hipStream_t st) {
    if (prec == kPrecC128)
        hipLaunchKernelGGL(filter_init_kernel<double2>, dim3(1), dim3(64), 0, st, rho0, bank, self_end_tab, N, theta,
                           capacity, keys, vals, count, overflow);
    else
        hipLaunchKernelGGL(filter_init_kernel<float2>, dim3(1), dim3(64), 0, st, rho0, bank, self_end_tab, N, theta,
                           capacity, keys, vals, count, overflow);
    return hipGetLastError();
}

}  // namespace quapi
