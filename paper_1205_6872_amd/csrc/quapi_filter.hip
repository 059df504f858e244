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
// sorted by the new key: no sort is needed, only exclusive scans to place
// them.  rho(t_n) comes from the same segments with the final-point classes.
//
// A step is: segment heads, their scan and the segment starts; a counting
// pass (keep flags per (o, segment) and the rho block partials); the scan of
// the flags; a writing pass that recomputes the outputs and stores the kept
// ones at their places.  Every pass has a fixed grid and reads its element
// count from device memory, so a run needs no host synchronization, and the
// integer scans and fixed-order partial sums make it deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "quapi_device.h"
#include "quapi_internal.h"

namespace quapi {
namespace {

constexpr int kFB = kFilterBlock;        // threads per block
constexpr int kScanItems = 4;            // scan items per thread and tile
constexpr int kScanTile = kFB * kScanItems;

// ------------------------------------------------------------------ scans
// Exclusive scan of x[0 .. n), n = *n_dev, in place, with kFilterScanBlocks
// blocks each owning one contiguous chunk: (1) chunk sums, (2) a scan of the
// sums (and the total to *total), (3) each chunk rescanned from its offset.
__device__ __forceinline__ unsigned long long scan_chunk(unsigned long long n, int b, unsigned long long *lo) {
    const unsigned long long chunk = (n + kFilterScanBlocks - 1) / kFilterScanBlocks;
    *lo = chunk * b;
    const unsigned long long hi = *lo + chunk;
    return hi < n ? hi : n;
}

// Block-wide exclusive scan of one value per thread: returns the prefix, and
// the block total in *tot.  Every thread of the block must call it.
__device__ unsigned block_excl_scan(unsigned v, unsigned *s_w, unsigned *tot) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    unsigned x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    unsigned before = 0, all = 0;
    for (int w = 0; w < kFB / 64; ++w) {
        if (w < wave) before += s_w[w];
        all += s_w[w];
    }
    __syncthreads();
    *tot = all;
    return before + x - v;
}

__global__ void __launch_bounds__(kFB) scan_sums_kernel(const unsigned *__restrict__ x,
                                                        const unsigned long long *n_dev, unsigned *sums) {
    __shared__ unsigned s_w[kFB / 64];
    unsigned long long lo;
    const unsigned long long hi = scan_chunk(*n_dev, blockIdx.x, &lo);
    unsigned acc = 0;
    for (unsigned long long k = lo + threadIdx.x; k < hi; k += kFB) acc += x[k];
    unsigned tot;
    (void)block_excl_scan(acc, s_w, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kFB) scan_offsets_kernel(unsigned *sums, unsigned long long *total) {
    __shared__ unsigned s_w[kFB / 64];
    constexpr int per = kFilterScanBlocks / kFB;
    unsigned v[per], acc = 0;
    for (int k = 0; k < per; ++k) {
        v[k] = sums[threadIdx.x * per + k];
        acc += v[k];
    }
    unsigned tot;
    unsigned run = block_excl_scan(acc, s_w, &tot);
    for (int k = 0; k < per; ++k) {
        sums[threadIdx.x * per + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ void __launch_bounds__(kFB) scan_apply_kernel(unsigned *__restrict__ x, const unsigned long long *n_dev,
                                                         const unsigned *__restrict__ offsets) {
    __shared__ unsigned s_w[kFB / 64];
    unsigned long long lo;
    const unsigned long long hi = scan_chunk(*n_dev, blockIdx.x, &lo);
    unsigned run = offsets[blockIdx.x];
    for (unsigned long long base = lo; base < hi; base += kScanTile) {
        unsigned v[kScanItems], acc = 0;
        const unsigned long long k0 = base + (unsigned long long)kScanItems * threadIdx.x;
        for (int u = 0; u < kScanItems; ++u) {
            v[u] = k0 + u < hi ? x[k0 + u] : 0u;
            acc += v[u];
        }
        unsigned tot;
        unsigned p = run + block_excl_scan(acc, s_w, &tot);
        for (int u = 0; u < kScanItems; ++u) {
            if (k0 + u < hi) x[k0 + u] = p;
            p += v[u];
        }
        run += tot;
    }
}

// -------------------------------------------------------------- segments
// The digits a segment shares: all but the oldest (full window), or all.
template <int N>
__device__ __forceinline__ unsigned long long seg_of(unsigned long long key, bool full) {
    return full ? key / N : key;
}

// head[k] = 1 where entry k starts a segment.
template <int N>
__global__ void __launch_bounds__(kFB) seg_head_kernel(const unsigned long long *__restrict__ keys,
                                                       const unsigned long long *n_dev, int full,
                                                       unsigned *__restrict__ head) {
    const unsigned long long n = *n_dev;
    for (unsigned long long k = (unsigned long long)blockIdx.x * kFB + threadIdx.x; k < n;
         k += (unsigned long long)gridDim.x * kFB)
        head[k] = (k == 0 || seg_of<N>(keys[k - 1], full) != seg_of<N>(keys[k], full)) ? 1u : 0u;
}

// seg_start[s] = the first entry of segment s, seg_start[S] = n; *nseg = S,
// *nflags = S * N (the outputs of the step).  excl: the scanned heads.
template <int N>
__global__ void __launch_bounds__(kFB) seg_start_kernel(const unsigned long long *__restrict__ keys,
                                                        const unsigned long long *n_dev, int full,
                                                        const unsigned *__restrict__ excl,
                                                        const unsigned long long *n_heads,
                                                        unsigned *__restrict__ seg_start, unsigned long long *nseg,
                                                        unsigned long long *nflags) {
    const unsigned long long n = *n_dev;
    for (unsigned long long k = (unsigned long long)blockIdx.x * kFB + threadIdx.x; k < n;
         k += (unsigned long long)gridDim.x * kFB)
        if (k == 0 || seg_of<N>(keys[k - 1], full) != seg_of<N>(keys[k], full)) seg_start[excl[k]] = (unsigned)k;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long S = *n_heads;
        seg_start[S] = (unsigned)n;
        *nseg = S;
        *nflags = S * N;
    }
}

// ------------------------------------------------------------ factor tables
// The factor product over the digits of m is split into levels of D digits:
// T_l[o][v] = prod over the digits of v of Tab_{lD + j}[o][digit_j(v)], so that
// P(o, m) = prod_l T_l[o][(m / S^l) % S] with S = N^D (FP64).  S is a power of
// two for N = 4, 16 and a compile-time constant for N = 9.
template <int N> struct FilterLevel {
    static constexpr int S = N == 4 ? 4096 : N == 9 ? 729 : N == 16 ? 4096 : 1;
};

__host__ __device__ inline int filter_level_size(int N) {
    return N == 4 ? 4096 : N == 9 ? 729 : N == 16 ? 4096 : 1;
}
__host__ __device__ inline int filter_level_digits(int N) { return N == 4 ? 6 : N == 1 ? 1 : 3; }

__global__ void __launch_bounds__(kFB) filter_plan_kernel(const FilterPlanArgs a) {
    const int N = a.N, S = filter_level_size(N), D = filter_level_digits(N);
    const long long per = (long long)N * S;
    const long long total = per * a.n_lv;
    const double2 one = make_double2(1.0, 0.0);
    for (long long idx = (long long)blockIdx.x * kFB + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * kFB) {
        const int l = (int)(idx / per);
        const int o = (int)((idx % per) / S);
        int v = (int)(idx % S);
        double2 p = one, pf = one;
        for (int j = l * D; j < a.nd && j < (l + 1) * D; ++j) {
            const int dg = v % N;
            v /= N;
            p = cmul(p, a.bank[(size_t)a.tab[j] * (N * N) + o * N + dg]);
            pf = cmul(pf, a.bank[(size_t)a.tabf[j] * (N * N) + o * N + dg]);
        }
        a.t[idx] = p;
        a.tf[idx] = pf;
    }
}

// ------------------------------------------------------------------- step
// The outputs of segment s for every new point o.  COUNT: the keep flags at
// [o * nseg + s] and, with RHO, the block partial sums of rho(t_n); otherwise
// the kept outputs at the places the scanned flags give.  The loop over o is
// not unrolled (at N = 9, 16 an unrolled one spills); each thread's rho sums
// sit in dynamic LDS, [o][thread] (filter_step_lds_bytes).
template <int N, typename S, typename T, bool COUNT, bool RHO>
__global__ void __launch_bounds__(kFB) filter_step_kernel(const FilterStepArgs a) {
    using C = typename Cx<T>::type;
    using CS = typename Cx<S>::type;
    using LV = FilterLevel<N>;
    extern __shared__ __align__(16) unsigned char f_smem[];
    double2 *s_acc = (double2 *)f_smem;
    __shared__ C s_old[N * N], s_oldf[N * N];
    __shared__ double2 s_red[kFB / 64][RHO ? N : 1];
    const int t = threadIdx.x;
    const bool full = a.full != 0;
    const double2 *__restrict__ bank = a.bank;
    for (int idx = t; idx < N * N; idx += kFB) {
        s_old[idx] = from_d2<C>(bank[(size_t)a.old_tab * (N * N) + idx]);
        if (RHO) s_oldf[idx] = from_d2<C>(bank[(size_t)a.oldf_tab * (N * N) + idx]);
    }
    if (RHO)
        for (int o = 0; o < N; ++o) s_acc[o * kFB + t] = make_double2(0.0, 0.0);
    __syncthreads();
    const unsigned long long nseg = *a.nseg;
    const unsigned long long nflags = nseg * N;
    const CS *__restrict__ vin = (const CS *)a.vals_in;
    CS *__restrict__ vout = (CS *)a.vals_out;
    const double2 *__restrict__ tp = a.t;
    const double2 *__restrict__ tpf = a.tf;
    for (unsigned long long s = (unsigned long long)blockIdx.x * kFB + t; s < nseg;
         s += (unsigned long long)gridDim.x * kFB) {
        const unsigned k0 = a.seg_start[s], k1 = a.seg_start[s + 1];
        const unsigned long long m = seg_of<N>(a.keys_in[k0], full);
        // the segment's values by oldest digit (the dropped ones are zero)
        C x[N];
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = C{};
        if (full) {
            for (unsigned k = k0; k < k1; ++k) {
                const int i = (int)(a.keys_in[k] % N);
                const C v = conv<C>(vin[k]);
#pragma unroll
                for (int ii = 0; ii < N; ++ii)
                    if (ii == i) x[ii] = v;
            }
        } else {
            x[0] = conv<C>(vin[k0]);
        }
#pragma unroll 1
        for (int o = 0; o < N; ++o) {
            double2 p = make_double2(1.0, 0.0), pf = p;
            unsigned long long v = m;
            for (int l = 0; l < a.n_lv; ++l) {
                const size_t e = ((size_t)l * N + o) * LV::S + (size_t)(v % LV::S);
                v /= LV::S;
                p = cmul(p, tp[e]);
                if (RHO) pf = cmul(pf, tpf[e]);
            }
            C sum = C{}, sumf = C{};
            if (full) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    cmac(sum, s_old[o * N + i], x[i]);
                    if (RHO) cmac(sumf, s_oldf[o * N + i], x[i]);
                }
            } else {
                sum = cmul(s_old[o * N], x[0]);
                if (RHO) sumf = cmul(s_oldf[o * N], x[0]);
            }
            const C out = cmul(from_d2<C>(p), sum);
            const unsigned long long slot = (unsigned long long)o * nseg + s;
            if (COUNT) {
                const double re = out.x, im = out.y;
                a.flags[slot] = sqrt(fma(re, re, im * im)) > a.theta ? 1u : 0u;
                if (RHO) {
                    const double2 w = cmul(pf, to_d2(sumf));
                    double2 &r = s_acc[o * kFB + t];
                    r.x += w.x;
                    r.y += w.y;
                }
            } else {
                // kept in the counting pass iff the scan steps up after this slot
                const unsigned long long pos = a.flags[slot];
                const unsigned long long next = slot + 1 < nflags ? a.flags[slot + 1] : *a.total;
                if (next > pos && pos < a.capacity) {
                    a.keys_out[pos] = m + a.stride_new * (unsigned long long)o;
                    vout[pos] = conv<CS>(out);
                }
            }
        }
    }
    if (COUNT && RHO) {
        const int lane = t & 63, wave = t >> 6;
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
            for (int w = 0; w < kFB / 64; ++w) {
                r.x += s_red[w][t].x;
                r.y += s_red[w][t].y;
            }
            a.partials[(size_t)blockIdx.x * N + t] = r;
        }
    }
}

// The entry count after a step (at most the capacity) and the overflow flag.
__global__ void filter_count_kernel(const unsigned long long *total, unsigned long long capacity,
                                    unsigned long long *count_out, int *overflow) {
    const unsigned long long k = *total;
    *count_out = k < capacity ? k : capacity;
    if (k > capacity) *overflow = 1;
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

template <int N>
hipError_t launch_filter_segments_n(const FilterSegArgs &a, hipStream_t st) {
    const dim3 g(kFilterStepBlocks), b(kFB);
    hipLaunchKernelGGL((seg_head_kernel<N>), g, b, 0, st, a.keys, a.count, a.full, a.flags);
    hipError_t e = launch_filter_scan(a.flags, a.count, a.sums, a.total, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((seg_start_kernel<N>), g, b, 0, st, a.keys, a.count, a.full, a.flags, a.total, a.seg_start,
                       a.nseg, a.nflags);
    return hipGetLastError();
}

}  // namespace

size_t filter_step_lds_bytes(int N, bool rho) { return rho ? (size_t)N * kFB * sizeof(double2) : 0; }

int filter_levels(int N, int n_digits) {
    const int D = filter_level_digits(N);
    return (n_digits + D - 1) / D;
}

size_t filter_plan_entries(int N, int n_digits) {
    return (size_t)filter_levels(N, n_digits) * N * filter_level_size(N);
}

hipError_t launch_filter_plan(const FilterPlanArgs &a, hipStream_t st) {
    const long long total = (long long)filter_plan_entries(a.N, a.nd);
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<long long>(1024, (total + kFB - 1) / kFB);
    hipLaunchKernelGGL(filter_plan_kernel, dim3(grid), dim3(kFB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_filter_scan(unsigned *x, const unsigned long long *n_dev, unsigned *sums,
                              unsigned long long *total, hipStream_t st) {
    static_assert(kFilterScanBlocks % kFB == 0, "the offsets scan gives each thread kFilterScanBlocks / kFB sums");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(kFilterScanBlocks), dim3(kFB), 0, st, x, n_dev, sums);
    hipLaunchKernelGGL(scan_offsets_kernel, dim3(1), dim3(kFB), 0, st, sums, total);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(kFilterScanBlocks), dim3(kFB), 0, st, x, n_dev, sums);
    return hipGetLastError();
}

hipError_t launch_filter_segments(int N, const FilterSegArgs &a, hipStream_t st) {
    switch (N) {
    case 1: return launch_filter_segments_n<1>(a, st);
    case 4: return launch_filter_segments_n<4>(a, st);
    case 9: return launch_filter_segments_n<9>(a, st);
    case 16: return launch_filter_segments_n<16>(a, st);
    default: return hipErrorInvalidValue;
    }
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

hipError_t launch_filter_count(const unsigned long long *total, unsigned long long capacity,
                               unsigned long long *count_out, int *overflow, hipStream_t st) {
    hipLaunchKernelGGL(filter_count_kernel, dim3(1), dim3(1), 0, st, total, capacity, count_out, overflow);
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
