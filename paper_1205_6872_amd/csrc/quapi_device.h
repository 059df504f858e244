// Device-side helpers shared by the kernel sources: complex arithmetic in
// double2 / float2, storage <-> arithmetic conversions, LDS carving and
// wave-uniform coefficient reads.
#pragma once

#include <hip/hip_runtime.h>

#include "quapi_internal.h"

namespace quapi {
namespace {

// ---------------------------------------------------------------- complex
template <typename T> struct Cx;
template <> struct Cx<double> { using type = double2; };
template <> struct Cx<float> { using type = float2; };

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
// c += a * b
__device__ __forceinline__ void cmac(double2 &c, double2 a, double2 b) {
    c.x = fma(a.x, b.x, c.x);
    c.x = fma(-a.y, b.y, c.x);
    c.y = fma(a.x, b.y, c.y);
    c.y = fma(a.y, b.x, c.y);
}
__device__ __forceinline__ void cmac(float2 &c, float2 a, float2 b) {
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(-a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(a.y, b.x, c.y);
}
template <typename C> __device__ __forceinline__ C from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
// storage <-> arithmetic complex types (identity, widen, or round to nearest)
template <typename To> __device__ __forceinline__ To conv(double2 v);
template <typename To> __device__ __forceinline__ To conv(float2 v);
template <> __device__ __forceinline__ double2 conv<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 conv<float2>(float2 v) { return v; }
template <> __device__ __forceinline__ double2 conv<double2>(float2 v) { return make_double2(v.x, v.y); }
template <> __device__ __forceinline__ float2 conv<float2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}

// ------------------------------------------------- the rows that carry the trace
// The entries of a diagonal new point o = (a, a) are K[o, p] times a plain
// sum over the summed point (every influence factor of a diagonal point is
// one), and sum_a K[(a, a), p] = delta_p exactly (the trace-exact rounding of
// K), so these rows carry the trace of rho from step to step.  With FP32
// arithmetic, rounding that sum before the products leaves an error in the
// trace at every step (L = 15, 1000 steps: 1.5e-6).  TraceSum<float2> forms
// the sum of the FP32 values exactly -- in FP64, which holds the sum of four
// FP32 values without rounding, the result an error-free (TwoSum) pair would
// give with more instructions -- and rounds each product k * sum once to FP32
// (2.7e-7 at L = 15, 1000 steps).  With FP64 arithmetic it is the plain sum
// and product.
template <typename C> struct TraceSum;
template <> struct TraceSum<double2> {
    double2 s;
    __device__ __forceinline__ void init(double2 v) { s = v; }
    __device__ __forceinline__ void add(double2 v) { s = cadd(s, v); }
    __device__ __forceinline__ double2 times(double2 k) const { return cmul(k, s); }       // k * sum
    __device__ __forceinline__ double2 times_right(double2 k) const { return cmul(s, k); } // sum * k
    __device__ __forceinline__ double2 rounded() const { return s; }
};
template <> struct TraceSum<float2> {
    double2 s;          // the exact sum of the FP32 values (FP64 holds it without rounding)
    __device__ __forceinline__ void init(float2 v) { s = make_double2(v.x, v.y); }
    __device__ __forceinline__ void add(float2 v) {
        s.x += (double)v.x;
        s.y += (double)v.y;
    }
    // k * sum, rounded once to FP32 per component
    __device__ __forceinline__ float2 times(float2 k) const {
        const double kx = k.x, ky = k.y;
        return make_float2((float)fma(kx, s.x, -ky * s.y), (float)fma(kx, s.y, ky * s.x));
    }
    __device__ __forceinline__ float2 times_right(float2 k) const { return times(k); }
    // the plain FP32 sum
    __device__ __forceinline__ float2 rounded() const { return make_float2((float)s.x, (float)s.y); }
};

// ------------------------------------------------------------------- LDS
// Carve `bytes` (16-byte aligned) out of a dynamic LDS block at offset `off`.
__host__ __device__ inline unsigned lds_take(unsigned &off, unsigned bytes) {
    const unsigned o = off;
    off = (off + bytes + 15u) & ~15u;
    return o;
}

// Wave-uniform read of a coefficient through the constant address space, so
// that it is fetched by a scalar load into scalar registers (the FMAs then
// take it as their scalar operand) instead of being broadcast to all 64 lanes
// from LDS.
template <typename T>
__device__ __forceinline__ typename Cx<T>::type coef_ld(const T *p, int k) {
    const __attribute__((address_space(4))) T *q = (const __attribute__((address_space(4))) T *)p;
    typename Cx<T>::type v;
    v.x = q[2 * k];
    v.y = q[2 * k + 1];
    return v;
}

}  // namespace
}  // namespace quapi
