// common.hpp -- small device-side helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define AGN_DEV __device__ __forceinline__

template <typename T>
struct __align__(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T> AGN_DEV cplx<T> cmk(T r, T i) { cplx<T> c; c.re = r; c.im = i; return c; }
template <typename T> AGN_DEV cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename T> AGN_DEV cplx<T> csub(cplx<T> a, cplx<T> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename T> AGN_DEV cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> AGN_DEV cplx<T> cconj(cplx<T> a) { return cmk(a.re, -a.im); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> AGN_DEV cplx<T> cmul_mi(cplx<T> a) {
    return INV ? cmk(-a.im, a.re) : cmk(a.im, -a.re);
}

// Order-preserving unsigned keys for IEEE values (ascending float order maps
// to ascending unsigned order); -0 is folded onto +0 so that the two tie.
AGN_DEV uint32_t ord_key(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
AGN_DEV uint64_t ord_key(double f) {
    uint64_t u = (uint64_t)__double_as_longlong(f);
    if (u == 0x8000000000000000ull) u = 0ull;
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// Returns x unchanged but opaque to the optimiser, so that per-item address
// arithmetic derived from it is recomputed where it is used instead of being
// hoisted out of long loops and kept live in registers.
AGN_DEV int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <typename T> struct key_of;
template <> struct key_of<float> { typedef uint32_t type; };
template <> struct key_of<double> { typedef uint64_t type; };
