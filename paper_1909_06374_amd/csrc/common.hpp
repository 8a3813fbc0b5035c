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

// Global-memory pointers typed as such.  Through a generic pointer the
// compiler emits flat loads, which count against both the vector-memory and
// the LDS counters, so every wait for LDS traffic also waits for them; typed
// global loads are counted by the vector-memory counter alone.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> AGN_DEV const gmem<T>* as_global(const T* p) { return (const gmem<T>*)p; }
template <typename T> AGN_DEV gmem<T>* as_global(T* p) { return (gmem<T>*)p; }

// Complex values through typed global pointers, as one 2-element vector load
// or store (a struct cannot be copied out of another address space).
template <typename T> struct vec2_of { typedef T type __attribute__((ext_vector_type(2))); };
template <typename T> AGN_DEV cplx<T> gload(const gmem<cplx<T>>* p) {
    const typename vec2_of<T>::type v = *(const gmem<typename vec2_of<T>::type>*)p;
    cplx<T> r;
    r.re = v.x;
    r.im = v.y;
    return r;
}
template <typename T> AGN_DEV void gstore(gmem<cplx<T>>* p, cplx<T> a) {
    typename vec2_of<T>::type v;
    v.x = a.re;
    v.y = a.im;
    *(gmem<typename vec2_of<T>::type>*)p = v;
}

template <typename T> struct key_of;
template <> struct key_of<float> { typedef uint32_t type; };
template <> struct key_of<double> { typedef uint64_t type; };
