// Shared device/host helpers for the RTE library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace rte {

// Complex number with the real and imaginary part interleaved (matches complex64/complex128).
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ inline cx<T> scale(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
// multiply by +i / -i
template <typename T>
__host__ __device__ inline cx<T> mul_i(cx<T> a) { return mk(-a.im, a.re); }
template <typename T>
__host__ __device__ inline cx<T> mul_mi(cx<T> a) { return mk(a.im, -a.re); }
// a += b * c
template <typename T>
__host__ __device__ inline void cmac(cx<T>& a, cx<T> b, cx<T> c) {
    // a += b c as four fused multiply-adds into the accumulator (no separately rounded product)
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}

template <typename To, typename Ti>
__host__ __device__ inline cx<To> cvt(cx<Ti> a) { return mk((To)a.re, (To)a.im); }

// Two consecutive elements of a real vector, loaded or stored as one access.
template <typename T>
struct pair_of;
template <>
struct pair_of<double> { using type = double2; };
template <>
struct pair_of<float> { using type = float2; };

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
inline int next_pow2(int v) { int p = 1; while (p < v) p <<= 1; return p; }

// Device-side status codes written by kernels that can detect bad input.
enum { DEV_OK = 0 };

}  // namespace rte

#define RTE_HIP_TRY(expr)                                                          \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) return ::rte::set_hip_error(_e, #expr, __FILE__, __LINE__); \
    } while (0)

namespace rte {
int set_error(int code, const char* fmt, ...);
int set_hip_error(hipError_t e, const char* what, const char* file, int line);
}  // namespace rte
