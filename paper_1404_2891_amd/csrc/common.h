// Internal definitions shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "../../include/feast_mi355x.h"

namespace fm {

// Interleaved complex value, layout-compatible with double _Complex / float _Complex.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
    cplx() = default;
    __host__ __device__ cplx(T r, T i = 0) : re(r), im(i) {}
    template <typename U>
    __host__ __device__ explicit cplx(const cplx<U>& o) : re(T(o.re)), im(T(o.im)) {}
};

template <typename T>
__host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T>
__host__ __device__ inline T abs1(cplx<T> a) {  // |re| + |im|, the pivot metric
    return (a.re < 0 ? -a.re : a.re) + (a.im < 0 ? -a.im : a.im);
}
template <typename T>
__host__ __device__ inline cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    // Smith's algorithm: avoids overflow of |b|^2
    T ar = b.re < 0 ? -b.re : b.re, ai = b.im < 0 ? -b.im : b.im;
    if (ar >= ai) {
        T r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        T r = b.re / b.im, d = b.im + b.re * r;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}

using z64 = cplx<double>;
using c32 = cplx<float>;

// Work precision of the node factorisations.
enum class Prec { F64 = 0, F32 = 1, F16 = 2 };

inline int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    fprintf(stderr, "[feast_mi355x] %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
    return FEAST_EDEVICE;
}

#define FM_HIP(call)                                                      \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return fm::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define FM_TRY(call)                  \
    do {                              \
        int rc_ = (call);             \
        if (rc_ != 0) return rc_;     \
    } while (0)

#define FM_LAUNCH_CHECK() FM_HIP(hipGetLastError())

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace fm
