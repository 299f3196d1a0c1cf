// rt_device.h -- FP32 complex and vector helpers for the gfx950 kernels.
//
// Complex numbers are (re, im) pairs of float held in VGPRs, the real-valued
// representation of complex quantities (Sec. "Channel Coefficients, Delays,
// and Doppler Shifts Computation", remark on real-valued representations).
// All routines are written from their mathematical definitions.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rtd {

struct cf {
    float re, im;
};

__device__ __forceinline__ cf mkc(float r, float i) { return cf{r, i}; }
__device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return cf{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
    return cf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cf cscale(cf a, float s) { return cf{a.re * s, a.im * s}; }
__device__ __forceinline__ cf cconj(cf a) { return cf{a.re, -a.im}; }
__device__ __forceinline__ float cabs2(cf a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
__device__ __forceinline__ cf cmulc(cf a, cf b) {
    return cf{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a / b: multiply by conj(b) / |b|^2.  Magnitudes in this library stay far
// inside the FP32 range (|eta| <= ~1e8), so no rescaling is needed.  The
// reciprocal is the hardware one (about 1 ulp).
__device__ __forceinline__ cf cdiv(cf a, cf b) {
    float inv = __builtin_amdgcn_rcpf(cabs2(b));
    return cf{(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
// Principal square root (Re >= 0).  With m = |z|:
//   Re >= 0 branch:  t = sqrt((m + x)/2),  sqrt(z) = t + j y/(2t)
//   x < 0:           t = sqrt((m - x)/2),  sqrt(z) = |y|/(2t) + j sign(y) t
// choosing the branch that avoids cancellation in m +- x.  Hardware square
// root and reciprocal (about 1 ulp each).
__device__ __forceinline__ cf csqrt_principal(cf z) {
    float x = z.re, y = z.im;
    float m = __builtin_amdgcn_sqrtf(x * x + y * y);
    if (m == 0.0f) return cf{0.0f, 0.0f};
    if (x >= 0.0f) {
        float t = __builtin_amdgcn_sqrtf(0.5f * (m + x));
        return cf{t, y * __builtin_amdgcn_rcpf(2.0f * t)};
    }
    float t = __builtin_amdgcn_sqrtf(0.5f * (m - x));
    return cf{fabsf(y) * __builtin_amdgcn_rcpf(2.0f * t), copysignf(t, y)};
}

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 unit3(float3 a) { return a * __builtin_amdgcn_rsqf(dot3(a, a)); }

// 2x2 complex matrix, row-major: [a b; c d]
struct cm2 {
    cf a, b, c, d;
};

}  // namespace rtd
