// sbr_common.h -- device building blocks of the SBR path (gfx950).
//
//   * Fibonacci ray generation with an exact 64-bit fixed-point phase
//     (Sec. "Sampling Initial Ray Directions")
//   * transmit field C_T in the launch basis (theta_hat, phi_hat) of a rotated
//     antenna (eq. rotation, eq. theta_phi_prime, eq. F_prime_2_F, eq. C),
//     templated on the scalar so that the adjoint can run it on dual numbers
//   * watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013)
//   * two-child slab test with a conservative upper bound
//   * vacuum Fresnel coefficients (eq. fresnel_vac) and their eta-derivatives
//   * the basis change W of eq. fresnel_in_vectors / eq. fresnel_out_vectors
#pragma once
#include <hip/hip_runtime.h>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtd {

// round(2^64 (phi_g - 1)): frac(n / phi_g) = frac(n (phi_g - 1)) = (n * C mod 2^64) / 2^64
constexpr uint64_t kPhiFrac = 0x9e3779b97f4a7c16ull;

// ---------------------------------------------------------------- duals
// FP32 forward-mode scalar carrying d/d(yaw, pitch, roll).
struct d3f {
    float v, d0, d1, d2;
};
__device__ __forceinline__ d3f operator+(d3f a, d3f b) { return d3f{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2}; }
__device__ __forceinline__ d3f operator-(d3f a, d3f b) { return d3f{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2}; }
__device__ __forceinline__ d3f operator-(d3f a) { return d3f{-a.v, -a.d0, -a.d1, -a.d2}; }
__device__ __forceinline__ d3f operator*(d3f a, d3f b) {
    return d3f{a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
__device__ __forceinline__ d3f chainf(d3f a, float f, float fp) { return d3f{f, fp * a.d0, fp * a.d1, fp * a.d2}; }
__device__ __forceinline__ d3f dsqrtf(d3f a) {
    float r = sqrtf(fmaxf(a.v, 0.0f));
    return chainf(a, r, r > 0.0f ? 0.5f / r : 0.0f);
}
__device__ __forceinline__ d3f drecip(d3f a) {
    float r = 1.0f / a.v;
    return chainf(a, r, -r * r);
}
__device__ __forceinline__ d3f dpowf(d3f a, float p) {
    float f = powf(fmaxf(a.v, 0.0f), p);
    return chainf(a, f, a.v > 0.0f ? p * f / a.v : 0.0f);
}
__device__ __forceinline__ float dsqrtf(float a) { return sqrtf(fmaxf(a, 0.0f)); }
__device__ __forceinline__ float drecip(float a) { return 1.0f / a; }
__device__ __forceinline__ float dpowf(float a, float p) { return powf(fmaxf(a, 0.0f), p); }
__device__ __forceinline__ float val(float a) { return a; }
__device__ __forceinline__ float val(d3f a) { return a.v; }
__device__ __forceinline__ float with_value(float, float v) { return v; }
__device__ __forceinline__ d3f with_value(d3f a, float v) { return d3f{v, a.d0, a.d1, a.d2}; }

template <typename S>
__device__ __forceinline__ S cst(float v);
template <>
__device__ __forceinline__ float cst<float>(float v) { return v; }
template <>
__device__ __forceinline__ d3f cst<d3f>(float v) { return d3f{v, 0.f, 0.f, 0.f}; }

// Entry (i, j) of R = Rz(yaw) Ry(pitch) Rx(roll) (eq. rotation) with its
// angle derivatives, both precomputed on the host per transmitter.
template <typename S>
__device__ __forceinline__ S rot(const TxDesc& t, int ij);
template <>
__device__ __forceinline__ float rot<float>(const TxDesc& t, int ij) { return t.R[ij]; }
template <>
__device__ __forceinline__ d3f rot<d3f>(const TxDesc& t, int ij) {
    return d3f{t.R[ij], t.dR[0][ij], t.dR[1][ij], t.dR[2][ij]};
}

// ------------------------------------------------------------ ray launch
struct Launch {
    double kx, ky, kz;      // direction
    double tx, ty, tz;      // theta_hat (launch polarisation basis, e_s)
    double px, py;          // phi_hat = (px, py, 0)
};

// sin and cos of 2 pi u, u = m 2^-53 turns (m < 2^53), in FP64: 4u quarter
// turns are split in integers at the nearest quarter turn q (exact), the
// remainder y = (pi/2)(4u - q) has |y| <= pi/4, sin y and cos y come from
// their Taylor series to y^13 and y^14 (truncation below 3e-14 relative), and
// q mod 4 rotates the pair.
__device__ __forceinline__ void sincos_turns53(uint64_t m, double& s, double& c) {
    const uint64_t q = (m + (1ull << 50)) >> 51;
    const double y = (double)((int64_t)m - (int64_t)(q << 51)) * (0.5 * RT_PI * 0x1.0p-51);
    const double y2 = y * y;
    double ps = 1.0 / 6227020800.0;
    ps = fma(ps, y2, -1.0 / 39916800.0);
    ps = fma(ps, y2, 1.0 / 362880.0);
    ps = fma(ps, y2, -1.0 / 5040.0);
    ps = fma(ps, y2, 1.0 / 120.0);
    ps = fma(ps, y2, -1.0 / 6.0);
    const double sy = fma(y * y2, ps, y);
    double pc = -1.0 / 87178291200.0;
    pc = fma(pc, y2, 1.0 / 479001600.0);
    pc = fma(pc, y2, -1.0 / 3628800.0);
    pc = fma(pc, y2, 1.0 / 40320.0);
    pc = fma(pc, y2, -1.0 / 720.0);
    pc = fma(pc, y2, 1.0 / 24.0);
    pc = fma(pc, y2, -0.5);
    const double cy = fma(y2, pc, 1.0);
    const int quad = (int)(q & 3);
    s = quad == 0 ? sy : quad == 1 ? cy : quad == 2 ? -sy : -cy;
    c = quad == 0 ? cy : quad == 1 ? -sy : quad == 2 ? -cy : sy;
}

// Lattice point n of an N-point spherical Fibonacci lattice, in FP64.
__device__ __forceinline__ Launch fib_launch(int64_t n, int64_t N) {
    double z;
    uint64_t m;                                               // azimuth in turns, times 2^53
    if (N == 1) {
        z = 0.0;
        m = 1ull << 52;                                       // half a turn
    } else {
        z = 1.0 - (double)n * (2.0 / (double)(N - 1));         // the quotient is hoisted per lattice
        m = ((uint64_t)n * kPhiFrac) >> 11;                   // product wraps mod 2^64
    }
    double st = sqrt(fmax(0.0, (1.0 - z) * (1.0 + z)));
    double sp, cp;
    sincos_turns53(m, sp, cp);
    Launch L;
    L.kx = st * cp;
    L.ky = st * sp;
    L.kz = z;
    L.tx = z * cp;
    L.ty = z * sp;
    L.tz = -st;
    L.px = -sp;
    L.py = cp;
    return L;
}

// sin and cos of the angle (pi/2) v for v in quarter turns: v is split at
// the nearest integer q (exact in FP64), the remainder y = (pi/2)(v - q),
// |y| <= pi/4, is taken to FP32, sin y and cos y come from their Taylor
// series to y^9 and y^10 (truncation below 2e-9 on |y| <= pi/4), and the
// quadrant q mod 4 rotates the pair.
__device__ __forceinline__ void sincos_quarter_turns(double v, float& s, float& c) {
    const double q = rint(v);
    const float y = (float)((v - q) * (0.5 * RT_PI));
    const float y2 = y * y;
    const float sy =
        y * (1.0f + y2 * (-1.0f / 6.0f + y2 * (1.0f / 120.0f + y2 * (-1.0f / 5040.0f + y2 * (1.0f / 362880.0f)))));
    const float cy = 1.0f + y2 * (-0.5f + y2 * (1.0f / 24.0f + y2 * (-1.0f / 720.0f +
                                                                     y2 * (1.0f / 40320.0f - y2 / 3628800.0f))));
    const int quad = (int)((long long)q & 3);
    s = quad == 0 ? sy : quad == 1 ? cy : quad == 2 ? -sy : -cy;
    c = quad == 0 ? cy : quad == 1 ? -sy : quad == 2 ? -cy : sy;
}

// |alpha|^2 of a synthetic transmit array for launch direction k
// (Sec. "Handling Multiple Transmit Antennas"): alpha = a_tx^T u_P with the
// array response a_tx[i] = exp(j 2 pi/lambda k.d_i) of
// eq. path-solver-array-response-vector.  The phase is formed in FP64 in
// quarter turns; the element data are the same for every lane.
__device__ __forceinline__ float array_gain(const Launch& L, const TxDesc& t) {
    float are = 0.0f, aim = 0.0f;
    for (int i = 0; i < t.n_ant; i++) {
        const double* d = t.ant_pos + 3 * (int64_t)i;
        const double v = (L.kx * d[0] + L.ky * d[1] + L.kz * d[2]) * t.four_inv_lambda;
        float s, c;
        sincos_quarter_turns(v, s, c);
        const float ur = t.precoding[2 * (int64_t)i], ui = t.precoding[2 * (int64_t)i + 1];
        are += ur * c - ui * s;
        aim += ur * s + ui * c;
    }
    return are * are + aim * aim;
}

// Transmit pattern components (C_theta, C_phi) on the launch basis
// (theta_hat, phi_hat) of direction k, for one polarisation (pol_index 0:
// C' = sqrt(G) theta_hat', 1: C' = sqrt(G) phi_hat').  The local direction is
// u = R^T k (eq. theta_phi_prime); theta_hat' and phi_hat' of eq. spherical_vecs
// are written in Cartesian components of u (cos theta' = u_z,
// sin theta' = rho = |u_xy|, (cos, sin) phi' = u_xy / rho, and phi' = 0 on the
// local poles, which is atan2(0, 0)); the local field is rotated back by R
// and projected on the launch basis, which is eq. F_prime_2_F.  With S = d3f
// the same code yields d/d(yaw, pitch, roll).
template <typename S>
__device__ __forceinline__ void tx_pattern(const Launch& L, const TxDesc& t, int pol_index, S& c_theta, S& c_phi) {
    const float kx = (float)L.kx, ky = (float)L.ky, kz = (float)L.kz;
    S R00 = rot<S>(t, 0), R01 = rot<S>(t, 1), R02 = rot<S>(t, 2);
    S R10 = rot<S>(t, 3), R11 = rot<S>(t, 4), R12 = rot<S>(t, 5);
    S R20 = rot<S>(t, 6), R21 = rot<S>(t, 7), R22 = rot<S>(t, 8);
    S ux = R00 * cst<S>(kx) + R10 * cst<S>(ky) + R20 * cst<S>(kz);
    S uy = R01 * cst<S>(kx) + R11 * cst<S>(ky) + R21 * cst<S>(kz);
    S uz = R02 * cst<S>(kx) + R12 * cst<S>(ky) + R22 * cst<S>(kz);
    S rho = dsqrtf(ux * ux + uy * uy);
    S cp, sp;
    if (val(rho) > 1e-12f) {
        S ir = drecip(rho);
        cp = ux * ir;
        sp = uy * ir;
    } else {
        cp = cst<S>(1.0f);
        sp = cst<S>(0.0f);
    }
    S amp = cst<S>(1.0f);
    if (t.pattern == 1) {
        // (1 + cos alpha)/2 with cos alpha = u_x = (R x_hat) . k, evaluated in
        // FP64: near the back lobe 1 + u_x cancels and FP32 would lose it
        double hx = 0.5 * (1.0 + (t.ax[0] * L.kx + t.ax[1] * L.ky + t.ax[2] * L.kz));
        S half = ux * cst<S>(0.5f);          // carries d(u_x)/d angle / 2
        half = with_value(half, (float)fmax(hx, 0.0));
        amp = dsqrtf(cst<S>(t.q + 1.0f) * dpowf(half, t.q));
    }
    S fx, fy, fz;
    if (pol_index == 0) {
        fx = amp * uz * cp;
        fy = amp * uz * sp;
        fz = -(amp * rho);
    } else {
        fx = -(amp * sp);
        fy = amp * cp;
        fz = cst<S>(0.0f);
    }
    S gx = R00 * fx + R01 * fy + R02 * fz;
    S gy = R10 * fx + R11 * fy + R12 * fz;
    S gz = R20 * fx + R21 * fy + R22 * fz;
    c_theta = cst<S>((float)L.tx) * gx + cst<S>((float)L.ty) * gy + cst<S>((float)L.tz) * gz;
    c_phi = cst<S>((float)L.px) * gx + cst<S>((float)L.py) * gy;
}

// ------------------------------------------------------------ geometry
// Relative slack of the slab test, above the rounding of the slab distances
// and of the triangle distance, so that a box is never culled while a
// triangle inside it can still win.
constexpr float kBoxSlack = 1.0f + 1e-5f;

struct Ray {
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;          // guarded reciprocal direction (slab test)
    float sx, sy, sz;          // watertight shear constants
    int kx, ky, kz;            // watertight axis permutation
    unsigned nx, ny, nz;       // byte offsets of the near planes in a 4-wide node
    float jx, jy, jz;          // reciprocal direction times kBoxSlack (far planes of box4)
    float cnx, cny, cnz;       // -o i lowered past its rounding (near planes of box4)
};

__device__ __forceinline__ float pick(float a, float b, float c, int i) { return i == 0 ? a : (i == 1 ? b : c); }

// Hardware reciprocal (about 1 ulp): the slab test has a relative slack far
// above that, and the shear constants below only need to be the same for
// every triangle a ray is tested against, which keeps the test watertight.
__device__ __forceinline__ float safe_inv(float d) {
    float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return __builtin_amdgcn_rcpf(a);
}

__device__ __forceinline__ void ray_setup(Ray& r) {
    float ax = fabsf(r.dx), ay = fabsf(r.dy), az = fabsf(r.dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dkz = pick(r.dx, r.dy, r.dz, kz);
    if (dkz < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.sz = __builtin_amdgcn_rcpf(dkz);
    r.sx = pick(r.dx, r.dy, r.dz, kx) * r.sz;
    r.sy = pick(r.dx, r.dy, r.dz, ky) * r.sz;
    r.ix = safe_inv(r.dx);
    r.iy = safe_inv(r.dy);
    r.iz = safe_inv(r.dz);
    r.jx = r.ix * kBoxSlack;
    r.jy = r.iy * kBoxSlack;
    r.jz = r.iz * kBoxSlack;
    // near planes are evaluated as p i + cn, one fma: cn is the rounded -o i
    // lowered by 2^-22 |o i|, which exceeds the rounding of -o i and of the
    // lowering itself (each at most 2^-24 |o i|), so p i + cn lies below
    // (p - o) i and the fma's own rounding is relative, like the product's
    // before, and covered by kBoxSlack: an entry distance can only come out
    // smaller, never culling a box.  Far planes keep the difference and
    // product, so boxes behind the origin (exit below tmin) stay culled as
    // sharply as before.
    {
        const float cx = -r.ox * r.ix, cy = -r.oy * r.iy, cz = -r.oz * r.iz;
        r.cnx = __builtin_fmaf(fabsf(cx), -0x1p-22f, cx);
        r.cny = __builtin_fmaf(fabsf(cy), -0x1p-22f, cy);
        r.cnz = __builtin_fmaf(fabsf(cz), -0x1p-22f, cz);
    }
    r.nx = r.ix < 0.0f ? 16u : 0u;
    r.ny = r.iy < 0.0f ? 48u : 32u;
    r.nz = r.iz < 0.0f ? 80u : 64u;
}

// Watertight ray/triangle test.  Returns t (> t_min) or a negative value.
// Edge cases where a scaled barycentric is exactly zero are recomputed in
// FP64, which is what makes shared edges watertight.
__device__ __forceinline__ float tri_hit(const Ray& r, float4 a, float4 b, float4 c, float t_min) {
#pragma clang fp contract(off)
    float Ax0 = a.x - r.ox, Ay0 = a.y - r.oy, Az0 = a.z - r.oz;
    float Bx0 = b.x - r.ox, By0 = b.y - r.oy, Bz0 = b.z - r.oz;
    float Cx0 = c.x - r.ox, Cy0 = c.y - r.oy, Cz0 = c.z - r.oz;
    float Ak = pick(Ax0, Ay0, Az0, r.kz), Bk = pick(Bx0, By0, Bz0, r.kz), Ck = pick(Cx0, Cy0, Cz0, r.kz);
    float Ax = pick(Ax0, Ay0, Az0, r.kx) - r.sx * Ak;
    float Ay = pick(Ax0, Ay0, Az0, r.ky) - r.sy * Ak;
    float Bx = pick(Bx0, By0, Bz0, r.kx) - r.sx * Bk;
    float By = pick(Bx0, By0, Bz0, r.ky) - r.sy * Bk;
    float Cx = pick(Cx0, Cy0, Cz0, r.kx) - r.sx * Ck;
    float Cy = pick(Cx0, Cy0, Cz0, r.ky) - r.sy * Ck;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return -1.0f;
    float det = U + V + W;
    if (det == 0.0f) return -1.0f;
    float Az = r.sz * Ak, Bz = r.sz * Bk, Cz = r.sz * Ck;
    float T = U * Az + V * Bz + W * Cz;
    float t = T / det;
    return t > t_min ? t : -1.0f;
}


// Slab test of the two children of a node.  lo/hi layout as in rt_internal.h.
__device__ __forceinline__ void box2(const Ray& r, float4 q0, float4 q1, float4 q2, float tmin, float tmax,
                                     bool& hitL, bool& hitR, float& tL, float& tR) {
    float lx0 = (q0.x - r.ox) * r.ix, lx1 = (q0.y - r.ox) * r.ix;
    float ly0 = (q0.z - r.oy) * r.iy, ly1 = (q0.w - r.oy) * r.iy;
    float lz0 = (q2.x - r.oz) * r.iz, lz1 = (q2.y - r.oz) * r.iz;
    float rx0 = (q1.x - r.ox) * r.ix, rx1 = (q1.y - r.ox) * r.ix;
    float ry0 = (q1.z - r.oy) * r.iy, ry1 = (q1.w - r.oy) * r.iy;
    float rz0 = (q2.z - r.oz) * r.iz, rz1 = (q2.w - r.oz) * r.iz;
    float aL = fmaxf(fmaxf(fminf(lx0, lx1), fminf(ly0, ly1)), fmaxf(fminf(lz0, lz1), tmin));
    float bL = fminf(fminf(fmaxf(lx0, lx1), fmaxf(ly0, ly1)), fmaxf(lz0, lz1)) * kBoxSlack;
    float aR = fmaxf(fmaxf(fminf(rx0, rx1), fminf(ry0, ry1)), fmaxf(fminf(rz0, rz1), tmin));
    float bR = fminf(fminf(fmaxf(rx0, rx1), fmaxf(ry0, ry1)), fmaxf(rz0, rz1)) * kBoxSlack;
    hitL = aL <= fminf(bL, tmax);
    hitR = aR <= fminf(bR, tmax);
    tL = aL;
    tR = aR;
}

// Buffer resource over the 4-wide node array: loads are range-checked by
// the hardware against the array's byte size (an offset outside reads
// zeros), so a bad node reference can never read outside the array.  The
// size is a 32-bit unsigned count: the build keeps n_wide below 2^25, so
// 128 n_wide stays below 2^32, and so do the node offsets node << 7.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wide_rsrc(const float4* wide, int n_wide) {
    const unsigned bytes = (unsigned)n_wide * 128u;
    return __builtin_amdgcn_make_buffer_rsrc((void*)wide, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float4 ld16(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}

// Slab test of the four children of the wide node at byte offset `base`.
// Per axis the ray reads its near planes (lo for a positive direction
// component, else hi) and its far planes, so that no min/max per axis is
// needed: entry = max(near distances, tmin), exit = min(far distances) times
// the slack.  Near distances take one fma each against the lowered offsets
// of ray_setup; far distances a difference and a product.  Also returns the
// four child references.
__device__ __forceinline__ void box4(const Ray& r, __amdgpu_buffer_rsrc_t rs, unsigned base, float tmin, float tmax,
                                     bool hit[4], float tent[4], int ref[4]) {
    const unsigned bx = base | r.nx, by = base | r.ny, bz = base | r.nz;
    const float4 nx = ld16(rs, bx), fx = ld16(rs, bx ^ 16u);
    const float4 ny = ld16(rs, by), fy = ld16(rs, by ^ 16u);
    const float4 nz = ld16(rs, bz), fz = ld16(rs, bz ^ 16u);
    const float4 rf = ld16(rs, base | 96u);
    const float nxa[4] = {nx.x, nx.y, nx.z, nx.w}, fxa[4] = {fx.x, fx.y, fx.z, fx.w};
    const float nya[4] = {ny.x, ny.y, ny.z, ny.w}, fya[4] = {fy.x, fy.y, fy.z, fy.w};
    const float nza[4] = {nz.x, nz.y, nz.z, nz.w}, fza[4] = {fz.x, fz.y, fz.z, fz.w};
#pragma unroll
    for (int c = 0; c < 4; c++) {
        float a = fmaxf(fmaxf(__builtin_fmaf(nxa[c], r.ix, r.cnx), __builtin_fmaf(nya[c], r.iy, r.cny)),
                        fmaxf(__builtin_fmaf(nza[c], r.iz, r.cnz), tmin));
        float b = fminf(fminf((fxa[c] - r.ox) * r.jx, (fya[c] - r.oy) * r.jy), (fza[c] - r.oz) * r.jz);
        hit[c] = a <= fminf(b, tmax);
        tent[c] = a;
    }
    ref[0] = __float_as_int(rf.x);
    ref[1] = __float_as_int(rf.y);
    ref[2] = __float_as_int(rf.z);
    ref[3] = __float_as_int(rf.w);
}

// ------------------------------------------------------------ Fresnel
struct Fresnel {
    cf rperp, rpar;       // eq. fresnel_vac
    cf drperp, drpar;     // d/d eta
    cf s;                 // sqrt(eta - sin^2 theta_1), principal branch
};

// c = cos(theta_1) >= 0, eta = eps_r - j sigma/(eps0 omega)  (eq. eta)
template <bool DERIV>
__device__ __forceinline__ Fresnel fresnel(float c, cf eta) {
    Fresnel F;
    cf s = csqrt_principal(cf{eta.re - (1.0f - c * c), eta.im});
    cf cp = cf{c + s.re, s.im};
    cf cm = cf{c - s.re, -s.im};
    cf ec = cscale(eta, c);
    cf lp = cadd(ec, s), lm = csub(ec, s);
    F.rperp = cdiv(cm, cp);
    F.rpar = cdiv(lm, lp);
    F.s = s;
    if (DERIV) {
        // r_perp = (c - s)/(c + s), s = sqrt(eta - sin^2): d r_perp/d eta = -c / (s (c + s)^2)
        // r_par = (eta c - s)/(eta c + s): d r_par/d eta = c (eta - 2 sin^2) / (s (eta c + s)^2)
        cf scp2 = cmul(s, cmul(cp, cp));
        F.drperp = cdiv(cf{-c, 0.0f}, scp2);
        cf num = cscale(cf{eta.re - 2.0f * (1.0f - c * c), eta.im}, c);
        F.drpar = cdiv(num, cmul(s, cmul(lp, lp)));
    } else {
        F.drperp = cf{0, 0};
        F.drpar = cf{0, 0};
    }
    return F;
}

// Single-layer slab (eq. fresnel_slab, eq. q_fresnel_slab) of phase constant
// k_d = 2 pi d / lambda: with x = exp(-j k_d s), each half-space r' held in F
// becomes r' (1 - x^2) / (1 - r'^2 x^2) in place, and the slab passes
// t = (1 - r'^2) x / (1 - r'^2 x^2).  Im s <= 0, so |x| <= 1.
__device__ __forceinline__ void slab(Fresnel& F, float k_d, cf& tperp, cf& tpar) {
    const float qre = k_d * F.s.re, qim = k_d * F.s.im;
    float sn, cs;
    sincosf(qre, &sn, &cs);
    const float m = __expf(qim);
    const cf x = cf{m * cs, -m * sn};
    const cf x2 = cmul(x, x);
    const cf one = cf{1.0f, 0.0f};
    const cf rp2 = cmul(F.rperp, F.rperp), rl2 = cmul(F.rpar, F.rpar);
    const cf dp = csub(one, cmul(rp2, x2)), dl = csub(one, cmul(rl2, x2));
    const cf omx2 = csub(one, x2);
    tperp = cdiv(cmul(csub(one, rp2), x), dp);
    tpar = cdiv(cmul(csub(one, rl2), x), dl);
    F.rperp = cdiv(cmul(F.rperp, omx2), dp);
    F.rpar = cdiv(cmul(F.rpar, omx2), dl);
}

// Slab coefficients of one polarisation with their eta-derivatives, from the
// half-space r1 and dr1 = dr1/d eta: with D = 1 - r1^2 x^2 and
// dx/d eta = -j k_d x / (2 s), r = r1 (1 - x^2) / D, t = (1 - r1^2) x / D
// and their derivatives by the quotient rule.
__device__ __forceinline__ void slab_pol_grad(cf r1, cf dr1, cf x, cf dx, cf& r, cf& dr, cf& t, cf& dt) {
    const cf one = cf{1.0f, 0.0f};
    const cf x2 = cmul(x, x), r12 = cmul(r1, r1);
    const cf D = csub(one, cmul(r12, x2));
    const cf two_r1 = cscale(r1, 2.0f);
    const cf dD = cscale(cadd(cmul(cmul(two_r1, dr1), x2), cmul(cmul(cscale(r12, 2.0f), x), dx)), -1.0f);
    const cf omx2 = csub(one, x2), om12 = csub(one, r12);
    r = cdiv(cmul(r1, omx2), D);
    t = cdiv(cmul(om12, x), D);
    dr = cdiv(csub(csub(cmul(dr1, omx2), cmul(cmul(two_r1, x), dx)), cmul(r, dD)), D);
    dt = cdiv(csub(cadd(cscale(cmul(cmul(two_r1, dr1), x), -1.0f), cmul(om12, dx)), cmul(t, dD)), D);
}

// slab() with derivatives: F (from fresnel<true>) becomes the slab r and
// dr/d eta; t and dt/d eta are returned.
__device__ __forceinline__ void slab_grad(Fresnel& F, float k_d, cf& tperp, cf& tpar, cf& dtperp, cf& dtpar) {
    const float qre = k_d * F.s.re, qim = k_d * F.s.im;
    float sn, cs;
    sincosf(qre, &sn, &cs);
    const float m = __expf(qim);
    const cf x = cf{m * cs, -m * sn};
    const cf dx = cdiv(cmul(cf{0.0f, -k_d}, x), cscale(F.s, 2.0f));
    cf r, dr;
    slab_pol_grad(F.rperp, F.drperp, x, dx, r, dr, tperp, dtperp);
    F.rperp = r;
    F.drperp = dr;
    slab_pol_grad(F.rpar, F.drpar, x, dx, r, dr, tpar, dtpar);
    F.rpar = r;
    F.drpar = dr;
}

// Normalisation F_alpha(theta_i) of a scattering lobe (eq. directive_model):
// 2^-alpha sum_k C(alpha, k) I_k with I_k = 2 pi/(k+1) for even k and
// 2 pi/(k+1) cos(theta_i) sum_{w <= (k-1)/2} C(2w, w) (sin^2(theta_i)/4)^w
// for odd k; the inner terms follow from C(2w, w)/4^w = (2w-1)/(2w) times
// the previous one.
__device__ __forceinline__ float lobe_norm(int alpha, float ci) {
    const float s2 = fmaxf(0.0f, 1.0f - ci * ci);
    float F = 0.0f, binom = 1.0f;
    for (int k = 0; k <= alpha; k++) {
        if (k > 0) binom = binom * (float)(alpha - k + 1) / (float)k;
        float Ik = 2.0f * (float)RT_PI / (float)(k + 1);
        if (k & 1) {
            float sum = 0.0f, term = 1.0f;
            for (int w = 0; w <= (k - 1) / 2; w++) {
                if (w > 0) term *= (float)(2 * w - 1) / (float)(2 * w) * s2;
                sum += term;
            }
            Ik *= ci * sum;
        }
        F += binom * Ik;
    }
    return ldexpf(F, -alpha);
}

// 2 pi f_s of a diffuse bounce: pp = (kind, alpha_R, alpha_I, Lambda) or
// null (Lambertian, eq. lambertian_model: 2 cos(theta_s)); kind 1 directive
// (eq. directive_model), 2 backscattering (eq. backscattering_model).  ci =
// cos(theta_i), cs = cos(theta_s), ki / ks / kr the incident, scattered and
// specular directions.
__device__ __forceinline__ float scatter_weight(const float* pp, float ci, float cs, float3 ki, float3 ks, float3 kr) {
    const int kind = pp ? (int)pp[0] : 0;
    if (kind == 0) return 2.0f * cs;
    const int aR = (int)pp[1];
    const float lam = kind == 1 ? 1.0f : pp[3];
    float num = lam * powf(0.5f * (1.0f + dot3(kr, ks)), (float)aR);
    float F = lam * lobe_norm(aR, ci);
    if (kind == 2) {
        const int aI = (int)pp[2];
        num += (1.0f - lam) * powf(0.5f * (1.0f - dot3(ki, ks)), (float)aI);
        F += (1.0f - lam) * lobe_norm(aI, ci);
    }
    return 2.0f * (float)RT_PI * num / F;
}

// theta_hat and phi_hat of direction k (eq. spherical_vecs); phi = 0 on the
// z axis.
__device__ __forceinline__ void sph_basis(float3 k, float3& th, float3& ph) {
    const float rho = sqrtf(k.x * k.x + k.y * k.y);
    float cp = 1.0f, sp = 0.0f;
    if (rho > 0.0f) {
        cp = k.x / rho;
        sp = k.y / rho;
    }
    th = f3(k.z * cp, k.z * sp, -rho);
    ph = f3(-sp, cp, 0.0f);
}

// Direction of polar cosine cs (sine ss) and azimuth (cph, sph) about the
// unit normal n, in the frame t1 = (a x n)/|a x n|, t2 = n x t1 with a the
// coordinate axis least aligned with n.
__device__ __forceinline__ float3 diffuse_direction(float3 n, float cs, float ss, float cph, float sph) {
    const float ax = fabsf(n.x), ay = fabsf(n.y), az = fabsf(n.z);
    const float3 a = (ax <= ay && ax <= az) ? f3(1, 0, 0) : (ay <= az ? f3(0, 1, 0) : f3(0, 0, 1));
    const float3 t1 = unit3(cross3(a, n));
    const float3 t2 = cross3(n, t1);
    return unit3(t1 * (ss * cph) + t2 * (ss * sph) + n * cs);
}

// Orthonormal TE direction e_perp = (k x n)/|k x n|; at normal incidence any
// direction transverse to k: k x a with a the axis least aligned with k.
__device__ __forceinline__ float3 te_direction(float3 k, float3 n) {
    float3 e = cross3(k, n);
    float l2 = dot3(e, e);
    if (l2 < 1e-14f) {
        float ax = fabsf(k.x), ay = fabsf(k.y), az = fabsf(k.z);
        float3 a = (ax <= ay && ax <= az) ? f3(1, 0, 0) : (ay <= az ? f3(0, 1, 0) : f3(0, 0, 1));
        e = cross3(k, a);
        l2 = dot3(e, e);
    }
    return e * __builtin_amdgcn_rsqf(l2);
}

// Reflection geometry at a hit.  The field of a segment is stored as complex
// components on (e_s, e_p = k x e_s).  After reflection the basis is
// (e_perp, k_r x e_perp); since the reflected TM direction of
// eq. fresnel_out_vectors is e_perp x k_r = -(k_r x e_perp), the TM
// coefficient enters with a minus sign: T <- diag(r_perp, -r_par) W T.
struct Bounce {
    float w00, w01, w10, w11;   // W(e_perp, e_par_i ; e_s, e_p)
    float c;                    // cos(theta_1)
    float3 kr;                  // reflected direction
    float3 es_new;              // e_perp
};

__device__ __forceinline__ Bounce bounce_geometry(float3 k, float3 es, float3 nrm) {
    Bounce b;
    float kn = dot3(k, nrm);
    if (kn > 0.0f) {          // orient the normal toward the incident side
        nrm = nrm * -1.0f;
        kn = -kn;
    }
    b.c = fminf(1.0f, -kn);
    float3 ep = cross3(k, es);
    float3 eperp = te_direction(k, nrm);
    float3 epar = cross3(eperp, k);
    b.w00 = dot3(eperp, es);
    b.w01 = dot3(eperp, ep);
    b.w10 = dot3(epar, es);
    b.w11 = dot3(epar, ep);
    float3 kr = k - nrm * (2.0f * kn);
    b.kr = unit3(kr);
    b.es_new = eperp;
    return b;
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), written from its
// definition: ten rounds, each multiplying words 0 and 2 by two odd constants,
// keeping the low halves and XORing the high halves with words 1, 3 and the
// round key, which advances by two Weyl constants.  Counter (n_lo, n_hi, l,
// stream), key (seed, 0); stream 0 decides early termination before segment
// l, stream 1 the interaction type at the end of segment l, stream 2 the
// direction and phases of a diffuse reflection there.
__device__ __forceinline__ uint4 philox4(unsigned seed, int64_t n, int l, unsigned stream) {
    unsigned c0 = (unsigned)((uint64_t)n & 0xffffffffu), c1 = (unsigned)((uint64_t)n >> 32), c2 = (unsigned)l,
             c3 = stream;
    unsigned k0 = seed, k1 = 0u;
#pragma unroll
    for (int round = 0; round < 10; round++) {
        const unsigned lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const unsigned lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform in [0, 1) from the top 24 bits of a word (exact in FP32).
__device__ __forceinline__ float word_uniform(unsigned w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

__device__ __forceinline__ float philox_uniform(unsigned seed, int64_t n, int l, unsigned stream) {
    return word_uniform(philox4(seed, n, l, stream).x);
}

}  // namespace rtd
