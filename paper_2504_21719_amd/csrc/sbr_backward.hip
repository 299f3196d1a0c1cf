// sbr_backward.hip -- adjoint (vector-Jacobian product) of the SBR radio map.
//
// The forward pass with a tape recorded, per traced segment l of every ray,
// its direction k_l, basis vector e_s,l, the slot of the triangle that ends
// it, the plane cell it crossed, and the field transfer matrix T_l (the
// per-bounce checkpoint).  For one ray and polarisation with launch pattern C
// the loss contribution is
//     J = sum_l a_l ||E_l||^2,   E_l = T_l C,   a_l = G[cell_l] kappa / |k_l,z|
// (G = dLoss/dMap; a_l = 0 when segment l crosses no cell), and
//     E_l = R_l E_{l-1},   R_l = diag(r_perp, -r_par) W_l
// with W_l the basis change at the hit that ends segment l-1 and r the
// vacuum Fresnel coefficients (eq. fresnel_vac) of the hit material's
// eta = eps_r - j sigma/(eps0 omega) (eq. eta).
//
// Reverse sweep (Wirtinger calculus for the real J): with
//     lambda_l = a_l E_l + R_{l+1}^H lambda_{l+1}
// the derivative with respect to a real parameter p of R_l is
//     dJ/dp = 2 Re( lambda_l^H (dR_l/dp) E_{l-1} ),
// where dR/d eta = diag(dr_perp/d eta, -dr_par/d eta) W, d eta/d eps_r = 1,
// d eta/d sigma = -j/(eps0 omega), and for the launch pattern
//     dJ/dp = 2 Re( lambda_0^H dC/dp ),  p in {yaw, pitch, roll},
// with dC/dp from FP32 forward-mode dual numbers through eq. theta_phi_prime,
// fed with R and its angle derivatives (eq. rotation) computed on the host.  Nothing is re-traced: geometry and fields come from
// the tape; only the normal (from the hit slot) and the Fresnel terms are
// recomputed.
//
// Reduction: every thread owns a fixed set of rays (grid-stride order) and
// registers for up to kMatChunk materials; sums go thread -> wave (butterfly)
// -> block (waves in order) -> per-block partials in FP64 -> one final kernel
// that adds the blocks in a fixed order.  The result does not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sbr_common.h"

using namespace rtd;

namespace {

constexpr int kMatChunk = 8;
constexpr int kBwdBlock = 256;
// One round of resident waves: both variants hold 2 waves per SIMD (their
// VGPR counts), so 256 CUs x 4 SIMDs x 2 waves = 512 workgroups of 4 waves.
// A second, partly filled round cost 1.7x in the adjoint's time.
constexpr int kBwdBlocks = 512;

struct BwdArgs {
    const float4* seg;
    const int* nseg;
    int64_t n;            // rays on the tape
    int64_t ray_begin;
    const float4* normals;
    const float* eps_r;
    const float* sigma;
    TxDesc tx;
    PlaneDesc pl;
    int npol;
    const float* grad_map;
    int64_t map_stride;
    int n_mat;
    int mat0;             // first material of this chunk
    int P;                // parameters written by this launch into partials
    double* partials;     // [gridDim.x][P]
    int write_orient;     // 1: this chunk also produces the orientation terms
    const float* thickness;  // slab thickness per material (m), or null
    int refraction;          // 1: the forward sampled reflection or transmission
    float k0;                // 2 pi / lambda
    int rr_depth;            // Russian roulette before segments l >= rr_depth
    float rr_p_max;          // (0 = off)
    const float* scattering; // diffuse reflection: S and K_x per material, or null
    const float* xpd;
    unsigned seed;           // key of the forward's random streams
};

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// EXT: the forward used slab walls, refraction, diffuse reflection or early
// termination; the plain variant carries none of their code (and registers).
template <bool EXT>
__global__ void __launch_bounds__(kBwdBlock) k_backward(const BwdArgs a) {
    float ge[kMatChunk], gs[kMatChunk];
#pragma unroll
    for (int j = 0; j < kMatChunk; j++) {
        ge[j] = 0.0f;
        gs[j] = 0.0f;
    }
    float go0 = 0.f, go1 = 0.f, go2 = 0.f;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t n = a.n;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += T) {
        const int ns = a.nseg[r];
        const int64_t ray = a.ray_begin + r;
        Launch Lr = fib_launch(ray, a.tx.n_rays);
        // transmit array: |alpha|^2 of the departure direction scales every
        // crossing of the ray and depends on none of the parameters
        const float kap = a.tx.n_ant > 0 ? a.tx.kappa * array_gain(Lr, a.tx) : a.tx.kappa;
        for (int p = 0; p < a.npol; p++) {
            int pol_index = (a.npol == 2) ? p : (a.tx.pol == 1 ? 1 : 0);
            d3f cth, cph;
            tx_pattern<d3f>(Lr, a.tx, pol_index, cth, cph);
            const float ct = cth.v, cp = cph.v;
            const float* G = a.grad_map + (int64_t)p * a.map_stride;
            cf lam0 = {0, 0}, lam1 = {0, 0};
            // records of segment l (s*) and of segment l-1 (p*); each is read
            // once, the step to l-1 carries p* over into s*
            float4 s0, s1, s2, s3, p0 = {}, p1 = {}, p2 = {}, p3 = {};
            for (int l = ns - 1; l >= 0; l--) {
                if (l == ns - 1) {
                    const float4* s = a.seg + (int64_t)l * 4 * n + r;
                    s0 = s[0];
                    s1 = s[n];
                    s2 = s[2 * n];
                    s3 = s[3 * n];
                } else {
                    s0 = p0;
                    s1 = p1;
                    s2 = p2;
                    s3 = p3;
                }
                int cell = __float_as_int(s1.w);
                if (cell >= 0) {
                    float g = G[cell];
                    if (g != 0.0f) {
                        float al = g * kap * __builtin_amdgcn_rcpf(fabsf(s0.z));
                        // E_l = T_l C
                        cf e0 = cadd(cscale(cf{s2.x, s2.y}, ct), cscale(cf{s2.z, s2.w}, cp));
                        cf e1 = cadd(cscale(cf{s3.x, s3.y}, ct), cscale(cf{s3.z, s3.w}, cp));
                        lam0 = cadd(lam0, cscale(e0, al));
                        lam1 = cadd(lam1, cscale(e1, al));
                    }
                }
                if (l == 0) break;
                // bounce at the end of segment l-1
                const float4* q = a.seg + (int64_t)(l - 1) * 4 * n + r;
                p0 = q[0];
                p1 = q[n];
                p2 = q[2 * n];
                p3 = q[3 * n];
                int slot = __float_as_int(p0.w);
                float4 nm = a.normals[slot];
                int mat = __float_as_int(nm.w);
                Bounce b = bounce_geometry(f3(p0.x, p0.y, p0.z), f3(p1.x, p1.y, p1.z), f3(nm.x, nm.y, nm.z));
                cf eta = cf{a.eps_r[mat], -a.sigma[mat] * a.pl.inv_eps0_omega};
                Fresnel F = fresnel<true>(b.c, eta);
                // coefficient of the interaction and its eta-derivative: the
                // slab r (or t for a transmitted ray, whose direction did not
                // change) divided by sqrt(q), the sampling probability held
                // constant
                cf kpe = F.rperp, kpa = F.rpar, dkpe = F.drperp, dkpa = F.drpar;
                const bool transmit = EXT && a.refraction && s0.x == p0.x && s0.y == p0.y && s0.z == p0.z;
                if (EXT && a.thickness) {
                    cf tp, tl, dtp, dtl;
                    slab_grad(F, a.k0 * a.thickness[mat], tp, tl, dtp, dtl);
                    kpe = F.rperp;
                    kpa = F.rpar;
                    dkpe = F.drperp;
                    dkpa = F.drpar;
                    if (a.refraction) {
                        const float ar = cabs2(F.rperp) + cabs2(F.rpar), at = cabs2(tp) + cabs2(tl);
                        const float tot = ar + at;
                        const float q = transmit ? (tot > 0.0f ? at / tot : 0.0f) : (tot > 0.0f ? ar / tot : 1.0f);
                        const float sc = __builtin_amdgcn_rsqf(q);
                        kpe = cscale(transmit ? tp : F.rperp, sc);
                        kpa = cscale(transmit ? tl : F.rpar, sc);
                        dkpe = cscale(transmit ? dtp : F.drperp, sc);
                        dkpa = cscale(transmit ? dtl : F.drpar, sc);
                    }
                }
                // a diffuse reflection: the taped direction of segment l is
                // the one drawn from stream 2 at this interaction (a specular
                // direction meets it with probability ~1e-9)
                bool diffuse = false;
                float dc1 = 0.f, ds1 = 0.f, dc2 = 0.f, ds2 = 0.f;
                if (EXT && a.scattering && !transmit && a.scattering[mat] > 0.0f) {
                    const uint4 w = philox4(a.seed, ray, l - 1, 2u);
                    const float cs = word_uniform(w.x), ss = sqrtf(fmaxf(0.0f, 1.0f - cs * cs));
                    float sph, cph;
                    sincospif(2.0f * word_uniform(w.y), &sph, &cph);
                    float3 nd = f3(nm.x, nm.y, nm.z);
                    if (dot3(f3(p0.x, p0.y, p0.z), nd) > 0.0f) nd = nd * -1.0f;
                    const float3 kd = diffuse_direction(nd, cs, ss, cph, sph) - f3(s0.x, s0.y, s0.z);
                    diffuse = dot3(kd, kd) < 1e-8f;
                    sincospif(2.0f * word_uniform(w.z), &ds1, &dc1);
                    sincospif(2.0f * word_uniform(w.w), &ds2, &dc2);
                }
                if (EXT && !diffuse && a.rr_p_max > 0.0f && l >= a.rr_depth) {
                    // a surviving path carries 1/sqrt(p), p held constant: the
                    // factor is the ratio of the recorded T_l to R_l T_{l-1}
                    const cf x0 = cadd(cscale(cf{p2.x, p2.y}, b.w00), cscale(cf{p3.x, p3.y}, b.w01));
                    const cf x1 = cadd(cscale(cf{p2.z, p2.w}, b.w00), cscale(cf{p3.z, p3.w}, b.w01));
                    const cf y0 = cadd(cscale(cf{p2.x, p2.y}, b.w10), cscale(cf{p3.x, p3.y}, b.w11));
                    const cf y1 = cadd(cscale(cf{p2.z, p2.w}, b.w10), cscale(cf{p3.z, p3.w}, b.w11));
                    const float pre = cabs2(kpe) * (cabs2(x0) + cabs2(x1)) + cabs2(kpa) * (cabs2(y0) + cabs2(y1));
                    const float rec = s2.x * s2.x + s2.y * s2.y + s2.z * s2.z + s2.w * s2.w + s3.x * s3.x +
                                      s3.y * s3.y + s3.z * s3.z + s3.w * s3.w;
                    const float sc = pre > 0.0f ? sqrtf(rec / pre) : 1.0f;
                    kpe = cscale(kpe, sc);
                    kpa = cscale(kpa, sc);
                    dkpe = cscale(dkpe, sc);
                    dkpa = cscale(dkpa, sc);
                }
                // u = W E_{l-1}
                cf f0 = cadd(cscale(cf{p2.x, p2.y}, ct), cscale(cf{p2.z, p2.w}, cp));
                cf f1 = cadd(cscale(cf{p3.x, p3.y}, ct), cscale(cf{p3.z, p3.w}, cp));
                cf u0 = cadd(cscale(f0, b.w00), cscale(f1, b.w01));
                cf u1 = cadd(cscale(f0, b.w10), cscale(f1, b.w11));
                int j = mat - a.mat0;
                if (EXT && diffuse) {
                    // E_l = sc N E with N = diag(x1, x2) [[ck, -sk], [sk, ck]] P
                    // unitary and sc^2 = c Gamma^2, Gamma^2 = ||D W E||^2 / ||E||^2
                    // (c, and a roulette factor, held constant).  Then
                    //   dL = 2 Re(lambda^H sc N dE) + (nu / Gamma^2) dGamma^2,
                    // nu = Re(lambda^H E_l), dGamma^2 = 2 Re((Q E - Gamma^2 E)^H dE) /
                    // ||E||^2 + 2 Re(Z d eta), Q = W^T |D|^2 W,
                    // Z = (conj(r_perp) dr_perp |u_0|^2 + conj(r_par) dr_par |u_1|^2) / ||E||^2
                    const float en2 = cabs2(f0) + cabs2(f1);
                    const float rp2 = cabs2(F.rperp), rl2 = cabs2(F.rpar);
                    const float g2 = en2 > 0.0f ? (rp2 * cabs2(u0) + rl2 * cabs2(u1)) / en2 : 0.0f;
                    const float tp = p2.x * p2.x + p2.y * p2.y + p2.z * p2.z + p2.w * p2.w + p3.x * p3.x +
                                     p3.y * p3.y + p3.z * p3.z + p3.w * p3.w;
                    const float tl = s2.x * s2.x + s2.y * s2.y + s2.z * s2.z + s2.w * s2.w + s3.x * s3.x +
                                     s3.y * s3.y + s3.z * s3.z + s3.w * s3.w;
                    if (g2 > 0.0f && tp > 0.0f) {
                        const float sc = sqrtf(tl / tp);   // ||N T||_F = ||T||_F
                        const cf el0 = cadd(cscale(cf{s2.x, s2.y}, ct), cscale(cf{s2.z, s2.w}, cp));
                        const cf el1 = cadd(cscale(cf{s3.x, s3.y}, ct), cscale(cf{s3.z, s3.w}, cp));
                        const float nu = cmulc(lam0, el0).re + cmulc(lam1, el1).re;
                        const float ig = nu / g2;
                        if (j >= 0 && j < kMatChunk) {
                            const cf Z = cscale(cadd(cscale(cmulc(F.rperp, F.drperp), cabs2(u0)),
                                                     cscale(cmulc(F.rpar, F.drpar), cabs2(u1))),
                                                1.0f / en2);
#pragma unroll
                            for (int jj = 0; jj < kMatChunk; jj++) {
                                if (jj == j) {
                                    ge[jj] += 2.0f * ig * Z.re;
                                    gs[jj] += 2.0f * ig * Z.im * a.pl.inv_eps0_omega;
                                }
                            }
                        }
                        // N from the incident basis (es, k x es) to (theta, phi)
                        const float3 kk = f3(p0.x, p0.y, p0.z), es = f3(p1.x, p1.y, p1.z);
                        float3 thi, phi_i;
                        sph_basis(kk, thi, phi_i);
                        const float3 ep = cross3(kk, es);
                        const float p00 = dot3(thi, es), p01 = dot3(thi, ep);
                        const float p10 = dot3(phi_i, es), p11 = dot3(phi_i, ep);
                        const float K = a.xpd[mat], sk = sqrtf(K), ck = sqrtf(1.0f - K);
                        const float a0 = ck * p00 - sk * p10, a1 = ck * p01 - sk * p11;
                        const float b0 = sk * p00 + ck * p10, b1 = sk * p01 + ck * p11;
                        // v = conj(diag(x1, x2)) lambda, then sc [[a0, b0], [a1, b1]] v
                        const cf v0 = cmulc(cf{dc1, ds1}, lam0), v1 = cmulc(cf{dc2, ds2}, lam1);
                        const float h = ig / en2;
                        // (Q E - Gamma^2 E) with Q E = W^T (|r_perp|^2 u0, |r_par|^2 u1)
                        const cf q0 = cadd(cscale(u0, rp2 * b.w00), cscale(u1, rl2 * b.w10));
                        const cf q1 = cadd(cscale(u0, rp2 * b.w01), cscale(u1, rl2 * b.w11));
                        lam0 = cadd(cscale(cadd(cscale(v0, a0), cscale(v1, b0)), sc), cscale(csub(q0, cscale(f0, g2)), h));
                        lam1 = cadd(cscale(cadd(cscale(v0, a1), cscale(v1, b1)), sc), cscale(csub(q1, cscale(f1, g2)), h));
                    } else {
                        lam0 = cf{0.0f, 0.0f};
                        lam1 = cf{0.0f, 0.0f};
                    }
                    continue;
                }
                if (j >= 0 && j < kMatChunk) {
                    // z = lambda^H dD/deta u, dD/deta = diag(dr_perp, -dr_par)
                    cf z = csub(cmulc(lam0, cmul(dkpe, u0)), cmulc(lam1, cmul(dkpa, u1)));
#pragma unroll
                    for (int jj = 0; jj < kMatChunk; jj++) {
                        if (jj == j) {
                            ge[jj] += 2.0f * z.re;
                            gs[jj] += 2.0f * z.im * a.pl.inv_eps0_omega;
                        }
                    }
                }
                // lambda <- R^H lambda = W^T diag(conj r_perp, -conj r_par) lambda
                cf v0 = cmulc(kpe, lam0);
                cf v1 = cmulc(kpa, lam1);
                v1 = cf{-v1.re, -v1.im};
                lam0 = cadd(cscale(v0, b.w00), cscale(v1, b.w10));
                lam1 = cadd(cscale(v0, b.w01), cscale(v1, b.w11));
            }
            if (a.write_orient) {
                // 2 Re(lambda_0^H dC), with C real
                go0 += 2.0f * (lam0.re * cth.d0 + lam1.re * cph.d0);
                go1 += 2.0f * (lam0.re * cth.d1 + lam1.re * cph.d1);
                go2 += 2.0f * (lam0.re * cth.d2 + lam1.re * cph.d2);
            }
        }
    }
    // ---- deterministic reduction: wave butterfly, then waves in order
    __shared__ double red[kBwdBlock / 64][2 * kMatChunk + 3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[2 * kMatChunk + 3];
#pragma unroll
    for (int j = 0; j < kMatChunk; j++) {
        v[j] = (double)ge[j];
        v[kMatChunk + j] = (double)gs[j];
    }
    v[2 * kMatChunk] = go0;
    v[2 * kMatChunk + 1] = go1;
    v[2 * kMatChunk + 2] = go2;
#pragma unroll
    for (int j = 0; j < 2 * kMatChunk + 3; j++) {
        double s = wave_sum_d(v[j]);
        if (lane == 0) red[wave][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMatChunk + 3) {
        double s = 0.0;
        for (int w = 0; w < kBwdBlock / 64; w++) s += red[w][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * (2 * kMatChunk + 3) + threadIdx.x] = s;
    }
}

// Sum the per-block partials of parameter j = blockIdx.x in a fixed order
// (lane i adds blocks i, i + 64, ... in turn, then a butterfly over the
// lanes) and scatter the sum to the outputs.  One wavefront per parameter:
// a single thread walking all blocks would chain hundreds of dependent loads.
__global__ void __launch_bounds__(64) k_backward_final(const double* __restrict__ partials, int nblocks, int n_mat,
                                                       int mat0, int write_orient, float* __restrict__ g_eps,
                                                       float* __restrict__ g_sig, float* __restrict__ g_orient) {
    const int P = 2 * kMatChunk + 3;
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) s += partials[(int64_t)b * P + j];
    s = wave_sum_d(s);
    if (threadIdx.x != 0) return;
    if (j < kMatChunk) {
        int m = mat0 + j;
        if (m < n_mat && g_eps) g_eps[m] = (float)s;
    } else if (j < 2 * kMatChunk) {
        int m = mat0 + j - kMatChunk;
        if (m < n_mat && g_sig) g_sig[m] = (float)s;
    } else if (write_orient && g_orient) {
        g_orient[j - 2 * kMatChunk] = (float)s;
    }
}

constexpr int kBwdP = 2 * kMatChunk + 3;

}  // namespace

// Per-block partial sums of the backward for callers that cannot allocate
// (rt_radio_map_backward_noalloc): one copy per GPU, kept until the process
// ends.  Every launch overwrites all kBwdBlocks x P entries before the final
// kernel reads them, so nothing needs clearing between calls; two calls that
// overlap on one GPU race on it.  In host code `scratch` is only a symbol:
// its device address comes from hipGetSymbolAddress (rt_backward_scratch).
static __device__ __align__(256) double scratch[(size_t)kBwdBlocks * kBwdP];

size_t rt_backward_scratch_bytes() { return sizeof(double) * (size_t)kBwdBlocks * kBwdP; }

rt_status rt_backward_scratch(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rt_hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return rt_fail(RT_EDEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the current device is `dev`: this resolves that device's copy
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return rt_hip_fail(e, "hipGetSymbolAddress(scratch)");
        addr[dev] = p;
    }
    *out = addr[dev];
    return RT_OK;
}

rt_status rt_launch_backward(const BwdLaunch& b, hipStream_t st) {
    rt_scene* s = const_cast<rt_scene*>(b.scene);
    const int P = kBwdP;
    size_t need = sizeof(double) * (size_t)kBwdBlocks * P;
    double* partials = (double*)b.workspace;
    if (partials) {
        if (b.workspace_bytes < need)
            return rt_fail(RT_EOVERFLOW, "rt_radio_map_backward: workspace smaller than the partial sums");
    } else if (s->grad_ws_bytes < need) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(s->grad_ws);
        s->grad_ws = nullptr;
        s->grad_ws_bytes = 0;
        hipError_t e = hipMalloc(&s->grad_ws, need);
        if (e != hipSuccess) return rt_hip_fail(e, "rt_radio_map_backward: workspace");
        s->grad_ws_bytes = need;
    }
    if (!partials) partials = (double*)s->grad_ws;
    BwdArgs a;
    a.seg = b.tape->seg;
    a.nseg = b.tape->nseg;
    a.n = b.tape->n_rays;
    a.ray_begin = b.ray_begin;
    a.normals = s->normals;
    a.eps_r = b.eps_r;
    a.sigma = b.sigma;
    a.tx = b.tx;
    a.pl = b.pl;
    a.npol = b.tx.pol == RT_POL_DUAL ? 2 : 1;
    a.thickness = b.thickness;
    a.refraction = b.refraction;
    a.k0 = b.k0;
    a.rr_depth = b.rr_depth;
    a.rr_p_max = b.rr_p_max;
    a.scattering = b.scattering;
    a.xpd = b.xpd;
    a.seed = b.seed;
    a.grad_map = b.grad_map;
    a.map_stride = (int64_t)b.pl.W * b.pl.H;
    a.n_mat = s->n_mat;
    a.P = P;
    a.partials = partials;
    const bool ext = a.thickness || a.refraction || a.scattering || a.rr_p_max > 0.0f;
    for (int m0 = 0; m0 < std::max(1, s->n_mat); m0 += kMatChunk) {
        a.mat0 = m0;
        a.write_orient = (m0 == 0) ? 1 : 0;
        if (ext)
            hipLaunchKernelGGL(k_backward<true>, dim3(kBwdBlocks), dim3(kBwdBlock), 0, st, a);
        else
            hipLaunchKernelGGL(k_backward<false>, dim3(kBwdBlocks), dim3(kBwdBlock), 0, st, a);
        hipLaunchKernelGGL(k_backward_final, dim3(P), dim3(64), 0, st, (const double*)partials, kBwdBlocks,
                           s->n_mat, m0, a.write_orient, b.grad_eps, b.grad_sigma, b.grad_orient);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rt_hip_fail(e, "backward launch");
    return RT_OK;
}
