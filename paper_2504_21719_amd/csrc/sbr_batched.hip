// sbr_batched.hip -- many transmitters and many material samples per call.
//
// Work over all transmitters is one index space: transmitter t owns the
// global ray indices [prefix[t], prefix[t+1]) (ordered largest budget first,
// so long lattices start early), and lanes of the persistent kernel pull
// indices from one device counter, whatever transmitter they belong to.
//
//  * one material set, forward only: a single persistent launch traces,
//    reflects and deposits into the map of each ray's transmitter;
//  * several material samples and/or gradients: the persistent launch traces
//    every ray once and records its geometry (hit slot, crossed cell,
//    direction and basis per segment).  The hit sequence does not depend on
//    the materials or the antenna, so one traversal serves every sample.  A
//    second kernel takes the rays 64 at a time: their launch patterns and
//    bounce geometry are computed once into LDS, and each wavefront of the
//    block then runs one sample at a time for the 64 rays (lane = ray): it
//    propagates the field through the recorded bounces with that sample's
//    permittivities (eq. fresnel_vac, eq. eta), deposits into the sample's
//    map, and, given upstream gradients, runs the same reverse sweep as the
//    plain adjoint (dJ/dp = 2 Re(lambda^H dR/dp E)) with the fields of the
//    forward pass kept in registers.  Slab walls without refraction
//    (eq. fresnel_slab) and transmit arrays fit this split: neither changes
//    a ray's path, only its coefficients or its weight.
//    The geometry records are kept in the launch order of the traversal
//    (azimuth-sorted chunks of each lattice), so the lanes of a wavefront of
//    the field pass hold nearby directions: they read consecutive records,
//    and their same-cell crossings are summed across the wavefront before
//    the atomics.  Measured on 16 samples of 1e6 rays forward + backward:
//    one thread per ray looping over the samples with every bounce's
//    geometry in registers (227 VGPRs, per-lane atomics with gradients)
//    took 1.13 ms; geometry in LDS shared by the block's wavefronts (157
//    VGPRs) with wavefront deposits took 0.74 ms; with the forward fields
//    in LDS as well for paths of at most six segments (124 VGPRs, four
//    wavefronts per SIMD) it takes 0.66 ms.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sbr_common.h"

using namespace rtd;

namespace {

constexpr int kMaxSeg = 9;      // segments per path of the sample kernel (L <= 8 with gradients)
constexpr int kMaxMat = 8;      // materials with gradients in batched mode
constexpr int kSampBlock = 256;

struct SampArgs {
    const float4* geom;     // [l][2][total]
    const int* nseg;        // [total]
    int64_t total;
    const TxDesc* txs;
    const int64_t* prefix;
    const int32_t* slots;
    int n_tx;
    int S;
    const float4* normals;
    const float* eps_r;     // [S][n_mat]
    const float* sigma;
    int n_mat;
    PlaneDesc pl;
    float* maps;            // [n_tx][S][H][W]
    const float* grad_maps; // [n_tx][S][H][W] or null
    const int64_t* woff;    // [n_tx + 1] prefix of the wavefronts each transmitter's rays touch
    double* gws;            // gradient mode: FP64 partial sums, transmitter t's block at
                            // woff[t] S P, laid out [s][j][wavefront of t]
    int P;                  // 2 n_mat + 3
    const float* thickness; // slab thickness per material (m, shared by the samples), or null
    float k0;               // 2 pi / lambda
    // launch order of the geometry tape: record g of transmitter t holds work
    // item n = g - prefix[t], whose lattice index is the chunk permutation of n
    const int* operm;       // null: records are in lattice order
    const int* oshift;
    int olog2m;
};

// Lattice index of work item n of transmitter td (the forward's launch order).
__device__ __forceinline__ int64_t lattice_index(const SampArgs& a, const TxDesc& td, int64_t n) {
    if (a.operm && (n >> a.olog2m) < td.n_chunks) {
        const int64_t M = (int64_t)1 << a.olog2m, c = n >> a.olog2m, c0 = c << a.olog2m;
        n = c0 + a.operm[((n - c0) + a.oshift[td.shift0 + c]) & (M - 1)];
    }
    return n;
}

__device__ __forceinline__ float wave_sum_f(float v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Deposit of one crossing per lane (cell < 0: none) into the map of the
// lane's transmitter slot: at most four groups of lanes with the same slot
// and cell are summed across the wavefront before one atomic each; lanes
// left over add their own crossings.  Every lane of the wavefront calls it.
__device__ __forceinline__ void deposit_wave(float* map, int cell, float w, int slot) {
    const int lane = threadIdx.x & 63;
    unsigned long long pend = __ballot(cell >= 0);
    bool done = cell < 0;
    for (int groups = 0; pend; groups++) {
        if (groups == 4) {
            if (!done) unsafeAtomicAdd(map + cell, w);
            break;
        }
        const int leader = __ffsll((long long)pend) - 1;
        const int lc = __shfl(cell, leader), ls = __shfl(slot, leader);
        const bool mine = !done && cell == lc && slot == ls;
        const unsigned long long grp = __ballot(mine);
        const float v = wave_sum_f(mine ? w : 0.0f);
        if (lane == leader) unsafeAtomicAdd(map + lc, v);
        if (mine) done = true;
        pend &= ~grp;
    }
}

__device__ __forceinline__ int find_tx_s(const int64_t* __restrict__ prefix, int n_tx, int64_t g) {
    int lo = 0, hi = n_tx;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double wsum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// A block is up to four wavefronts over the same 64 consecutive rays.  The
// rays' launch patterns and the geometry of every bounce (basis change W,
// cos(theta_1), material, crossed cell, 1 / |cos| of the plane crossing) are
// computed once per ray, cooperatively, into LDS; wavefront w then runs
// samples w, w + n_w, ... for the 64 rays (lane = ray), so that a lane keeps
// only one sample's fields in registers, and a wavefront's deposits go to one
// sample's map.
constexpr int kSampRays = 64;
constexpr int kShortSeg = 6;    // paths of at most 6 segments (L <= 5): the short variant
template <int NSEG>
struct SampShared {
    float geo[NSEG][6][kSampRays];      // w00, w01, w10, w11, cos(theta_1), 1 / |cos| at the plane
    int mc[NSEG][2][kSampRays];         // material of the bounce ending the segment, crossed cell
    float hdr[9][kSampRays];            // C_theta (value, d/d yaw, pitch, roll), C_phi (same), kappa
    int ns[kSampRays], slot[kSampRays], txi[kSampRays];
};

// NSEG: segments per path the variant holds (kShortSeg or kMaxSeg).  With
// gradients the short variant keeps the forward fields for the reverse sweep
// in LDS too (a lane's four floats per segment), which leaves it few enough
// registers for four wavefronts per SIMD; the long one keeps them in
// registers.
template <bool GRAD, bool SLAB, bool ARR, int NSEG>
__global__ void __launch_bounds__(kSampBlock) k_samples(const SampArgs a) {
    __shared__ SampShared<NSEG> sh;
    constexpr bool kLdsFields = GRAD && NSEG <= kShortSeg;
    // [segment][wavefront][Re E0, Im E0, Re E1, Im E1][lane]
    __shared__ float fld[kLdsFields ? NSEG * 4 * 4 * kSampRays : 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n_wv = blockDim.x >> 6;
    const int64_t HW = (int64_t)a.pl.W * a.pl.H;
    const int64_t T = a.total;
    const int S = a.S;
    for (int64_t g0 = (int64_t)blockIdx.x * kSampRays; g0 < T; g0 += (int64_t)gridDim.x * kSampRays) {
        // ---- per ray: transmitter, segment count, launch pattern (wavefront 0)
        if (wv == 0) {
            const int64_t g = g0 + lane;
            int ns = 0, slot_out = -1, tx_i = -1;
            d3f cth = {0, 0, 0, 0}, cph = {0, 0, 0, 0};
            float kap = 0.0f;
            if (g < T) {
                const int t = find_tx_s(a.prefix, a.n_tx, g);
                const TxDesc td = a.txs[t];
                tx_i = t;
                slot_out = a.slots[t];
                ns = a.nseg[g];
                const int64_t n = lattice_index(a, td, g - a.prefix[t]);
                Launch Lr = fib_launch(n, td.n_rays);
                if (GRAD) {
                    tx_pattern<d3f>(Lr, td, td.pol == 1 ? 1 : 0, cth, cph);
                } else {
                    tx_pattern<float>(Lr, td, td.pol == 1 ? 1 : 0, cth.v, cph.v);
                }
                // |alpha|^2 of a transmit array depends on the direction only
                kap = ARR && td.n_ant > 0 ? td.kappa * array_gain(Lr, td) : td.kappa;
            }
            sh.ns[lane] = ns;
            sh.slot[lane] = slot_out;
            sh.txi[lane] = tx_i;
            sh.hdr[0][lane] = cth.v;
            sh.hdr[1][lane] = cth.d0;
            sh.hdr[2][lane] = cth.d1;
            sh.hdr[3][lane] = cth.d2;
            sh.hdr[4][lane] = cph.v;
            sh.hdr[5][lane] = cph.d0;
            sh.hdr[6][lane] = cph.d1;
            sh.hdr[7][lane] = cph.d2;
            sh.hdr[8][lane] = kap;
        }
        // ---- bounce geometry of every (segment, ray), all lanes of the block
        for (int it = threadIdx.x; it < NSEG * kSampRays; it += blockDim.x) {
            const int l = it / kSampRays, r = it % kSampRays;
            const int64_t g = g0 + r;
            if (g >= T) continue;
            const int ns = a.nseg[g];
            if (l >= ns) continue;
            const float4* sp = a.geom + (int64_t)l * 2 * T + g;
            const float4 s0 = sp[0], s1 = sp[T];
            sh.mc[l][1][r] = __float_as_int(s1.w);
            sh.geo[l][5][r] = __builtin_amdgcn_rcpf(fabsf(s0.z));
            if (l + 1 < ns) {
                const float4 nm = a.normals[__float_as_int(s0.w)];
                sh.mc[l][0][r] = __float_as_int(nm.w);
                Bounce b = bounce_geometry(f3(s0.x, s0.y, s0.z), f3(s1.x, s1.y, s1.z), f3(nm.x, nm.y, nm.z));
                sh.geo[l][0][r] = b.w00;
                sh.geo[l][1][r] = b.w01;
                sh.geo[l][2][r] = b.w10;
                sh.geo[l][3][r] = b.w11;
                sh.geo[l][4][r] = b.c;
            }
        }
        __syncthreads();
        const int ns = sh.ns[lane], slot_out = sh.slot[lane], tx_i = sh.txi[lane];
        const bool valid = tx_i >= 0;
        const d3f cth = {sh.hdr[0][lane], sh.hdr[1][lane], sh.hdr[2][lane], sh.hdr[3][lane]};
        const d3f cph = {sh.hdr[4][lane], sh.hdr[5][lane], sh.hdr[6][lane], sh.hdr[7][lane]};
        const float kap = sh.hdr[8][lane];
        for (int s = wv; s < S; s += n_wv) {
            float ge[kMaxMat], gs[kMaxMat], go[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < kMaxMat; j++) {
                ge[j] = 0.f;
                gs[j] = 0.f;
            }
            cf E0[NSEG], E1[NSEG];
            float* const fl = fld + (kLdsFields ? wv * 4 * kSampRays + lane : 0);
            const float* eps = a.eps_r + (int64_t)s * a.n_mat;
            const float* sig = a.sigma + (int64_t)s * a.n_mat;
            {
                // forward field pass: every lane takes part in the wavefront
                // deposits (lanes without a ray have ns = 0)
                float* map = a.maps + ((int64_t)max(slot_out, 0) * S + s) * HW;
                cf e0 = {cth.v, 0.f}, e1 = {cph.v, 0.f};
#pragma unroll
                for (int l = 0; l < NSEG; l++) {
                    const int cl = l < ns ? sh.mc[l][1][lane] : -1;
                    const float gk = kap * sh.geo[l][5][lane];
                    if (__ballot(l < ns) == 0ull) break;
                    deposit_wave(map, cl, cl >= 0 ? gk * (cabs2(e0) + cabs2(e1)) : 0.0f, slot_out);
                    if (l >= ns) continue;
                    if (kLdsFields) {
                        float* f = fl + l * 16 * kSampRays;
                        f[0] = e0.re;
                        f[kSampRays] = e0.im;
                        f[2 * kSampRays] = e1.re;
                        f[3 * kSampRays] = e1.im;
                    } else {
                        E0[l] = e0;
                        E1[l] = e1;
                    }
                    if (l + 1 < ns) {
                        const int m = sh.mc[l][0][lane];
                        Fresnel F = fresnel<false>(sh.geo[l][4][lane], cf{eps[m], -sig[m] * a.pl.inv_eps0_omega});
                        if (SLAB) {
                            cf tp, tl;
                            slab(F, a.k0 * a.thickness[m], tp, tl);
                        }
                        const float w00 = sh.geo[l][0][lane], w01 = sh.geo[l][1][lane];
                        const float w10 = sh.geo[l][2][lane], w11 = sh.geo[l][3][lane];
                        cf u0 = cadd(cscale(e0, w00), cscale(e1, w01));
                        cf u1 = cadd(cscale(e0, w10), cscale(e1, w11));
                        e0 = cmul(F.rperp, u0);
                        e1 = cmul(cf{-F.rpar.re, -F.rpar.im}, u1);
                    }
                }
            }
            if (GRAD && valid) {
                const float* G = a.grad_maps + ((int64_t)slot_out * S + s) * HW;
                cf lam0 = {0, 0}, lam1 = {0, 0};
                auto field = [&](int l, cf& f0, cf& f1) {
                    if (kLdsFields) {
                        const float* f = fl + l * 16 * kSampRays;
                        f0 = cf{f[0], f[kSampRays]};
                        f1 = cf{f[2 * kSampRays], f[3 * kSampRays]};
                    } else {
                        f0 = E0[l];
                        f1 = E1[l];
                    }
                };
#pragma unroll
                for (int l = NSEG - 1; l >= 0; l--) {
                    if (l >= ns) continue;
                    const int cl = sh.mc[l][1][lane];
                    if (cl >= 0) {
                        float al = G[cl] * (kap * sh.geo[l][5][lane]);
                        cf f0, f1;
                        field(l, f0, f1);
                        lam0 = cadd(lam0, cscale(f0, al));
                        lam1 = cadd(lam1, cscale(f1, al));
                    }
                    if (l == 0) continue;
                    const int k = l - 1;      // the bounce that ends segment l-1
                    const int m = sh.mc[k][0][lane];
                    Fresnel F = fresnel<true>(sh.geo[k][4][lane], cf{eps[m], -sig[m] * a.pl.inv_eps0_omega});
                    if (SLAB) {
                        cf tp, tl, dtp, dtl;
                        slab_grad(F, a.k0 * a.thickness[m], tp, tl, dtp, dtl);
                    }
                    const float w00 = sh.geo[k][0][lane], w01 = sh.geo[k][1][lane];
                    const float w10 = sh.geo[k][2][lane], w11 = sh.geo[k][3][lane];
                    cf f0, f1;
                    field(k, f0, f1);
                    cf u0 = cadd(cscale(f0, w00), cscale(f1, w01));
                    cf u1 = cadd(cscale(f0, w10), cscale(f1, w11));
                    cf z = csub(cmulc(lam0, cmul(F.drperp, u0)), cmulc(lam1, cmul(F.drpar, u1)));
#pragma unroll
                    for (int jj = 0; jj < kMaxMat; jj++) {
                        if (jj == m) {
                            ge[jj] += 2.0f * z.re;
                            gs[jj] += 2.0f * z.im * a.pl.inv_eps0_omega;
                        }
                    }
                    cf v0 = cmulc(F.rperp, lam0);
                    cf v1 = cmulc(F.rpar, lam1);
                    v1 = cf{-v1.re, -v1.im};
                    lam0 = cadd(cscale(v0, w00), cscale(v1, w10));
                    lam1 = cadd(cscale(v0, w01), cscale(v1, w11));
                }
                go[0] = 2.0f * (lam0.re * cth.d0 + lam1.re * cph.d0);
                go[1] = 2.0f * (lam0.re * cth.d1 + lam1.re * cph.d1);
                go[2] = 2.0f * (lam0.re * cth.d2 + lam1.re * cph.d2);
            }
            if (GRAD) {
                // one partial sum per (transmitter, 64-ray group, sample,
                // parameter), summed later in a fixed order: the lanes of each
                // transmitter in this group (usually one) are summed with a
                // butterfly and their leader stores the sums in that
                // transmitter's entry for this group
                const int64_t gw = g0 >> 6;
                unsigned long long pend = __ballot(valid);
                bool done = !valid;
                while (pend) {
                    int leader = __ffsll((long long)pend) - 1;
                    int lt = __shfl(tx_i, leader);
                    bool mine = !done && tx_i == lt;
                    unsigned long long grp = __ballot(mine);
                    const int64_t w0 = a.woff[lt], nw = a.woff[lt + 1] - w0;
                    double* dst = a.gws + w0 * S * a.P + (int64_t)s * a.P * nw + (gw - (a.prefix[lt] >> 6));
                    for (int j = 0; j < a.n_mat && j < kMaxMat; j++) {
                        double v = wsum(mine ? (double)ge[j] : 0.0);
                        double u = wsum(mine ? (double)gs[j] : 0.0);
                        if (lane == leader) {
                            dst[j * nw] = v;
                            dst[(a.n_mat + j) * nw] = u;
                        }
                    }
                    for (int j = 0; j < 3; j++) {
                        double v = wsum(mine ? (double)go[j] : 0.0);
                        if (lane == leader) dst[(2 * a.n_mat + j) * nw] = v;
                    }
                    if (mine) done = true;
                    pend &= ~grp;
                }
            }
        }
        // the next group of rays overwrites the shared records
        __syncthreads();
    }
}

// Depth > 8 without gradients: one thread per (ray, sample), geometry
// recomputed per sample.
__global__ void __launch_bounds__(kSampBlock) k_samples_deep(const SampArgs a) {
    const int s = blockIdx.y;
    const int64_t HW = (int64_t)a.pl.W * a.pl.H;
    const int64_t T = a.total;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < T; g += (int64_t)gridDim.x * blockDim.x) {
        const int t = find_tx_s(a.prefix, a.n_tx, g);
        const TxDesc td = a.txs[t];
        const int slot_out = a.slots[t];
        const int ns = a.nseg[g];
        const int64_t nl = lattice_index(a, td, g - a.prefix[t]);
        const float* eps = a.eps_r + (int64_t)s * a.n_mat;
        const float* sig = a.sigma + (int64_t)s * a.n_mat;
        float* map = a.maps + ((int64_t)slot_out * a.S + s) * HW;
        Launch Lr = fib_launch(nl, td.n_rays);
        float ct, cp;
        tx_pattern<float>(Lr, td, td.pol == 1 ? 1 : 0, ct, cp);
        const float kap = td.n_ant > 0 ? td.kappa * array_gain(Lr, td) : td.kappa;
        cf e0 = {ct, 0.f}, e1 = {cp, 0.f};
        for (int l = 0; l < ns; l++) {
            const float4* sp = a.geom + (int64_t)l * 2 * T + g;
            float4 s0 = sp[0], s1 = sp[T];
            int cell = __float_as_int(s1.w);
            if (cell >= 0) unsafeAtomicAdd(map + cell, kap * __builtin_amdgcn_rcpf(fabsf(s0.z)) * (cabs2(e0) + cabs2(e1)));
            if (l + 1 < ns) {
                float4 nm = a.normals[__float_as_int(s0.w)];
                int m = __float_as_int(nm.w);
                Bounce b = bounce_geometry(f3(s0.x, s0.y, s0.z), f3(s1.x, s1.y, s1.z), f3(nm.x, nm.y, nm.z));
                Fresnel F = fresnel<false>(b.c, cf{eps[m], -sig[m] * a.pl.inv_eps0_omega});
                if (a.thickness) {
                    cf tp, tl;
                    slab(F, a.k0 * a.thickness[m], tp, tl);
                }
                cf u0 = cadd(cscale(e0, b.w00), cscale(e1, b.w01));
                cf u1 = cadd(cscale(e0, b.w10), cscale(e1, b.w11));
                e0 = cmul(F.rperp, u0);
                e1 = cmul(cf{-F.rpar.re, -F.rpar.im}, u1);
            }
        }
    }
}

// Gradient of parameter j = blockIdx.x for sample s = blockIdx.y of ordered
// transmitter t = blockIdx.z: the sum of its per-wavefront partials in a fixed
// order (thread i adds entries i, i + 256, ... in turn; butterflies within
// wavefronts; the four wavefront sums in order), written to the caller's
// [slot][s][j] entry.
constexpr int kFinalBlock = 256;
__global__ void __launch_bounds__(kFinalBlock) k_grads_final(const double* __restrict__ gws,
                                                             const int64_t* __restrict__ woff,
                                                             const int32_t* __restrict__ slots, int S, int P,
                                                             float* __restrict__ out) {
    __shared__ double part[kFinalBlock / 64];
    const int j = blockIdx.x, s = blockIdx.y, t = blockIdx.z;
    const int64_t w0 = woff[t], nw = woff[t + 1] - w0;
    const double* src = gws + w0 * S * P + ((int64_t)s * P + j) * nw;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nw; k += kFinalBlock) acc += src[k];
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kFinalBlock / 64; w++) tot += part[w];
        out[((int64_t)slots[t] * S + s) * P + j] = (float)tot;
    }
}

}  // namespace

// Grow the batched workspaces (never called while a graph is being captured).
rt_status rt_batched_workspace(const BatchLaunch& b, hipStream_t st) {
    rt_scene* s = const_cast<rt_scene*>(b.scene);
    const bool grad = b.grad_maps != nullptr;
    if (grad && (b.L + 1 > kMaxSeg || s->n_mat > kMaxMat))
        return rt_fail(RT_EUNSUPPORTED, "rt_radio_map_batched: gradients need max_depth <= 8 and <= 8 materials");
    if (b.n_samples == 1 && !grad) return RT_OK;
    size_t need = sizeof(float4) * 2 * (size_t)(b.L + 1) * (size_t)b.total_rays + sizeof(int) * (size_t)b.total_rays;
    if (s->geom_ws_bytes < need) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(s->geom_ws);
        s->geom_ws = nullptr;
        s->geom_ws_bytes = 0;
        hipError_t e = hipMalloc(&s->geom_ws, need);
        if (e != hipSuccess) return rt_hip_fail(e, "rt_radio_map_batched: geometry tape");
        s->geom_ws_bytes = need;
    }
    size_t gneed = sizeof(double) * (size_t)b.total_waves * b.n_samples * (2 * s->n_mat + 3);
    if (grad && s->bgrad_ws_bytes < gneed) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(s->bgrad_ws);
        s->bgrad_ws = nullptr;
        s->bgrad_ws_bytes = 0;
        hipError_t e = hipMalloc(&s->bgrad_ws, gneed);
        if (e != hipSuccess) return rt_hip_fail(e, "rt_radio_map_batched: gradient workspace");
        s->bgrad_ws_bytes = gneed;
    }
    return RT_OK;
}

// Queue the batched work on `st`.  Allocates nothing (rt_batched_workspace
// must have run), so the sequence can be captured into a HIP graph.
rt_status rt_launch_batched(const BatchLaunch& b, hipStream_t st) {
    rt_scene* s = const_cast<rt_scene*>(b.scene);
    const int64_t HW = (int64_t)b.pl.W * b.pl.H;
    const int S = b.n_samples;
    const bool grad = b.grad_maps != nullptr;
    if (S == 1 && !grad) {
        return rt_launch_forward_multi(s, b.eps_r, b.sigma, b.pl, b.L, b.t_min, b.block, b.deposit, b.refill,
                                       b.order, b.max_chunks, b.tx_dev, b.prefix_dev, b.tx_slot_dev, b.n_tx,
                                       b.total_rays, false, b.maps, HW, HW * b.n_tx, nullptr, nullptr, &b.ext, st);
    }
    size_t need = sizeof(float4) * 2 * (size_t)(b.L + 1) * (size_t)b.total_rays + sizeof(int) * (size_t)b.total_rays;
    const int P = 2 * s->n_mat + 3;
    if (s->geom_ws_bytes < need || (grad && s->bgrad_ws_bytes < sizeof(double) * (size_t)b.total_waves * S * P))
        return rt_fail(RT_EINVAL, "rt_radio_map_batched: workspace not prepared");
    float4* geom = (float4*)s->geom_ws;
    int* nseg = (int*)((char*)s->geom_ws + sizeof(float4) * 2 * (size_t)(b.L + 1) * (size_t)b.total_rays);
    rt_status r = rt_launch_forward_multi(s, b.eps_r, b.sigma, b.pl, b.L, b.t_min, b.block, b.deposit, b.refill,
                                          b.order, b.max_chunks, b.tx_dev, b.prefix_dev, b.tx_slot_dev, b.n_tx,
                                          b.total_rays, true, b.maps, HW, HW * b.n_tx * S, geom, nseg, nullptr, st);
    if (r != RT_OK) return r;
    SampArgs a;
    a.geom = geom;
    a.nseg = nseg;
    a.total = b.total_rays;
    a.txs = b.tx_dev;
    a.prefix = b.prefix_dev;
    a.slots = b.tx_slot_dev;
    a.n_tx = b.n_tx;
    a.S = S;
    a.normals = s->normals;
    a.eps_r = b.eps_r;
    a.sigma = b.sigma;
    a.n_mat = s->n_mat;
    a.pl = b.pl;
    a.maps = b.maps;
    a.grad_maps = b.grad_maps;
    a.woff = b.woff_dev;
    a.gws = (double*)s->bgrad_ws;
    a.P = P;
    a.thickness = b.ext.thickness;
    a.k0 = b.ext.k0;
    a.operm = b.order ? b.order->perm : nullptr;
    a.oshift = s->shifts;
    a.olog2m = b.order ? b.order->log2m : 0;
    unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1 << 20, (b.total_rays + 63) / 64));
    const unsigned sblock = 64u * (unsigned)std::min(4, S);   // wavefronts of one 64-ray group, one per sample
    if (b.total_rays > 0) {
        // slab walls and transmit arrays each get their own variant, so that
        // the plain one keeps its registers
        const bool slab_walls = a.thickness != nullptr, arrays = b.has_arrays;
        if (grad || b.L + 1 <= kMaxSeg) {
            const int v = (grad ? 4 : 0) + (slab_walls ? 2 : 0) + (arrays ? 1 : 0);
            if (b.L + 1 <= kShortSeg) {
                switch (v) {
                case 0: hipLaunchKernelGGL((k_samples<false, false, false, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 1: hipLaunchKernelGGL((k_samples<false, false, true, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 2: hipLaunchKernelGGL((k_samples<false, true, false, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 3: hipLaunchKernelGGL((k_samples<false, true, true, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 4: hipLaunchKernelGGL((k_samples<true, false, false, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 5: hipLaunchKernelGGL((k_samples<true, false, true, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 6: hipLaunchKernelGGL((k_samples<true, true, false, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                default: hipLaunchKernelGGL((k_samples<true, true, true, kShortSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                }
            } else {
                switch (v) {
                case 0: hipLaunchKernelGGL((k_samples<false, false, false, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 1: hipLaunchKernelGGL((k_samples<false, false, true, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 2: hipLaunchKernelGGL((k_samples<false, true, false, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 3: hipLaunchKernelGGL((k_samples<false, true, true, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 4: hipLaunchKernelGGL((k_samples<true, false, false, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 5: hipLaunchKernelGGL((k_samples<true, false, true, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                case 6: hipLaunchKernelGGL((k_samples<true, true, false, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                default: hipLaunchKernelGGL((k_samples<true, true, true, kMaxSeg>), dim3(bx), dim3(sblock), 0, st, a); break;
                }
            }
        } else {
            unsigned by = (unsigned)std::min<int64_t>(65535, (b.total_rays + kSampBlock - 1) / kSampBlock);
            hipLaunchKernelGGL(k_samples_deep, dim3(by, S), dim3(kSampBlock), 0, st, a);
        }
    }
    if (grad && b.total_rays > 0)
        hipLaunchKernelGGL(k_grads_final, dim3(P, S, b.n_tx), dim3(kFinalBlock), 0, st, (const double*)s->bgrad_ws,
                           b.woff_dev, b.tx_slot_dev, S, P, b.grads);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rt_hip_fail(e, "batched launch");
    return RT_OK;
}
