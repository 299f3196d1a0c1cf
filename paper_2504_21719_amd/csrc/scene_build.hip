// scene_build.hip -- on-device LBVH construction for gfx950.
//
// Pipeline (all device work on the caller's stream):
//   ingest      validate indices / materials / finiteness, per-triangle AABB,
//               centroid bounds (block-reduced, then ordered-int atomics)
//   morton      63-bit Morton code (21 bits per axis) of every AABB centre,
//               quantised with one scale for all axes (the largest extent)
//   radix sort  stable LSD sort of (code, triangle) pairs, 8 passes of 8 bits;
//               equal codes keep input order, and the Karras split below breaks
//               ties by index, so every key is effectively unique
//   karras      one thread per internal node finds its key range and split
//               from longest-common-prefix lengths (Karras, HPG 2012)
//   depth       each internal node walks to the root to learn its depth
//   refit       one launch per depth level, deepest first: a node's two child
//               boxes are written only after every deeper level finished, so
//               no inter-block flags or fences are needed
//   gather      triangles, unit normals (computed in FP64) and materials in
//               Morton order, so that traversal touches nearby memory
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rt_internal.h"

#define HIPCHK(x)                                            \
    do {                                                     \
        hipError_t _e = (x);                                 \
        if (_e != hipSuccess) {                              \
            cleanup();                                       \
            return rt_hip_fail(_e, #x);                      \
        }                                                    \
    } while (0)

namespace {

constexpr int kBlock = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;

__device__ __forceinline__ unsigned f2ord(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
float ord2f_host(unsigned u) {
    unsigned v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    float f;
    std::memcpy(&f, &v, 4);
    return f;
}

// Validation + AABB + centroid bounds.
__global__ void k_ingest(const float* __restrict__ V, int64_t n_v, const int32_t* __restrict__ F,
                         const int32_t* __restrict__ M, int32_t n_mat, int64_t n_tri,
                         float4* __restrict__ raw, float4* __restrict__ cen,
                         unsigned* __restrict__ bounds, unsigned* __restrict__ err) {
    __shared__ unsigned sb[6];
    if (threadIdx.x < 6) sb[threadIdx.x] = (threadIdx.x < 3) ? 0xffffffffu : 0u;
    __syncthreads();
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tri) {
        int32_t i0 = F[3 * t], i1 = F[3 * t + 1], i2 = F[3 * t + 2];
        int32_t m = M[t];
        bool ok = true;
        if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= n_v || i1 >= n_v || i2 >= n_v) {
            atomicOr(err, 1u);
            ok = false;
        }
        if (m < 0 || m >= n_mat) {
            atomicOr(err, 2u);
            ok = false;
        }
        if (ok) {
            float p[9];
            const int32_t idx[3] = {i0, i1, i2};
            bool fin = true;
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) {
                    p[3 * a + c] = V[3 * (int64_t)idx[a] + c];
                    fin = fin && isfinite(p[3 * a + c]);
                }
            if (!fin) {
                atomicOr(err, 4u);
            } else {
                raw[3 * t + 0] = make_float4(p[0], p[1], p[2], 0.0f);
                raw[3 * t + 1] = make_float4(p[3], p[4], p[5], 0.0f);
                raw[3 * t + 2] = make_float4(p[6], p[7], p[8], 0.0f);
                float c[3];
                for (int a = 0; a < 3; a++) {
                    float lo = fminf(fminf(p[a], p[3 + a]), p[6 + a]);
                    float hi = fmaxf(fmaxf(p[a], p[3 + a]), p[6 + a]);
                    c[a] = 0.5f * (lo + hi);
                    atomicMin(&sb[a], f2ord(c[a]));
                    atomicMax(&sb[3 + a], f2ord(c[a]));
                }
                cen[t] = make_float4(c[0], c[1], c[2], 0.0f);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], sb[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&bounds[threadIdx.x], sb[threadIdx.x]);
}

__device__ __forceinline__ uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_morton(const float4* __restrict__ cen, int64_t n, float lx, float ly, float lz,
                         float sx, float sy, float sz, uint64_t* __restrict__ keys,
                         uint32_t* __restrict__ vals) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float4 c = cen[t];
    const float qmax = 2097151.0f;
    uint32_t qx = (uint32_t)fminf(fmaxf((c.x - lx) * sx, 0.0f), qmax);
    uint32_t qy = (uint32_t)fminf(fmaxf((c.y - ly) * sy, 0.0f), qmax);
    uint32_t qz = (uint32_t)fminf(fmaxf((c.z - lz) * sz, 0.0f), qmax);
    keys[t] = (spread21(qx) << 2) | (spread21(qy) << 1) | spread21(qz);
    vals[t] = (uint32_t)t;
}

// ---- radix sort -----------------------------------------------------------
__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          unsigned* __restrict__ hist, int nblocks) {
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int i = 0; i < kRsItems; i++) {
        int64_t idx = base + (int64_t)i * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `count` unsigned values in place, one block of 1024
// (used for the per-tile sums of the multi-block scan below).
__global__ void k_scan1(unsigned* __restrict__ data, int64_t count) {
    __shared__ unsigned part[1024];
    const int T = 1024;
    int64_t per = (count + T - 1) / T;
    int64_t b = threadIdx.x * per, e = min(count, b + per);
    unsigned s = 0;
    for (int64_t i = b; i < e; i++) s += data[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        unsigned v = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned run = part[threadIdx.x] - s;   // exclusive prefix of this chunk
    for (int64_t i = b; i < e; i++) {
        unsigned v = data[i];
        data[i] = run;
        run += v;
    }
}

// Multi-block exclusive scan: tiles of kScanTile values, one 256-thread block
// each.  Pass 1 writes every tile's sum, the sums are scanned by k_scan1, and
// pass 2 scans each tile from its offset.  A tile is staged in LDS with one
// pad word per 32 so that a thread's 16 consecutive values sit in distinct
// banks.
constexpr int kScanTile = 4096;
constexpr int kScanPer = kScanTile / kBlock;

__device__ __forceinline__ int scan_pad(int j) { return j + (j >> 5); }

__global__ void __launch_bounds__(kBlock) k_scan_sums(const unsigned* __restrict__ data, int64_t count,
                                                      unsigned* __restrict__ sums) {
    __shared__ unsigned red[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    unsigned s = 0;
    for (int i = 0; i < kScanPer; i++) {
        const int64_t idx = base + (int64_t)i * kBlock + threadIdx.x;
        if (idx < count) s += data[idx];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlock) k_scan_tiles(unsigned* __restrict__ data, int64_t count,
                                                       const unsigned* __restrict__ offs) {
    __shared__ unsigned tile[kScanTile + kScanTile / 32];
    __shared__ unsigned part[kBlock];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int i = 0; i < kScanPer; i++) {
        const int j = i * kBlock + t;
        tile[scan_pad(j)] = base + j < count ? data[base + j] : 0u;
    }
    __syncthreads();
    unsigned s = 0;
    for (int i = 0; i < kScanPer; i++) s += tile[scan_pad(t * kScanPer + i)];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        unsigned v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned run = offs[blockIdx.x] + part[t] - s;
    for (int i = 0; i < kScanPer; i++) {
        const int j = scan_pad(t * kScanPer + i);
        const unsigned v = tile[j];
        tile[j] = run;
        run += v;
    }
    __syncthreads();
    for (int i = 0; i < kScanPer; i++) {
        const int j = i * kBlock + t;
        if (base + j < count) data[base + j] = tile[scan_pad(j)];
    }
}

__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
                             int shift, const unsigned* __restrict__ offs, int nblocks) {
    __shared__ unsigned running[256];
    __shared__ unsigned wcnt[kBlock / 64][256];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    running[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int c = 0; c < kRsItems; c++) {
        int64_t idx = base + (int64_t)c * kBlock + tid;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0ull;
        unsigned digit = valid ? (unsigned)((key >> shift) & 255u) : 0u;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            bool bit = (digit >> b) & 1u;
            uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        for (int w = 0; w < kBlock / 64; w++) wcnt[w][tid] = 0u;
        __syncthreads();
        unsigned rank = (unsigned)__popcll(m & lt);
        bool last = valid && ((m >> lane) == 1ull);
        if (last) wcnt[wave][digit] = rank + 1;
        __syncthreads();
        if (valid) {
            unsigned off = running[digit];
            for (int w = 0; w < wave; w++) off += wcnt[w][digit];
            kout[off + rank] = key;
            vout[off + rank] = vin[idx];
        }
        __syncthreads();
        unsigned add = 0;
        for (int w = 0; w < kBlock / 64; w++) add += wcnt[w][tid];
        running[tid] += add;
        __syncthreads();
    }
}

// ---- hierarchy ------------------------------------------------------------
__device__ __forceinline__ int lcp(const uint64_t* __restrict__ k, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((unsigned)(i ^ j));
    return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t* __restrict__ keys, int64_t n, int4* __restrict__ child,
                         int* __restrict__ parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (lcp(keys, n, i, i + 1) - lcp(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = lcp(keys, n, i, i - d);
    int64_t lmax = 2;
    while (lcp(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (lcp(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = lcp(keys, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (lcp(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t g = i + s * d + min(d, 0);
    int left = (min(i, j) == g) ? ~(int)g : (int)g;
    int right = (max(i, j) == g + 1) ? ~(int)(g + 1) : (int)(g + 1);
    child[i] = make_int4(left, right, 0, 0);
    if (left >= 0) parent[left] = (int)i;
    if (right >= 0) parent[right] = (int)i;
}

__global__ void k_depth(const int* __restrict__ parent, const int4* __restrict__ child, int64_t n_int,
                        int* __restrict__ depth, int* __restrict__ maxdepth) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    // walk to the root; the bound and the range check turn a malformed
    // hierarchy into an error flag instead of a runaway loop
    int d = 0;
    int p = (int)i;
    while (p != 0) {
        p = parent[p];
        d++;
        if (p < 0 || p >= n_int || d > 4096) {
            atomicMax(maxdepth, 1 << 30);
            depth[i] = -1;
            return;
        }
    }
    depth[i] = d;
    int4 c = child[i];
    if (c.x < 0 || c.y < 0) atomicMax(maxdepth, d + 1);
    else atomicMax(maxdepth, d);
}

__device__ __forceinline__ void tri_box(const float4* __restrict__ raw, const uint32_t* __restrict__ order,
                                        int slot, float lo[3], float hi[3]) {
    int64_t t = order[slot];
    float4 a = raw[3 * t], b = raw[3 * t + 1], c = raw[3 * t + 2];
    lo[0] = fminf(fminf(a.x, b.x), c.x);
    lo[1] = fminf(fminf(a.y, b.y), c.y);
    lo[2] = fminf(fminf(a.z, b.z), c.z);
    hi[0] = fmaxf(fmaxf(a.x, b.x), c.x);
    hi[1] = fmaxf(fmaxf(a.y, b.y), c.y);
    hi[2] = fmaxf(fmaxf(a.z, b.z), c.z);
}

__device__ __forceinline__ void node_box(const float4* __restrict__ nodes, int c, float lo[3], float hi[3]) {
    float4 q0 = nodes[4 * (int64_t)c], q1 = nodes[4 * (int64_t)c + 1], q2 = nodes[4 * (int64_t)c + 2];
    lo[0] = fminf(q0.x, q1.x);
    hi[0] = fmaxf(q0.y, q1.y);
    lo[1] = fminf(q0.z, q1.z);
    hi[1] = fmaxf(q0.w, q1.w);
    lo[2] = fminf(q2.x, q2.z);
    hi[2] = fmaxf(q2.y, q2.w);
}

__global__ void k_refit_level(const int4* __restrict__ child, const int* __restrict__ depth, int level,
                              int64_t n_int, const float4* __restrict__ raw,
                              const uint32_t* __restrict__ order, float4* __restrict__ nodes) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int || depth[i] != level) return;
    int4 c = child[i];
    float llo[3], lhi[3], rlo[3], rhi[3];
    if (c.x < 0) tri_box(raw, order, ~c.x, llo, lhi);
    else node_box(nodes, c.x, llo, lhi);
    if (c.y < 0) tri_box(raw, order, ~c.y, rlo, rhi);
    else node_box(nodes, c.y, rlo, rhi);
    nodes[4 * i + 0] = make_float4(llo[0], lhi[0], llo[1], lhi[1]);
    nodes[4 * i + 1] = make_float4(rlo[0], rhi[0], rlo[1], rhi[1]);
    nodes[4 * i + 2] = make_float4(llo[2], lhi[2], rlo[2], rhi[2]);
    nodes[4 * i + 3] = make_float4(__int_as_float(c.x), __int_as_float(c.y), 0.0f, 0.0f);
}

// ---- 4-wide collapse -------------------------------------------------------
// A wide node is rooted at a binary node; its children are obtained by
// repeatedly replacing the internal child with the largest box surface area by
// its two children, until there are four children or only leaves.
__device__ __forceinline__ float box_area(const float lo[3], const float hi[3]) {
    float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return dx * dy + dy * dz + dz * dx;
}

__device__ __forceinline__ int wide_children(const int4* __restrict__ child, const float4* __restrict__ nodes, int i,
                                             int refs[4]) {
    int4 c = child[i];
    refs[0] = c.x;
    refs[1] = c.y;
    int cnt = 2;
    while (cnt < 4) {
        int best = -1;
        float bestA = -1.0f;
        for (int j = 0; j < cnt; j++) {
            if (refs[j] >= 0) {
                float lo[3], hi[3];
                node_box(nodes, refs[j], lo, hi);
                float A = box_area(lo, hi);
                if (A > bestA) {
                    bestA = A;
                    best = j;
                }
            }
        }
        if (best < 0) break;
        int4 g = child[refs[best]];
        refs[best] = g.x;
        refs[cnt++] = g.y;
    }
    return cnt;
}

__global__ void k_wide_mark(const int4* __restrict__ child, const float4* __restrict__ nodes,
                            const int* __restrict__ depth, int level, int64_t n_int, int* __restrict__ is_root) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int || depth[i] != level || !is_root[i]) return;
    int refs[4];
    int cnt = wide_children(child, nodes, (int)i, refs);
    for (int j = 0; j < cnt; j++)
        if (refs[j] >= 0) is_root[refs[j]] = 1;
}

__global__ void k_wide_emit(const int4* __restrict__ child, const float4* __restrict__ nodes,
                            const float4* __restrict__ tris, const int* __restrict__ is_root,
                            const unsigned* __restrict__ index4, int64_t n_int, float4* __restrict__ wide) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int || !is_root[i]) return;
    int refs[4];
    int cnt = wide_children(child, nodes, (int)i, refs);
    float lo[4][3], hi[4][3];
    int out[4];
    for (int j = 0; j < 4; j++) {
        if (j >= cnt) {
            // inverted box: no ray ever enters it
            for (int a = 0; a < 3; a++) {
                lo[j][a] = INFINITY;
                hi[j][a] = -INFINITY;
            }
            out[j] = RT_WIDE_EMPTY;
        } else if (refs[j] < 0) {
            int64_t sl = ~refs[j];
            float4 a0 = tris[3 * sl], a1 = tris[3 * sl + 1], a2 = tris[3 * sl + 2];
            lo[j][0] = fminf(fminf(a0.x, a1.x), a2.x);
            lo[j][1] = fminf(fminf(a0.y, a1.y), a2.y);
            lo[j][2] = fminf(fminf(a0.z, a1.z), a2.z);
            hi[j][0] = fmaxf(fmaxf(a0.x, a1.x), a2.x);
            hi[j][1] = fmaxf(fmaxf(a0.y, a1.y), a2.y);
            hi[j][2] = fmaxf(fmaxf(a0.z, a1.z), a2.z);
            out[j] = refs[j];
        } else {
            node_box(nodes, refs[j], lo[j], hi[j]);
            out[j] = (int)index4[refs[j]];
        }
    }
    float4* w = wide + 8 * (int64_t)index4[i];
    for (int a = 0; a < 3; a++) {
        w[2 * a] = make_float4(lo[0][a], lo[1][a], lo[2][a], lo[3][a]);
        w[2 * a + 1] = make_float4(hi[0][a], hi[1][a], hi[2][a], hi[3][a]);
    }
    w[6] = make_float4(__int_as_float(out[0]), __int_as_float(out[1]), __int_as_float(out[2]),
                       __int_as_float(out[3]));
    w[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void k_flags_to_u32(const int* __restrict__ f, unsigned* __restrict__ u, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = (unsigned)f[i];
}

__global__ void k_gather(const float4* __restrict__ raw, const uint32_t* __restrict__ order,
                         const int32_t* __restrict__ M, int64_t n, float4* __restrict__ tris,
                         float4* __restrict__ normals) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t t = order[s];
    float4 a = raw[3 * t], b = raw[3 * t + 1], c = raw[3 * t + 2];
    int32_t m = M[t];
    tris[3 * s + 0] = make_float4(a.x, a.y, a.z, __int_as_float((int)t));
    tris[3 * s + 1] = make_float4(b.x, b.y, b.z, __int_as_float(m));
    tris[3 * s + 2] = make_float4(c.x, c.y, c.z, 0.0f);
    double e1x = (double)b.x - a.x, e1y = (double)b.y - a.y, e1z = (double)b.z - a.z;
    double e2x = (double)c.x - a.x, e2y = (double)c.y - a.y, e2z = (double)c.z - a.z;
    double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    double len = sqrt(nx * nx + ny * ny + nz * nz);
    if (len > 0.0) {
        nx /= len;
        ny /= len;
        nz /= len;
    } else {
        nx = 0.0;
        ny = 0.0;
        nz = 1.0;
    }
    normals[s] = make_float4((float)nx, (float)ny, (float)nz, __int_as_float(m));
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)std::max<int64_t>(1, (n + block - 1) / block); }

// Sort key of lattice index n for the coherent launch order: the chunk
// (M consecutive indices, i.e. a thin band of polar angle) in the high bits,
// the Fibonacci azimuth frac(n (phi_g - 1)) in the low 32 bits.
__global__ void k_order_keys(int64_t N, int64_t M, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint64_t az = ((uint64_t)n * 0x9e3779b97f4a7c16ull) >> 32;
    keys[n] = ((uint64_t)(n / M) << 32) | az;
    vals[n] = (uint32_t)n;
}

__global__ void k_low32(const uint64_t* __restrict__ k, unsigned* __restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (unsigned)(k[i] & 0xffffffffu);
}

// Rotation of every full chunk c of a lattice: the azimuths of the rays
// c M + j are those of j shifted by the (fixed-point) azimuth of c M, so the
// chunk's sorted order starts at the first sorted j whose azimuth is at
// least 2^32 minus that shift.  (Carries from the low 32 bits are ignored:
// the order only needs to be nearly sorted.)
__global__ void k_order_shifts(const TxDesc* __restrict__ txs, int64_t N1, int log2m, const unsigned* __restrict__ az,
                               int* __restrict__ shifts, int64_t max_chunks) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t chunks, base;
    if (txs) {
        chunks = txs[blockIdx.y].n_chunks;
        base = txs[blockIdx.y].shift0;
    } else {
        chunks = N1 >> log2m;
        base = 0;
    }
    if (c >= chunks || c >= max_chunks) return;
    unsigned off = (unsigned)(((uint64_t)(c << log2m) * 0x9e3779b97f4a7c16ull) >> 32);
    unsigned target = 0u - off;
    int lo = 0, hi = 1 << log2m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (az[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    shifts[base + c] = (lo == (1 << log2m)) ? 0 : lo;
}

}  // namespace

// Tile sums needed by scan_exclusive for `count` values.
int64_t scan_sums_len(int64_t count) { return (count + kScanTile - 1) / kScanTile; }

// In-place exclusive scan of `count` values; `sums` holds scan_sums_len(count)
// values of scratch.
void scan_exclusive(unsigned* data, int64_t count, unsigned* sums, hipStream_t st) {
    const int64_t tiles = scan_sums_len(count);
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)tiles), dim3(kBlock), 0, st, data, count, sums);
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, sums, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, st, data, count, sums);
}

// Histogram buffer of the radix sort for n keys: 256 digit counts per tile of
// kRsTile keys, then the scan's tile sums.
int64_t rs_hist_len(int64_t n) {
    const int64_t cells = 256 * ((n + kRsTile - 1) / kRsTile);
    return cells + scan_sums_len(cells);
}

// LSD radix sort of (key, value) pairs on the low `bits` bits of the keys.
// Results end in (k0, v0) when the number of 8-bit passes is even, else in
// (k1, v1); the return value says which (0 or 1).
int rt_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int bits, unsigned* hist,
                  hipStream_t st) {
    const int rs_blocks = (int)((n + kRsTile - 1) / kRsTile);
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    int which = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(rs_blocks), dim3(kBlock), 0, st, ka, n, shift, hist, rs_blocks);
        scan_exclusive(hist, (int64_t)256 * rs_blocks, hist + (int64_t)256 * rs_blocks, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(rs_blocks), dim3(kBlock), 0, st, ka, va, kb, vb, n, shift, hist,
                           rs_blocks);
        std::swap(ka, kb);
        std::swap(va, vb);
        which ^= 1;
    }
    return which;
}

int rt_order_log2m(int64_t N) {
    // wave patches of roughly equal extent in polar and azimuthal angle:
    // a chunk spans 2M/N in z, a wave 2 pi 64/M in azimuth -> M^2 ~ 64 pi N
    double m = std::sqrt(64.0 * 3.14159265358979 * (double)N);
    int l = (int)std::lround(std::log2(std::max(m, 1.0)));
    return std::max(12, std::min(18, l));
}

// Sorted azimuths of j in [0, 2^log2m): key = top 32 bits of j (phi_g - 1)
// in 64-bit fixed point.
rt_status rt_order_table(rt_scene* s, int log2m, hipStream_t st, const rt_scene::OrderTable** out) {
    for (int i = 0; i < s->n_otab; i++)
        if (s->otab[i].log2m == log2m) {
            *out = &s->otab[i];
            return RT_OK;
        }
    if (s->n_otab >= 12) return rt_fail(RT_EINVAL, "launch order: too many chunk sizes");
    const int64_t M = (int64_t)1 << log2m;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    unsigned *hist = nullptr, *az = nullptr;
    const int rs_blocks = (int)((M + kRsTile - 1) / kRsTile);
    bool keep = false;
    auto cleanup = [&]() {
        (void)hipFree(k0);
        (void)hipFree(k1);
        (void)hipFree(v1);
        (void)hipFree(hist);
        if (!keep) {
            (void)hipFree(v0);
            (void)hipFree(az);
        }
    };
    HIPCHK(hipMalloc(&k0, sizeof(uint64_t) * M));
    HIPCHK(hipMalloc(&k1, sizeof(uint64_t) * M));
    HIPCHK(hipMalloc(&v0, sizeof(uint32_t) * M));
    HIPCHK(hipMalloc(&v1, sizeof(uint32_t) * M));
    HIPCHK(hipMalloc(&az, sizeof(unsigned) * M));
    HIPCHK(hipMalloc(&hist, sizeof(unsigned) * (size_t)rs_hist_len(M)));
    hipLaunchKernelGGL(k_order_keys, dim3(grid_for(M, kBlock)), dim3(kBlock), 0, st, M, M, k0, v0);
    int which = rt_radix_sort(k0, v0, k1, v1, M, 32, hist, st);
    if (which) {
        std::swap(v0, v1);
        std::swap(k0, k1);
    }
    hipLaunchKernelGGL(k_low32, dim3(grid_for(M, kBlock)), dim3(kBlock), 0, st, k0, az, M);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    keep = true;
    cleanup();
    rt_scene::OrderTable& t = s->otab[s->n_otab++];
    t.log2m = log2m;
    t.perm = (int*)v0;
    t.az = az;
    s->bytes += sizeof(int) * 2 * M;
    *out = &t;
    return RT_OK;
}

rt_status rt_order_reserve(rt_scene* s, size_t entries, hipStream_t st) {
    if (s->shifts_cap >= entries) return RT_OK;
    (void)hipStreamSynchronize(st);
    (void)hipFree(s->shifts);
    s->shifts = nullptr;
    s->shifts_cap = 0;
    size_t cap = std::max<size_t>(entries, 4096);
    hipError_t e = hipMalloc(&s->shifts, sizeof(int) * cap);
    if (e != hipSuccess) return rt_hip_fail(e, "launch order: shift table");
    s->shifts_cap = cap;
    return RT_OK;
}

void rt_order_shifts_single(const rt_scene::OrderTable* t, int64_t N, int* shifts, hipStream_t st) {
    int64_t chunks = N >> t->log2m;
    if (chunks <= 0) return;
    hipLaunchKernelGGL(k_order_shifts, dim3(grid_for(chunks, kBlock), 1), dim3(kBlock), 0, st,
                       (const TxDesc*)nullptr, N, t->log2m, (const unsigned*)t->az, shifts, chunks);
}

void rt_order_shifts_multi(const rt_scene::OrderTable* t, const TxDesc* txs, int n_tx, int64_t max_chunks,
                           int* shifts, hipStream_t st) {
    if (max_chunks <= 0) return;
    hipLaunchKernelGGL(k_order_shifts, dim3(grid_for(max_chunks, kBlock), n_tx), dim3(kBlock), 0, st, txs,
                       (int64_t)0, t->log2m, (const unsigned*)t->az, shifts, max_chunks);
}

rt_status rt_build_lbvh(rt_scene* s, const float* V, int64_t n_v, const int32_t* F, const int32_t* M,
                        hipStream_t st) {
    const int64_t n = s->n_tri;
    if (n == 0) {
        s->root = -1;
        s->depth = 0;
        return RT_OK;
    }
    // temporaries
    float4 *raw = nullptr, *cen = nullptr;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    unsigned *hist = nullptr, *bounds = nullptr;
    int4* child = nullptr;
    int *parent = nullptr, *depth = nullptr;
    bool keep_keys = false;
    auto cleanup = [&]() {
        (void)hipFree(raw);
        (void)hipFree(cen);
        if (!keep_keys) (void)hipFree(k0);
        (void)hipFree(k1);
        (void)hipFree(v0);
        (void)hipFree(v1);
        (void)hipFree(hist);
        (void)hipFree(bounds);
        (void)hipFree(child);
        (void)hipFree(parent);
        (void)hipFree(depth);
    };
    const int64_t n_int = std::max<int64_t>(0, n - 1);
    const int rs_blocks = (int)((n + kRsTile - 1) / kRsTile);
    HIPCHK(hipMalloc(&raw, sizeof(float4) * 3 * n));
    HIPCHK(hipMalloc(&cen, sizeof(float4) * n));
    HIPCHK(hipMalloc(&k0, sizeof(uint64_t) * n));
    HIPCHK(hipMalloc(&k1, sizeof(uint64_t) * n));
    HIPCHK(hipMalloc(&v0, sizeof(uint32_t) * n));
    HIPCHK(hipMalloc(&v1, sizeof(uint32_t) * n));
    HIPCHK(hipMalloc(&hist, sizeof(unsigned) * (size_t)rs_hist_len(n)));
    HIPCHK(hipMalloc(&bounds, sizeof(unsigned) * 8));
    HIPCHK(hipMalloc(&child, sizeof(int4) * std::max<int64_t>(1, n_int)));
    HIPCHK(hipMalloc(&parent, sizeof(int) * std::max<int64_t>(1, n_int)));
    HIPCHK(hipMalloc(&depth, sizeof(int) * (std::max<int64_t>(1, n_int) + 1)));

    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));

    unsigned hb[8] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u, 0u, 0u};
    HIPCHK(hipMemcpyAsync(bounds, hb, sizeof(hb), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ingest, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, V, n_v, F, M, s->n_mat, n,
                       raw, cen, bounds, bounds + 6);
    HIPCHK(hipGetLastError());
    unsigned hres[8];
    HIPCHK(hipMemcpyAsync(hres, bounds, sizeof(hres), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hres[6] != 0) {
        cleanup();
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::string why;
        if (hres[6] & 1u) why += " vertex index out of range;";
        if (hres[6] & 2u) why += " material id out of range;";
        if (hres[6] & 4u) why += " non-finite vertex coordinate;";
        return rt_fail(RT_EINVAL, "rt_build_scene: invalid mesh:" + why);
    }
    // One scale for all three axes, from the largest extent of the centres'
    // box: the codes then split the longest axis first and keep splitting
    // it until the cells are about as long as the shorter axes are, so a
    // flat scene (2 x 2 km of terrain, tens of metres high) is not cut by
    // height near the root.  On the 1.02 M-triangle scene this takes a third
    // of the node visits off the traversal against a scale per axis.
    float lo[3], hi[3], sc[3];
    float ext_max = 0.0f;
    for (int a = 0; a < 3; a++) {
        lo[a] = ord2f_host(hres[a]);
        hi[a] = ord2f_host(hres[3 + a]);
        ext_max = std::max(ext_max, hi[a] - lo[a]);
    }
    for (int a = 0; a < 3; a++) sc[a] = ext_max > 0.0f ? 2097151.0f / ext_max : 0.0f;
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, cen, n, lo[0], lo[1], lo[2],
                       sc[0], sc[1], sc[2], k0, v0);
    HIPCHK(hipGetLastError());
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int shift = 0; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(rs_blocks), dim3(kBlock), 0, st, ka, n, shift, hist, rs_blocks);
        scan_exclusive(hist, (int64_t)256 * rs_blocks, hist + (int64_t)256 * rs_blocks, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(rs_blocks), dim3(kBlock), 0, st, ka, va, kb, vb, n, shift, hist,
                           rs_blocks);
        HIPCHK(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // after 8 passes the sorted data is back in (k0, v0)
    size_t node_bytes = sizeof(float4) * 4 * (size_t)std::max<int64_t>(1, n_int);
    HIPCHK(hipMalloc(&s->nodes, node_bytes));
    HIPCHK(hipMalloc(&s->tris, sizeof(float4) * 3 * n));
    HIPCHK(hipMalloc(&s->normals, sizeof(float4) * n));
    s->bytes += node_bytes + sizeof(float4) * 4 * n;
    int maxdepth = 0;
    if (n_int > 0) {
        HIPCHK(hipMemsetAsync(parent, 0xff, sizeof(int) * n_int, st));
        hipLaunchKernelGGL(k_karras, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, ka, n, child, parent);
        HIPCHK(hipMemsetAsync(depth + n_int, 0, sizeof(int), st));
        hipLaunchKernelGGL(k_depth, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, parent, child, n_int,
                           depth, depth + n_int);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&maxdepth, depth + n_int, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (maxdepth > 4096) {
            cleanup();
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rt_fail(RT_EDEVICE, "rt_build_scene: LBVH hierarchy is malformed");
        }
        for (int lvl = maxdepth - 1; lvl >= 0; lvl--) {
            hipLaunchKernelGGL(k_refit_level, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, child, depth,
                               lvl, n_int, raw, va, s->nodes);
        }
        HIPCHK(hipGetLastError());
        s->root = 0;
    } else {
        s->root = ~0;   // single triangle: the root is a leaf
        maxdepth = 0;
    }
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, raw, va, M, n, s->tris,
                       s->normals);
    HIPCHK(hipGetLastError());
    if (n_int > 0) {
        // 4-wide collapse: mark wide roots top-down, number them, emit
        int* is_root = (int*)k1;                 // reuse the sort buffers (>= 8 n bytes each)
        unsigned* index4 = (unsigned*)(k1) + n_int;
        HIPCHK(hipMemsetAsync(is_root, 0, sizeof(int) * n_int, st));
        int one = 1;
        HIPCHK(hipMemcpyAsync(is_root, &one, sizeof(int), hipMemcpyHostToDevice, st));
        for (int lvl = 0; lvl < maxdepth; lvl++)
            hipLaunchKernelGGL(k_wide_mark, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, child, s->nodes,
                               depth, lvl, n_int, is_root);
        hipLaunchKernelGGL(k_flags_to_u32, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, is_root, index4,
                           n_int);
        unsigned last_flag = 0, last_index = 0;
        HIPCHK(hipMemcpyAsync(&last_flag, index4 + n_int - 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        // the radix histogram (at least n / 16 values) is free again: it holds the tile sums
        scan_exclusive(index4, n_int, hist, st);
        HIPCHK(hipMemcpyAsync(&last_index, index4 + n_int - 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t n4 = (int64_t)last_index + last_flag;
        // the traversal addresses wide nodes with 32-bit byte offsets; larger
        // trees are traversed as binary trees
        if (n4 < ((int64_t)1 << 25)) {
            HIPCHK(hipMalloc(&s->wide, sizeof(float4) * 8 * n4));
            s->bytes += sizeof(float4) * 8 * n4;
            hipLaunchKernelGGL(k_wide_emit, dim3(grid_for(n_int, kBlock)), dim3(kBlock), 0, st, child, s->nodes,
                               s->tris, is_root, index4, n_int, s->wide);
            HIPCHK(hipGetLastError());
            s->n_wide = n4;
        }
    }
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->build_ms = ms;
    s->depth = maxdepth;
    // the sorted Morton codes stay with the scene (rt_scene_export)
    s->morton = k0;
    s->bytes += sizeof(uint64_t) * n;
    keep_keys = true;
    for (int a = 0; a < 3; a++) {
        s->lo[a] = lo[a];
        s->hi[a] = hi[a];
    }
    cleanup();
    return RT_OK;
}
