// sbr_forward.hip -- persistent SBR radio-map kernel for gfx950.
//
// One lane carries one ray at a time.  A lane whose ray has ended takes the
// next lattice index from a device work queue (one atomic per wavefront,
// shared out with ballot/mbcnt), so wavefronts stay full while ray lengths
// differ.  The work indices are split into contiguous queues with separate
// counters; a wavefront starts on its own queue and moves on to the next once
// that is drained, until it has found every queue drained.  Per traced segment l the lane
//   1. finds the closest hit through the LBVH (short LDS stack, spill to a
//      per-lane global area sized from the tree depth), or by testing every
//      triangle when accel = brute force (validation);
//   2. deposits ||T C_T||^2 * lambda^2 / (4 pi N_S |M_i| |k_z|) into the plane
//      cell it crosses, if any (estimator eq. radio-map-solver-ci-all-2-
//      estimator for specular chains), either with one FP32 atomic or after
//      summing same-cell crossings across the wavefront;
//   3. unless the segment escaped or l = L, reflects specularly and updates
//      the 2x2 field transfer matrix T (eq. fresnel_vac and the bases of
//      eq. fresnel_in_vectors / eq. fresnel_out_vectors).
// The extended variant (template flag EXT) adds, per hit, the single-layer
// slab coefficients, the sampled interaction type (specular or diffuse
// reflection, transmission) with its 1/sqrt(q) weight, and early
// termination by Russian roulette or gain thresholding before the next
// segment; its random draws come from a counter-based Philox4x32-10 stream.
// Ray state (origin, direction, basis, T) stays in VGPRs for the whole ray.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstring>

#include "sbr_common.h"

using namespace rtd;

namespace {

struct FwdArgs {
    const float4* nodes;
    const float4* wide;
    const float4* tris;
    const float4* normals;
    int root;
    int n_tri;
    int n_wide;              // 4-wide nodes (0 when the tree is binary only)
    const float* eps_r;
    const float* sigma;
    TxDesc tx;
    PlaneDesc pl;
    int64_t ray_begin;
    int64_t n_work;
    int L;
    float t_min;
    int deposit;       // 1 atomic, 2 wave
    int npol;
    float* map;
    int64_t map_stride;
    float4* tape_seg;
    int* tape_nseg;
    int64_t tape_n;
    int32_t* hits;
    int32_t* cells;
    float* weights;
    unsigned long long* stats;
    unsigned long long* counter;   // RT_QUEUES heads, RT_QUEUE_STRIDE apart
    int nq;                        // queues in use (1..RT_QUEUES)
    int qrem;                      // queues q < qrem hold qper + 1 work indices, the others qper
    unsigned long long qper;
    int claim;                     // work indices claimed per queue atomic (>= 64)
    // early termination (kernel variant EXT): before segments l >= rr_depth
    int rr_depth;
    float rr_p_max;                // Russian roulette, 0 = off
    float gain_threshold;          // gain thresholding, 0 = off
    unsigned seed;
    float gain_scale;              // lambda^2 / (16 pi^2): path gain = gain_scale ||E||^2 / r^2
    float inv_kappa;               // 1 / tx.kappa: |alpha|^2 = kap * inv_kappa
    // finite-thickness walls and refraction (kernel variant EXT)
    const float* thickness;        // slab thickness per material (m), or null
    const float* scattering;       // scattering coefficient S per material, or null (no diffuse)
    const float* xpd;              // cross-polarisation share K_x per material
    const float* pattern;          // [n_mat][4] scattering pattern, or null (Lambertian)
    int refraction;                // 1: sample reflection or transmission at every hit
    float k0;                      // 2 pi / lambda
    int* spill;
    int64_t spill_stride;
    int spill_depth;
    int tape_groups;         // float4 records per segment on the tape (4, or 2 = geometry only)
    const int* operm;        // coherent launch order: sorted chunk order, or null
    const int* oshift;       // rotation of every full chunk
    int olog2m;              // chunk size 2^olog2m
    int64_t ray_end;
    int refill;              // refill a wavefront once this many lanes are idle
    // several transmitters (MODE_MULTI, MODE_GEOM): device tables
    const TxDesc* txs;       // ordered largest budget first
    const int64_t* prefix;   // [n_tx + 1] exclusive prefix of the budgets
    const int32_t* slots;    // output slot of each ordered transmitter
    int n_tx;
    int64_t slot_stride;     // floats between the maps of consecutive slots
};

// Kernel modes: one transmitter; several transmitters with one material set
// (deposits into per-transmitter maps); several transmitters, geometry only
// (records hit slots, cells, directions and bases for a later field pass).
enum { MODE_SINGLE = 0, MODE_MULTI = 1, MODE_GEOM = 2 };

// Wavefront deposit: same-cell groups summed before the atomics (4 measured
// best against 1, 2 and no limit on the Manhattan and rooftop workloads).
constexpr int kDepositGroups = 4;

// Index of the transmitter whose ray range holds global ray g.
__device__ __forceinline__ int find_tx(const int64_t* __restrict__ prefix, int n_tx, int64_t g) {
    int lo = 0, hi = n_tx;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Value of lane 0 (the caller runs with every lane active), in scalar registers.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffu));
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long v, int src) {
    unsigned lo = __shfl((unsigned)(v & 0xffffffffu), src);
    unsigned hi = __shfl((unsigned)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Per-lane traversal stack: the first RT_STACK_LDS entries {node, entry
// distance} live in LDS, laid out [entry][lane] (8 bytes each, so a
// wavefront's pushes are contiguous); deeper entries (node only) go to a
// per-lane global spill area.  `top` is the LDS slot of entry sp while
// sp <= RT_STACK_LDS.
struct TravStack {
    int2* top;
    int stride;   // lanes per workgroup
    int sp;
};

__device__ __forceinline__ void push_entry(const FwdArgs& a, TravStack& st, int64_t gtid, int ref, float key,
                                           unsigned& overflow) {
    if (st.sp < RT_STACK_LDS) {
        *st.top = make_int2(ref, __float_as_int(key));
        st.top += st.stride;
    } else if (st.sp - RT_STACK_LDS < a.spill_depth) {
        a.spill[(st.sp - RT_STACK_LDS) * a.spill_stride + gtid] = ref;
    } else {
        overflow++;   // cannot happen: the spill area is sized from the tree depth
        return;
    }
    st.sp++;
}

// Pop until an entry whose box may still hold a hit closer than `lim`.
__device__ __forceinline__ bool pop_entry(const FwdArgs& a, TravStack& st, int64_t gtid, float lim, int& node) {
    while (st.sp > 0) {
        st.sp--;
        if (st.sp < RT_STACK_LDS) {
            st.top -= st.stride;
            const int2 e = *st.top;
            if (__int_as_float(e.y) <= lim) {
                node = e.x;
                return true;
            }
        } else {
            node = a.spill[(st.sp - RT_STACK_LDS) * a.spill_stride + gtid];
            return true;
        }
    }
    return false;
}

// Closest hit of ray r among all triangles but `last` (a slot).  Ties in t go
// to the smallest original triangle id.  Returns the slot or -1.
template <bool BRUTE, bool WIDE>
__device__ __forceinline__ int closest_hit(const FwdArgs& a, const Ray& r, int last, float& t_best, int& id_best,
                                           int2* __restrict__ stk, int lstride, int64_t gtid,
                                           unsigned& n_nodes, unsigned& n_tris, unsigned& overflow) {
    t_best = INFINITY;
    id_best = 0x7fffffff;
    int slot_best = -1;
    // cull limit: t_best times the slack, kept finite so that the INFINITY
    // keys of missed, leaf and empty slots never pass it, also before the
    // first hit; updated with t_best
    float lim = FLT_MAX;
    // canonical once, so that the min/max below need no per-use quieting
    const float tmin = __builtin_canonicalizef(a.t_min);
    if (a.n_tri == 0) return -1;
    auto test = [&](int s) {
        if (s == last) return;
        float4 v0 = a.tris[3 * (int64_t)s], v1 = a.tris[3 * (int64_t)s + 1], v2 = a.tris[3 * (int64_t)s + 2];
        n_tris++;
        float t = tri_hit(r, v0, v1, v2, tmin);
        if (t > 0.0f) {
            int id = __float_as_int(v0.w);
            if (t < t_best || (t == t_best && id < id_best)) {
                t_best = t;
                id_best = id;
                slot_best = s;
                lim = fminf(t * kBoxSlack, FLT_MAX);
            }
        }
    };
    if (BRUTE) {
        for (int s = 0; s < a.n_tri; s++) test(s);
        return slot_best;
    }
    if (a.root < 0) {
        test(~a.root);
        return slot_best;
    }
    TravStack st{stk, lstride, 0};
    if (WIDE) {
        // 4-wide traversal: four slab tests per node fetch (empty child slots
        // hold inverted boxes and never hit); leaf children are tested at once,
        // internal hits are sorted by entry distance, the nearest is descended
        // and the others are pushed farthest first
        int node = 0;
        const __amdgpu_buffer_rsrc_t rs = wide_rsrc(a.wide, a.n_wide);
        for (int guard = 0; guard < a.n_tri; guard++) {
            n_nodes++;
            bool h[4];
            float te[4];
            int ref[4];
            box4(r, rs, (unsigned)node << 7, tmin, lim, h, te, ref);
            float key[4];
            unsigned leaves = 0;
#pragma unroll
            for (int c = 0; c < 4; c++) {
                key[c] = (h[c] && ref[c] >= 0) ? te[c] : INFINITY;
                leaves |= (h[c] && ref[c] < 0) ? 1u << c : 0u;
            }
            // one triangle-test body for the whole wavefront: it runs as many
            // times as the lane with the most leaf hits needs
            while (leaves) {
                const int c = __builtin_ctz(leaves);
                leaves &= leaves - 1u;
                // select by the bits of c (selects, not a branch per slot)
                const int r01 = (c & 1) ? ref[1] : ref[0];
                const int r23 = (c & 1) ? ref[3] : ref[2];
                test(~((c & 2) ? r23 : r01));
            }
            // sort the four (key, ref) pairs by key (misses sort last)
#define RT_CSWAP(i, j)                                  \
    if (key[j] < key[i]) {                              \
        float tk = key[i];                              \
        key[i] = key[j];                                \
        key[j] = tk;                                    \
        int tr = ref[i];                                \
        ref[i] = ref[j];                                \
        ref[j] = tr;                                    \
    }
            RT_CSWAP(0, 1) RT_CSWAP(2, 3) RT_CSWAP(0, 2) RT_CSWAP(1, 3) RT_CSWAP(1, 2)
#undef RT_CSWAP
            // children entered beyond the closest hit so far are dropped (the
            // same outcome as a box test with the new bound)
            if (key[0] <= lim) {
#pragma unroll
                for (int c = 3; c >= 1; c--)
                    if (key[c] <= lim) push_entry(a, st, gtid, ref[c], key[c], overflow);
                node = ref[0];
            } else if (!pop_entry(a, st, gtid, lim, node)) {
                break;
            }
        }
        return slot_best;
    }
    int node = a.root;
    // every internal node is visited at most once per query; the bound only
    // guards against a malformed tree
    for (int guard = 0; guard < a.n_tri; guard++) {
        if ((unsigned)node >= (unsigned)(a.n_tri - 1)) {
            overflow++;
            break;
        }
        n_nodes++;
        const float4* q = a.nodes + 4 * (int64_t)node;
        float4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
        bool hL, hR;
        float tL, tR;
        box2(r, q0, q1, q2, tmin, t_best * kBoxSlack, hL, hR, tL, tR);
        int cl = __float_as_int(q3.x), cr = __float_as_int(q3.y);
        if (hL && cl < 0) {
            test(~cl);
            hL = false;
        }
        if (hR && cr < 0) {
            test(~cr);
            hR = false;
        }
        if (hL && hR) {
            // the far child's entry distance goes with it, so that it can be
            // dropped at pop time without fetching its node
            const bool lnear = tL <= tR;
            push_entry(a, st, gtid, lnear ? cr : cl, lnear ? tR : tL, overflow);
            node = lnear ? cl : cr;
        } else if (hL) {
            node = cl;
        } else if (hR) {
            node = cr;
        } else if (!pop_entry(a, st, gtid, t_best * kBoxSlack, node)) {
            break;
        }
    }
    return slot_best;
}

template <bool BRUTE, int MODE, bool WIDE, bool EXT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_forward(const FwdArgs a) {
    extern __shared__ int2 s_stack[];
    const int lstride = blockDim.x;
    int2* stk = s_stack + threadIdx.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int L = a.L;
    const int stride = L + 1;
    const int W = a.pl.W, H = a.pl.H;

    unsigned st_seg = 0, st_cross = 0, st_nodes = 0, st_tris = 0, st_over = 0;

    bool active = false;
    bool exhausted = false;
    // this wavefront's first queue (held in scalar registers)
    int q = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % a.nq));
    int drained = 0;                   // queues found drained so far
    const unsigned long long claim = (unsigned long long)a.claim;   // work indices per atomic
    unsigned long long res_b = 0, res_e = 0;                         // claimed, not yet started
    int64_t rid = 0;          // ray index relative to ray_begin
    int l = 0;
    int last = -1;
    float3 o = f3(0, 0, 0), k = f3(0, 0, 0), es = f3(0, 0, 0);
    cf Ta = {1, 0}, Tb = {0, 0}, Tc = {0, 0}, Td = {1, 0};
    float c0t = 0.f, c0p = 0.f, c1t = 0.f, c1p = 0.f;   // C_T per polarisation
    float kap = a.tx.kappa;   // lambda^2 / (4 pi N_S |M|) of the lane's transmitter
    float rlen = 0.0f;        // unfolded length to the last interaction (early termination only)
    float* mapb = a.map;      // map of the lane's transmitter
    // several transmitters: lattice index of the lane's ray within its
    // transmitter (the counter of its random streams, as in a single call)
    // and 1 / kappa of that transmitter
    int64_t nlat = 0;
    float ikap = a.inv_kappa;
    int tslot = 0;            // output slot of the lane's transmitter (several transmitters)

    while (true) {
        // ---- refill lanes without a ray: from this wavefront's reservoir of
        // claimed work indices, claiming a new batch from the queues when the
        // reservoir cannot cover every idle lane
        if (!exhausted || res_b < res_e) {
            unsigned long long need = __ballot(!active);
            if (need && (__popcll(need) >= a.refill || need == ~0ull)) {
                const unsigned cnt = (unsigned)__popcll(need);
                // wave-uniform: every value below is the same on all lanes
                unsigned long long b1 = res_b, e1 = res_e, b2 = 0, e2 = 0;
                if (e1 - b1 < cnt && !exhausted) {
                    while (true) {
                        // queue q holds work indices [qb, qe): per or per + 1 of them
                        const unsigned long long qb = (unsigned long long)q * a.qper + (unsigned)min(q, a.qrem);
                        const unsigned long long qn = a.qper + (q < a.qrem ? 1ull : 0ull);
                        unsigned long long b = 0;
                        if (lane == 0) b = atomicAdd(a.counter + q * RT_QUEUE_STRIDE, claim);
                        b = uniform_u64(b);
                        const bool got = b < qn;
                        if (got) {
                            b2 = qb + b;
                            e2 = qb + min(qn, b + claim);
                        }
                        if (got && b + claim >= qn) {
                            // this claim drained queue q (exactly one claim per queue does)
                            if (lane == 0) atomicAdd(a.counter + RT_QUEUES * RT_QUEUE_STRIDE, 1ull);
                        }
                        if (!got) {
                            // drained earlier: stop once every queue is, else try the next
                            unsigned long long nd = 0;
                            if (lane == 0)
                                nd = __hip_atomic_load(a.counter + RT_QUEUES * RT_QUEUE_STRIDE, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                            nd = uniform_u64(nd);
                            if (nd >= (unsigned long long)a.nq || ++drained >= a.nq) exhausted = true;
                        }
                        if (!got || b + claim >= qn) q = q + 1 == a.nq ? 0 : q + 1;
                        if (got || exhausted) break;
                    }
                }
                // idle lanes take the reservoir first, then the new batch
                const unsigned long long n1 = e1 - b1;
                const unsigned long long take1 = min((unsigned long long)cnt, n1);
                const unsigned long long take2 = min((unsigned long long)cnt - take1, e2 - b2);
                res_b = take1 < n1 ? b1 + take1 : b2 + take2;
                res_e = take1 < n1 ? e1 : e2;
                if (!active) {
                    const unsigned long long rank = (unsigned long long)__popcll(need & lt);
                    const bool mine = rank < take1 + take2;
                    const unsigned long long my = rank < take1 ? b1 + rank : b2 + (rank - take1);
                    if (mine) {
                        rid = (int64_t)my;
                        int64_t n;
                        TxDesc td;
                        const int64_t M = (int64_t)1 << a.olog2m;
                        if (MODE == MODE_SINGLE) {
                            n = a.ray_begin + rid;
                            if (a.operm) {
                                // permuted only inside full chunks that the range covers
                                int64_t c = n >> a.olog2m, c0 = c << a.olog2m;
                                if (c < (a.tx.n_rays >> a.olog2m) && c0 >= a.ray_begin && c0 + M <= a.ray_end)
                                    n = c0 + a.operm[((n - c0) + a.oshift[c]) & (M - 1)];
                            }
                            rid = n - a.ray_begin;   // records stay indexed by lattice index
                            td = a.tx;
                        } else {
                            int t = find_tx(a.prefix, a.n_tx, rid);
                            n = rid - a.prefix[t];
                            td = a.txs[t];
                            if (a.operm && (n >> a.olog2m) < td.n_chunks) {
                                int64_t c = n >> a.olog2m, c0 = c << a.olog2m;
                                n = c0 + a.operm[((n - c0) + a.oshift[td.shift0 + c]) & (M - 1)];
                                // the geometry tape stays in launch order (a
                                // wavefront of the field pass then reads
                                // consecutive records of nearby directions)
                                if (MODE != MODE_GEOM) rid = a.prefix[t] + n;
                            }
                            kap = td.kappa;
                            mapb = a.map + (int64_t)a.slots[t] * a.slot_stride;
                            nlat = n;
                            ikap = 1.0f / td.kappa;
                            tslot = a.slots[t];
                        }
                        Launch Lr = fib_launch(n, td.n_rays);
                        if (MODE != MODE_GEOM) {
                            tx_pattern<float>(Lr, td, td.pol == 1 ? 1 : 0, c0t, c0p);
                            if (a.npol == 2) tx_pattern<float>(Lr, td, 1, c1t, c1p);
                            // a transmit array scales the ray's field by alpha
                            // and its weights by |alpha|^2
                            kap = td.kappa;
                            if (td.n_ant > 0) kap *= array_gain(Lr, td);
                        }
                        k = f3((float)Lr.kx, (float)Lr.ky, (float)Lr.kz);
                        es = f3((float)Lr.tx, (float)Lr.ty, (float)Lr.tz);
                        o = f3(td.pos[0], td.pos[1], td.pos[2]);
                        Ta = cf{1, 0};
                        Tb = cf{0, 0};
                        Tc = cf{0, 0};
                        Td = cf{1, 0};
                        l = 0;
                        rlen = 0.0f;
                        last = -1;
                        active = true;
                        if (a.hits) {
                            for (int j = 0; j < stride; j++) a.hits[rid * stride + j] = -2;
                        }
                        if (a.cells) {
                            for (int j = 0; j < stride; j++) a.cells[rid * stride + j] = -1;
                        }
                        if (a.weights) {
                            for (int j = 0; j < stride; j++) a.weights[rid * stride + j] = 0.0f;
                        }
                    }
                }
            }
        }
        if (__ballot(active) == 0ull) break;

        // ---- closest hit of the current segment
        int slot = -1, hit_id = -1, cell = -1;
        float t_hit = INFINITY;
        float w0 = 0.f, w1 = 0.f;
        if (active) {
            Ray r;
            r.ox = o.x;
            r.oy = o.y;
            r.oz = o.z;
            r.dx = k.x;
            r.dy = k.y;
            r.dz = k.z;
            ray_setup(r);
            int idb;
            slot = closest_hit<BRUTE, WIDE>(a, r, last, t_hit, idb, stk, lstride, gtid, st_nodes,
                                            st_tris, st_over);
            hit_id = slot >= 0 ? idb : -1;
            st_seg++;
            // ---- plane crossing of this segment
            if (k.z != 0.0f) {
                float tm = (a.pl.z - o.z) * __builtin_amdgcn_rcpf(k.z);
                if (tm > 0.0f && tm < t_hit) {
                    float x = o.x + tm * k.x, y = o.y + tm * k.y;
                    float fx = (x - a.pl.x0) * a.pl.inv_dx, fy = (y - a.pl.y0) * a.pl.inv_dy;
                    if (fx >= 0.0f && fy >= 0.0f && fx < (float)W && fy < (float)H) {
                        int i = min((int)fx, W - 1), j = min((int)fy, H - 1);
                        cell = j * W + i;
                        st_cross++;
                    }
                }
                if (MODE != MODE_GEOM && cell >= 0) {
                        float g = kap * __builtin_amdgcn_rcpf(fabsf(k.z));
                        cf e0 = cadd(cscale(Ta, c0t), cscale(Tb, c0p));
                        cf e1 = cadd(cscale(Tc, c0t), cscale(Td, c0p));
                        w0 = g * (cabs2(e0) + cabs2(e1));
                        if (a.npol == 2) {
                            cf f0 = cadd(cscale(Ta, c1t), cscale(Tb, c1p));
                            cf f1 = cadd(cscale(Tc, c1t), cscale(Td, c1p));
                            w1 = g * (cabs2(f0) + cabs2(f1));
                        }
                }
            }
            if (a.hits) a.hits[rid * stride + l] = hit_id;
            if (a.cells) a.cells[rid * stride + l] = cell;
            if (a.weights) a.weights[rid * stride + l] = w0;
            if (a.tape_seg) {
                const int64_t tn = a.tape_n;
                float4* ts = a.tape_seg + (int64_t)l * a.tape_groups * tn + rid;
                ts[0] = make_float4(k.x, k.y, k.z, __int_as_float(slot));
                ts[tn] = make_float4(es.x, es.y, es.z, __int_as_float(cell));
                if (MODE != MODE_GEOM) {
                    ts[2 * tn] = make_float4(Ta.re, Ta.im, Tb.re, Tb.im);
                    ts[3 * tn] = make_float4(Tc.re, Tc.im, Td.re, Td.im);
                }
            }
        }

        // ---- deposit (all lanes reconverged here)
        if (MODE == MODE_GEOM) {
            // fields are computed later, per material sample
        } else if (a.deposit == 2) {
            // at most kDepositGroups same-cell groups are summed across the
            // wavefront; lanes left over add their own crossings (crossings
            // scattered over many cells would otherwise cost one wavefront
            // reduction per cell)
            unsigned long long pend = __ballot(cell >= 0);
            bool done = cell < 0;
            int groups = 0;
            while (pend) {
                if (groups == kDepositGroups) {
                    if (!done) {
                        unsafeAtomicAdd(mapb + cell, w0);
                        if (a.npol == 2) unsafeAtomicAdd(mapb + a.map_stride + cell, w1);
                    }
                    break;
                }
                groups++;
                int leader = __ffsll((long long)pend) - 1;
                int lc = __shfl(cell, leader);
                bool mine = !done && cell == lc;
                if (MODE == MODE_MULTI) {
                    // lanes of other transmitters deposit into other maps
                    const int ls = __shfl(tslot, leader);
                    mine = mine && tslot == ls;
                }
                unsigned long long grp = __ballot(mine);
                float v0 = wave_sum(mine ? w0 : 0.0f);
                float v1 = 0.0f;
                if (a.npol == 2) v1 = wave_sum(mine ? w1 : 0.0f);
                if (lane == leader) {
                    unsafeAtomicAdd(mapb + lc, v0);
                    if (a.npol == 2) unsafeAtomicAdd(mapb + a.map_stride + lc, v1);
                }
                if (mine) done = true;
                pend &= ~grp;
            }
        } else if (cell >= 0) {
            unsafeAtomicAdd(mapb + cell, w0);
            if (a.npol == 2) unsafeAtomicAdd(mapb + a.map_stride + cell, w1);
        }

        // ---- reflect, or end the ray
        if (active) {
            if (slot < 0 || l == L) {
                if (a.tape_nseg) a.tape_nseg[rid] = l + 1;
                active = false;
            } else {
                float4 nm = a.normals[slot];
                int mat = __float_as_int(nm.w);
                Bounce b = bounce_geometry(k, es, f3(nm.x, nm.y, nm.z));
                int kind = 0;          // 0 specular reflection, 1 diffuse reflection, 2 transmission
                float3 knew = b.kr, esnew = b.es_new;
                if (MODE != MODE_GEOM) {
                    cf eta = cf{a.eps_r[mat], -a.sigma[mat] * a.pl.inv_eps0_omega};
                    Fresnel F = fresnel<false>(b.c, eta);
                    cf cperp = F.rperp, cpar = F.rpar;
                    float qs = 1.0f, s2 = 0.0f;
                    if (EXT) {
                        // single-layer slab: r and t from r' and x = exp(-j q)
                        cf tperp = cf{0.0f, 0.0f}, tpar = cf{0.0f, 0.0f};
                        if (a.thickness) slab(F, a.k0 * a.thickness[mat], tperp, tpar);
                        cperp = F.rperp;
                        cpar = F.rpar;
                        const float Sm = a.scattering ? a.scattering[mat] : 0.0f;
                        if (a.refraction || Sm > 0.0f) {
                            // interaction shares with A = |r|^2, B = |t|^2 (0
                            // without refraction): q(R) = R^2 A/(A+B),
                            // q(S) = S^2 A/(A+B), q(T) = B/(A+B); the sampled
                            // branch carries 1/sqrt(q)
                            const float ar = cabs2(F.rperp) + cabs2(F.rpar);
                            const float at = a.refraction ? cabs2(tperp) + cabs2(tpar) : 0.0f;
                            const float tot = ar + at;
                            const float fa = tot > 0.0f ? ar / tot : 1.0f;
                            s2 = Sm * Sm;
                            const float qr = (1.0f - s2) * fa;
                            qs = s2 * fa;
                            const float u = philox_uniform(a.seed, MODE == MODE_SINGLE ? a.ray_begin + rid : nlat, l, 1u);
                            kind = u < qr ? 0 : (u < qr + qs ? 1 : 2);
                            if (kind != 1) {
                                const float q = kind == 0 ? qr : (tot > 0.0f ? at / tot : 0.0f);
                                // specular share R = sqrt(1 - S^2) (eq. R)
                                const float sc = __builtin_amdgcn_rsqf(q) * (kind == 0 ? sqrtf(1.0f - s2) : 1.0f);
                                cperp = cscale(kind == 2 ? tperp : F.rperp, sc);
                                cpar = cscale(kind == 2 ? tpar : F.rpar, sc);
                                if (kind == 2) knew = k;
                            }
                        }
                    }
                    if (EXT && kind == 1) {
                        // diffuse reflection (Lambertian): direction drawn over
                        // the hemisphere of the incident side, field scaled by
                        // sqrt(2 cos(theta_s) S^2 Gamma^2 / q(S)) and mixed by
                        // the cross-polarisation matrix with random phases, in
                        // the theta/phi bases of the incident and new direction
                        const cf e0 = cadd(cscale(Ta, c0t), cscale(Tb, c0p));
                        const cf e1 = cadd(cscale(Tc, c0t), cscale(Td, c0p));
                        const cf ap = cadd(cscale(e0, b.w00), cscale(e1, b.w01));
                        const cf al = cadd(cscale(e0, b.w10), cscale(e1, b.w11));
                        const float en2 = cabs2(e0) + cabs2(e1);
                        const float g2 = en2 > 0.0f ? (cabs2(cmul(F.rperp, ap)) + cabs2(cmul(F.rpar, al))) / en2 : 0.0f;
                        const uint4 w = philox4(a.seed, MODE == MODE_SINGLE ? a.ray_begin + rid : nlat, l, 2u);
                        const float cs = word_uniform(w.x), ss = sqrtf(fmaxf(0.0f, 1.0f - cs * cs));
                        float sph, cph, s1, c1, s2p, c2p;
                        sincospif(2.0f * word_uniform(w.y), &sph, &cph);
                        sincospif(2.0f * word_uniform(w.z), &s1, &c1);
                        sincospif(2.0f * word_uniform(w.w), &s2p, &c2p);
                        float3 n = f3(nm.x, nm.y, nm.z);
                        if (dot3(k, n) > 0.0f) n = n * -1.0f;
                        knew = diffuse_direction(n, cs, ss, cph, sph);
                        float3 thi, phi_i, phs;
                        sph_basis(k, thi, phi_i);
                        sph_basis(knew, esnew, phs);
                        const float3 ep = cross3(k, es);
                        const float p00 = dot3(thi, es), p01 = dot3(thi, ep);
                        const float p10 = dot3(phi_i, es), p11 = dot3(phi_i, ep);
                        const float K = a.xpd[mat], sk = sqrtf(K), ck = sqrtf(1.0f - K);
                        const float fw = scatter_weight(a.pattern ? a.pattern + 4 * mat : nullptr, b.c, cs, k, knew, b.kr);
                        const float sc = sqrtf(fw * s2 * g2) * __builtin_amdgcn_rsqf(qs);
                        const float a0 = ck * p00 - sk * p10, a1 = ck * p01 - sk * p11;   // theta row
                        const float b0 = sk * p00 + ck * p10, b1 = sk * p01 + ck * p11;   // phi row
                        const cf x1 = cf{c1 * sc, s1 * sc}, x2 = cf{c2p * sc, s2p * sc};
                        const cf na = cmul(x1, cadd(cscale(Ta, a0), cscale(Tc, a1)));
                        const cf nb = cmul(x1, cadd(cscale(Tb, a0), cscale(Td, a1)));
                        const cf nc = cmul(x2, cadd(cscale(Ta, b0), cscale(Tc, b1)));
                        const cf nd = cmul(x2, cadd(cscale(Tb, b0), cscale(Td, b1)));
                        Ta = na;
                        Tb = nb;
                        Tc = nc;
                        Td = nd;
                    } else {
                        // T <- diag(c_perp, -c_par) W T: the new basis is
                        // (e_perp, k' x e_perp), whose second vector is -e_par
                        // of the outgoing wave for both k' = k_r and k' = k
                        cf na = cadd(cscale(Ta, b.w00), cscale(Tc, b.w01));
                        cf nb = cadd(cscale(Tb, b.w00), cscale(Td, b.w01));
                        cf nc = cadd(cscale(Ta, b.w10), cscale(Tc, b.w11));
                        cf nd = cadd(cscale(Tb, b.w10), cscale(Td, b.w11));
                        Ta = cmul(cperp, na);
                        Tb = cmul(cperp, nb);
                        cf mr = cf{-cpar.re, -cpar.im};
                        Tc = cmul(mr, nc);
                        Td = cmul(mr, nd);
                    }
                }
                o = o + k * t_hit;
                k = knew;
                es = esnew;
                last = slot;
                l++;
                if (EXT) rlen = kind == 1 ? 0.0f : rlen + t_hit;   // a diffuse point starts a new tube
                if (EXT && l >= a.rr_depth && (a.rr_p_max > 0.0f || a.gain_threshold > 0.0f)) {
                    // early termination before segment l: the distance-normalised
                    // gain ||T C||^2 of polarisation 0 (times |alpha|^2)
                    const cf e0 = cadd(cscale(Ta, c0t), cscale(Tb, c0p));
                    const cf e1 = cadd(cscale(Tc, c0t), cscale(Td, c0p));
                    const float gn = (cabs2(e0) + cabs2(e1)) * (kap * (MODE == MODE_SINGLE ? a.inv_kappa : ikap));
                    bool drop = false;
                    if (a.gain_threshold > 0.0f && rlen > 0.0f)
                        drop = a.gain_scale * gn * __builtin_amdgcn_rcpf(rlen * rlen) < a.gain_threshold;
                    if (!drop && a.rr_p_max > 0.0f) {
                        const float p = fminf(gn, a.rr_p_max);
                        if (philox_uniform(a.seed, MODE == MODE_SINGLE ? a.ray_begin + rid : nlat, l, 0u) < p) {
                            const float sc = __builtin_amdgcn_rsqf(p);   // survivors carry 1/sqrt(p)
                            Ta = cscale(Ta, sc);
                            Tb = cscale(Tb, sc);
                            Tc = cscale(Tc, sc);
                            Td = cscale(Td, sc);
                        } else {
                            drop = true;
                        }
                    }
                    if (drop) {
                        active = false;
                        if (a.tape_nseg) a.tape_nseg[rid] = l;   // segments 0..l-1 were traced
                    }
                }
            }
        }
    }

    if (a.stats) {
        unsigned long long v[5] = {st_seg, st_cross, st_nodes, st_tris, st_over};
        for (int i = 0; i < 5; i++) {
            unsigned long long s = v[i];
            for (int off = 32; off >= 1; off >>= 1) {
                unsigned lo = __shfl_xor((unsigned)(s & 0xffffffffu), off);
                unsigned hi = __shfl_xor((unsigned)(s >> 32), off);
                s += ((unsigned long long)hi << 32) | lo;
            }
            if (lane == 0 && s) atomicAdd(a.stats + i, s);
        }
    }
}

// Zero the map (unless accumulating) and reset the work-queue heads and the
// drained count (launched with at least two 256-thread blocks, so that the
// grid has more than RT_QUEUES threads).  A kernel,
// not a memset, so that the whole call can be captured in a HIP graph.
__global__ void k_prepare(float* __restrict__ map, int64_t n, unsigned long long* __restrict__ counter) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= RT_QUEUES) counter[i * RT_QUEUE_STRIDE] = 0ull;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) map[i] = 0.0f;
}

}  // namespace

int rt_persistent_blocks(int block, int device) {
    static int cu[64] = {0};
    int dev = device < 64 ? device : 0;
    if (!cu[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c <= 0) c = 256;
        cu[dev] = c;
    }
    // enough resident waves per CU to hide traversal latency
    int waves_per_cu = 32;
    int blocks_per_cu = std::max(1, waves_per_cu * 64 / block);
    return cu[dev] * blocks_per_cu;
}

static void base_args(FwdArgs& a, const rt_scene* s, int block, const float* eps_r, const float* sigma,
                      const PlaneDesc& pl, int L, float t_min) {
    memset(&a, 0, sizeof(a));
    a.nodes = s->nodes;
    a.wide = s->wide;
    a.n_wide = (int)s->n_wide;
    a.tris = s->tris;
    a.normals = s->normals;
    a.root = s->root;
    a.n_tri = (int)s->n_tri;
    a.eps_r = eps_r;
    a.sigma = sigma;
    a.pl = pl;
    a.L = L;
    a.t_min = t_min;
    a.counter = s->counters;
    a.spill = s->spill;
    a.tape_groups = 4;
    a.npol = 1;
    a.refill = 1;
}

static rt_status size_spill(FwdArgs& a, const rt_scene* s, int block, int* blocks_out) {
    // persistent grid, but no more workgroups than give each lane about four rays
    int blocks = rt_persistent_blocks(block, s->device);
    blocks = (int)std::min<int64_t>(blocks, std::max<int64_t>(256, (a.n_work + 4LL * block - 1) / (4LL * block)));
    int64_t threads = (int64_t)blocks * block;
    // a wide traversal pushes up to 3 entries per wide level (= 2 binary levels)
    int64_t need_depth = std::max<int64_t>(0, rt_stack_need(s) - RT_STACK_LDS);
    if ((int64_t)s->spill_entries < need_depth * threads)
        return rt_fail(RT_EOVERFLOW, "traversal spill area too small for this launch");
    a.spill_stride = threads;
    a.spill_depth = (int)need_depth;
    *blocks_out = blocks;
    return RT_OK;
}

template <int MODE>
static void launch_mode(const FwdArgs& args, int accel, bool wide, int blocks, int block, hipStream_t st,
                        bool ext = false) {
    FwdArgs a = args;
    // about 4096 work items per queue, at most RT_QUEUES queues
    a.nq = (int)std::max<int64_t>(1, std::min<int64_t>(RT_QUEUES, a.n_work / 4096));
    if (const char* env = getenv("RTMAP_QUEUES"))
        a.nq = std::max(1, std::min(RT_QUEUES, atoi(env)));
    a.qper = (unsigned long long)a.n_work / (unsigned long long)a.nq;
    a.qrem = (int)((unsigned long long)a.n_work % (unsigned long long)a.nq);
    // claims small enough that every wavefront makes about 16 of them (a
    // wavefront runs its claimed rays one after another, so large claims
    // lengthen the tail), large enough to keep queue atomics rare; whole
    // multiples of the wavefront, so that a refill stays on one stretch of the
    // launch order
    a.claim = 64 * (int)std::max<int64_t>(1, std::min<int64_t>(4, a.n_work / ((int64_t)blocks * block * 16)));
    if (const char* env = getenv("RTMAP_CLAIM"))
        a.claim = std::max(64, std::min(4096, atoi(env)));
    size_t lds = sizeof(int2) * RT_STACK_LDS * block;   // {node, entry distance} per entry
    if constexpr (MODE != MODE_GEOM) {
        if (ext) {
            if constexpr (MODE == MODE_SINGLE) {
                if (accel == RT_ACCEL_BRUTE) {
                    hipLaunchKernelGGL((k_forward<true, MODE, false, true>), dim3(blocks), dim3(block), lds, st, a);
                    return;
                }
            }
            if (wide)
                hipLaunchKernelGGL((k_forward<false, MODE, true, true>), dim3(blocks), dim3(block), lds, st, a);
            else
                hipLaunchKernelGGL((k_forward<false, MODE, false, true>), dim3(blocks), dim3(block), lds, st, a);
            return;
        }
    }
    if (accel == RT_ACCEL_BRUTE)
        hipLaunchKernelGGL((k_forward<true, MODE, false, false>), dim3(blocks), dim3(block), lds, st, a);
    else if (wide)
        hipLaunchKernelGGL((k_forward<false, MODE, true, false>), dim3(blocks), dim3(block), lds, st, a);
    else
        hipLaunchKernelGGL((k_forward<false, MODE, false, false>), dim3(blocks), dim3(block), lds, st, a);
}

// Tree width: forced by accel, else tuned (or overridden), default 4-wide.
static bool use_wide(const rt_scene* s, int accel = RT_ACCEL_BVH) {
    if (!s->wide || s->root < 0 || accel == RT_ACCEL_BVH2 || accel == RT_ACCEL_BRUTE) return false;
    if (accel == RT_ACCEL_BVH4) return true;
    if (const char* env = getenv("RTMAP_WIDTH")) return atoi(env) != 2;
    return s->tuned_width != 2;
}

rt_status rt_launch_forward(const FwdLaunch& f, hipStream_t st) {
    const rt_scene* s = f.scene;
    FwdArgs a;
    base_args(a, s, f.block, f.eps_r, f.sigma, f.pl, f.L, f.t_min);
    a.tx = f.tx;
    a.ray_begin = f.ray_begin;
    a.n_work = f.ray_end - f.ray_begin;
    a.deposit = f.deposit;
    a.npol = f.tx.pol == RT_POL_DUAL ? 2 : 1;
    a.map = f.map;
    a.map_stride = (int64_t)f.pl.W * f.pl.H;
    a.tape_seg = f.tape ? f.tape->seg : nullptr;
    a.tape_nseg = f.tape ? f.tape->nseg : nullptr;
    a.tape_n = f.tape ? f.tape->n_rays : 0;
    a.hits = f.hits;
    a.cells = f.cells;
    a.weights = f.weights;
    a.stats = f.stats;
    a.refill = std::max(1, std::min(64, f.refill));
    a.ray_end = f.ray_end;
    if (f.order) {
        a.operm = f.order->perm;
        a.oshift = s->shifts;
        a.olog2m = f.order->log2m;
    }
    int blocks = 0;
    rt_status r = size_spill(a, s, f.block, &blocks);
    if (r != RT_OK) return r;
    int64_t map_n = a.map_stride * a.npol;
    {
        int64_t zn = f.zero_map ? map_n : 0;
        int g = (int)std::min<int64_t>(2048, std::max<int64_t>(2, (zn + 255) / 256));
        hipLaunchKernelGGL(k_prepare, dim3(g), dim3(256), 0, st, f.map, zn, s->counters);
    }
    if (f.order) rt_order_shifts_single(f.order, f.tx.n_rays, s->shifts, st);
    a.rr_depth = f.rr_depth;
    a.rr_p_max = f.rr_p_max;
    a.gain_threshold = f.gain_threshold;
    a.seed = f.seed;
    a.gain_scale = f.gain_scale;
    a.inv_kappa = 1.0f / f.tx.kappa;
    a.thickness = f.thickness;
    a.scattering = f.scattering;
    a.xpd = f.xpd;
    a.pattern = f.pattern;
    a.refraction = f.refraction;
    a.k0 = f.k0;
    const bool ext = f.rr_p_max > 0.0f || f.gain_threshold > 0.0f || f.thickness != nullptr || f.scattering != nullptr;
    if (a.n_work > 0) launch_mode<MODE_SINGLE>(a, f.accel, use_wide(s, f.accel), blocks, f.block, st, ext);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rt_hip_fail(e, "forward launch");
    return RT_OK;
}

// Several transmitters in one persistent launch.  geom_only = false: deposit
// into maps[slot] (one material set, map stride slot_stride, maps zeroed
// here); geom_only = true: write the geometry tape (2 records per segment).
rt_status rt_launch_forward_multi(const rt_scene* s, const float* eps_r, const float* sigma, const PlaneDesc& pl,
                                  int L, float t_min, int block, int deposit, int refill,
                                  const rt_scene::OrderTable* order, int64_t max_chunks, const TxDesc* txs,
                                  const int64_t* prefix, const int32_t* slots, int n_tx, int64_t total_rays,
                                  bool geom_only, float* maps, int64_t slot_stride, int64_t zero_floats,
                                  float4* geom_seg, int* geom_nseg, const FwdExt* ext, hipStream_t st) {
    FwdArgs a;
    base_args(a, s, block, eps_r, sigma, pl, L, t_min);
    a.ray_begin = 0;
    a.n_work = total_rays;
    a.deposit = deposit;
    a.map = maps;
    a.map_stride = (int64_t)pl.W * pl.H;
    a.txs = txs;
    a.prefix = prefix;
    a.slots = slots;
    a.n_tx = n_tx;
    a.slot_stride = slot_stride;
    a.refill = std::max(1, std::min(64, refill));
    if (order) {
        a.operm = order->perm;
        a.oshift = s->shifts;
        a.olog2m = order->log2m;
    }
    if (geom_only) {
        a.tape_seg = geom_seg;
        a.tape_nseg = geom_nseg;
        a.tape_n = total_rays;
        a.tape_groups = 2;
    }
    int blocks = 0;
    rt_status r = size_spill(a, s, block, &blocks);
    if (r != RT_OK) return r;
    int g = (int)std::min<int64_t>(4096, std::max<int64_t>(2, (zero_floats + 255) / 256));
    hipLaunchKernelGGL(k_prepare, dim3(g), dim3(256), 0, st, maps, zero_floats, s->counters);
    if (order) rt_order_shifts_multi(order, txs, n_tx, max_chunks, s->shifts, st);
    bool use_ext = false;
    if (ext && !geom_only) {
        a.rr_depth = ext->rr_depth;
        a.rr_p_max = ext->rr_p_max;
        a.gain_threshold = ext->gain_threshold;
        a.gain_scale = ext->gain_scale;
        a.seed = ext->seed;
        a.thickness = ext->thickness;
        a.scattering = ext->scattering;
        a.xpd = ext->xpd;
        a.pattern = ext->pattern;
        a.refraction = ext->refraction;
        a.k0 = ext->k0;
        use_ext = ext->rr_p_max > 0.0f || ext->gain_threshold > 0.0f || ext->thickness != nullptr ||
                  ext->scattering != nullptr;
    }
    if (total_rays > 0) {
        if (geom_only) launch_mode<MODE_GEOM>(a, RT_ACCEL_BVH, use_wide(s), blocks, block, st);
        else launch_mode<MODE_MULTI>(a, RT_ACCEL_BVH, use_wide(s), blocks, block, st, use_ext);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rt_hip_fail(e, "batched forward launch");
    return RT_OK;
}
