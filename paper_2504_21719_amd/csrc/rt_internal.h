// rt_internal.h -- library-internal types shared by the host ABI layer and the
// kernel launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/rt.h"

// Physical constants (SI).  The paper prints none of them; these are the
// exact speed of light and the CODATA 2018 vacuum permittivity.
#define RT_C0 299792458.0
#define RT_EPS0 8.8541878128e-12
#define RT_PI 3.14159265358979323846

// Traversal stack: RT_STACK_LDS entries per lane live in LDS; deeper entries
// spill to a per-lane global buffer sized from the BVH depth.
#define RT_STACK_LDS 16

// Empty child slot of a 4-wide node.
#define RT_WIDE_EMPTY 0x7fffffff
// Work queues of the persistent kernels: the launch's work indices are split
// into up to RT_QUEUES contiguous ranges, each with its own counter on its own
// 256-byte line, so that lane refills do not serialise on one address.  One
// more line after them counts the queues drained so far.
#define RT_QUEUES 256
#define RT_QUEUE_STRIDE 32

// LBVH layout.  Internal node = 4 x float4 (64 B, one cache line):
//   q0 = (L.lo.x, L.hi.x, L.lo.y, L.hi.y)
//   q1 = (R.lo.x, R.hi.x, R.lo.y, R.hi.y)
//   q2 = (L.lo.z, L.hi.z, R.lo.z, R.hi.z)
//   q3 = (left ref, right ref, -, -)   (int bits)
// A child reference r >= 0 is an internal node; r < 0 is the leaf holding
// triangle slot ~r.  Triangles are stored in Morton order ("slots"):
//   tris[3 s + 0] = (v0.xyz, original id bits)
//   tris[3 s + 1] = (v1.xyz, material bits)
//   tris[3 s + 2] = (v2.xyz, 0)
//   normals[s]    = (unit geometric normal, material bits)
struct rt_scene {
    int device = 0;
    int64_t n_tri = 0;
    int32_t n_mat = 0;
    int32_t depth = 0;        // deepest leaf depth (root = 0)
    int32_t root = -1;        // child reference of the root (unused if n_tri == 0)
    float4* nodes = nullptr;
    float4* tris = nullptr;
    float4* normals = nullptr;
    // 4-wide BVH collapsed from the binary one: 8 x float4 (128 B) per node,
    //   w0 = x_lo of children 0..3, w1 = x_hi, w2 = y_lo, w3 = y_hi,
    //   w4 = z_lo, w5 = z_hi, w6 = child refs (>= 0 wide node, < 0 leaf
    //   slot ~r, RT_WIDE_EMPTY), w7 unused;
    // node 0 is the root.  Built when n_tri >= 2.  A ray reads, per axis, the
    // near plane first (lo for a positive direction component, else hi) and
    // the far one at the byte offset XOR 16.
    float4* wide = nullptr;
    int64_t n_wide = 0;
    uint64_t* morton = nullptr;   // sorted Morton codes (kept for rt_scene_export)
    int tuned_width = 0;      // 2 binary, 4 wide (0 = default)
    size_t bytes = 0;
    double build_ms = 0.0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    // per-scene workspace: RT_QUEUES work-queue heads and the drained-queue
    // count, RT_QUEUE_STRIDE apart
    unsigned long long* counters = nullptr;
    int* spill = nullptr;     // traversal stack spill
    size_t spill_entries = 0; // ints available in `spill`
    // autotuned launch configuration (0 = not tuned)
    int tuned_block = 0;
    int tuned_deposit = 0;
    int tuned_refill = 0;     // refill a wavefront once this many lanes are idle
    int tuned_order = 0;      // 1 coherent launch order, 2 lattice order
    // coherent launch order: per chunk size 2^log2m, the azimuth-sorted order
    // of j in [0, 2^log2m) (perm) and its sorted azimuths (az); any chunk's
    // order is a rotation of it (see rt_order_table)
    struct OrderTable {
        int log2m = 0;
        int* perm = nullptr;
        unsigned* az = nullptr;
    } otab[12];
    int n_otab = 0;
    int* shifts = nullptr;          // per-call rotation of every full chunk
    size_t shifts_cap = 0;
    // backward workspace: per-block FP64 partial sums
    void* grad_ws = nullptr;
    size_t grad_ws_bytes = 0;
    // batched workspaces: geometry tape of every ray, FP64 gradient sums
    void* geom_ws = nullptr;
    size_t geom_ws_bytes = 0;
    void* bgrad_ws = nullptr;
    size_t bgrad_ws_bytes = 0;
    // batched-call staging (device copies of per-transmitter descriptors)
    void* tx_desc = nullptr;
    size_t tx_desc_bytes = 0;
    void* tx_desc_host = nullptr;  // pinned host staging
    // captured batched step, replayed while the call key repeats
    uint64_t graph_key = 0;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
};

// Tape: per segment (l, ray) four float4 records, stored [l][g][ray] for
// coalesced access:
//   g = 0: (k.xyz, hit slot bits or -1)
//   g = 1: (e_s.xyz, crossed cell bits or -1)
//   g = 2: (T.a, T.b)   complex re/im
//   g = 3: (T.c, T.d)
// plus one int per ray: number of traced segments.
struct rt_tape {
    int64_t n_rays = 0;       // rays in the range the tape was created for
    int32_t max_depth = 0;
    float4* seg = nullptr;
    int* nseg = nullptr;
    size_t bytes = 0;
    // identity of the forward call that filled it
    uint64_t key = 0;
    bool filled = false;
};

// Per-transmitter launch descriptor (host-computed constants).
struct TxDesc {
    float pos[3];
    int32_t pattern;         // 0 iso, 1 directional
    float R[9];              // R(yaw, pitch, roll), row-major
    float dR[3][9];          // dR/d yaw, dR/d pitch, dR/d roll
    double ax[3];            // local +x axis in global coordinates (first column of R), FP64
    double yaw, pitch, roll;
    float q;
    int32_t pol;             // 0 V, 1 H, 2 dual
    int64_t n_rays;          // N_S of this transmitter's lattice
    int64_t shift0;          // first entry of this lattice's chunks in the shift table
    int64_t n_chunks;        // full chunks of the launch order (0 = lattice order)
    float kappa;             // lambda^2 / (4 pi N_S dx dy)
    int32_t n_ant;           // synthetic transmit array (0 = single element)
    const double* ant_pos;   // [n_ant][3] element offsets, metres, global frame
    const float* precoding;  // [n_ant][2] complex weights
    double four_inv_lambda;  // 4 / lambda: phase in quarter turns per metre
};

// Plane + physics constants for one call.
struct PlaneDesc {
    float z, x0, y0, inv_dx, inv_dy;
    int32_t W, H;
    float inv_eps0_omega;    // 1 / (eps0 omega): sigma -> Im(eta) scale
};

// Error channel (thread-local message).
void rt_set_error(const std::string& msg);
rt_status rt_fail(rt_status st, const std::string& msg);
rt_status rt_hip_fail(hipError_t e, const char* what);

// Builders and launchers (device code lives in the .hip files).
rt_status rt_build_lbvh(rt_scene* s, const float* V, int64_t n_v, const int32_t* F,
                        const int32_t* M, hipStream_t st);

struct FwdLaunch {
    const rt_scene* scene;
    const float* eps_r;
    const float* sigma;
    TxDesc tx;
    PlaneDesc pl;
    int64_t ray_begin, ray_end;
    int32_t L;
    float t_min;
    int accel;               // 0 BVH, 1 brute force
    int deposit;             // 1 atomic, 2 wave
    int block;
    int refill;              // 1..64
    const rt_scene::OrderTable* order;   // coherent launch order, or null
    bool zero_map;
    float* map;
    rt_tape* tape;
    int32_t* hits;
    int32_t* cells;
    float* weights;
    unsigned long long* stats;
    int32_t rr_depth;        // early termination before segments l >= rr_depth (>= 1)
    float rr_p_max;          // Russian roulette (0 = off)
    float gain_threshold;    // gain thresholding (0 = off)
    uint32_t seed;
    float gain_scale;        // lambda^2 / (16 pi^2)
    const float* thickness;  // slab thickness per material (m), or null (half-space)
    const float* scattering; // scattering coefficient per material, or null (no diffuse)
    const float* xpd;        // cross-polarisation share per material
    const float* pattern;    // [n_mat][4] scattering pattern, or null (Lambertian)
    int32_t refraction;      // sample reflection or transmission at every hit
    float k0;                // 2 pi / lambda
};
rt_status rt_launch_forward(const FwdLaunch& f, hipStream_t st);

struct BwdLaunch {
    const rt_scene* scene;
    const float* eps_r;
    const float* sigma;
    TxDesc tx;
    PlaneDesc pl;
    int64_t ray_begin, ray_end;
    int32_t L;
    const rt_tape* tape;
    const float* grad_map;
    float* grad_eps;
    float* grad_sigma;
    float* grad_orient;
    const float* thickness;  // slab thickness per material (m), or null
    int32_t refraction;
    float k0;                // 2 pi / lambda
    int32_t rr_depth;        // Russian roulette in the forward before segments l >= rr_depth
    float rr_p_max;          // (0 = off)
    const float* scattering; // diffuse reflection: S and K_x per material, or null
    const float* xpd;
    uint32_t seed;           // key of the forward's random streams
    void* workspace;         // per-block partial sums, or null (the scene's, grown on demand)
    size_t workspace_bytes;
};
rt_status rt_launch_backward(const BwdLaunch& b, hipStream_t st);
// Device address of this GPU's static backward workspace (resolved once per
// device) and its size.
rt_status rt_backward_scratch(void** out);
size_t rt_backward_scratch_bytes();

// The extensions of the single-transmitter forward (slab walls, refraction,
// diffuse reflection, early termination) for a launch over several
// transmitters with one material set.
struct FwdExt {
    const float* thickness;  // slab thickness per material (m), or null
    const float* scattering; // S per material, or null
    const float* xpd;        // K_x per material (with scattering)
    const float* pattern;    // [n_mat][4] scattering patterns, or null (Lambertian)
    int32_t refraction;
    float k0;                // 2 pi / lambda
    int32_t rr_depth;        // early termination before segments l >= rr_depth (>= 1)
    float rr_p_max;          // Russian roulette (0 = off)
    float gain_threshold;    // (0 = off)
    float gain_scale;        // lambda^2 / (16 pi^2)
    uint32_t seed;
};

struct BatchLaunch {
    const rt_scene* scene;
    const float* eps_r;      // [S][n_mat]
    const float* sigma;
    int32_t n_samples;
    int32_t n_tx;
    const TxDesc* tx_dev;    // device [n_tx], ordered largest budget first
    const int64_t* prefix_dev;  // device [n_tx + 1] exclusive prefix of budgets
    const int32_t* tx_slot_dev; // device [n_tx]: output slot of ordered tx
    const int64_t* woff_dev;    // device [n_tx + 1]: exclusive prefix of the 64-ray
                                // wavefronts each ordered tx's rays touch
    int64_t total_waves;        // woff[n_tx]
    int64_t total_rays;
    PlaneDesc pl;
    int32_t L;
    float t_min;
    int block;
    int deposit;
    int refill;
    const rt_scene::OrderTable* order;   // coherent launch order, or null
    int64_t max_chunks;      // largest number of full chunks of one lattice
    float* maps;             // [n_tx][S][H][W]
    const float* grad_maps;  // [n_tx][S][H][W] or null
    float* grads;            // [n_tx][S][2 n_mat + 3] or null
    FwdExt ext;              // all of it for one material set without gradients;
                             // thickness alone for material samples and gradients
    bool has_arrays;         // a transmitter has a transmit array
};
rt_status rt_batched_workspace(const BatchLaunch& b, hipStream_t st);
rt_status rt_launch_batched(const BatchLaunch& b, hipStream_t st);

rt_status rt_launch_forward_multi(const rt_scene* s, const float* eps_r, const float* sigma, const PlaneDesc& pl,
                                  int L, float t_min, int block, int deposit, int refill,
                                  const rt_scene::OrderTable* order, int64_t max_chunks, const TxDesc* txs,
                                  const int64_t* prefix, const int32_t* slots, int n_tx, int64_t total_rays,
                                  bool geom_only, float* maps, int64_t slot_stride, int64_t zero_floats,
                                  float4* geom_seg, int* geom_nseg, const FwdExt* ext, hipStream_t st);

int rt_persistent_blocks(int block, int device);

// Traversal stack entries a query can need: the binary tree pushes at most one
// entry per level; the wide tree at most three per wide level, and a wide
// level spans at least one binary level.
inline int64_t rt_stack_need(const rt_scene* s) { return 3 * (int64_t)s->depth + 2; }

// Coherent launch order.  rt_order_log2m picks the chunk size for an N-ray
// lattice; rt_order_table builds (once, synchronously) the sorted order of a
// chunk; rt_order_reserve grows the shift table (synchronously, outside any
// capture); rt_order_shifts_* queue the per-chunk rotations.
int rt_order_log2m(int64_t N);
rt_status rt_order_table(rt_scene* s, int log2m, hipStream_t st, const rt_scene::OrderTable** out);
rt_status rt_order_reserve(rt_scene* s, size_t entries, hipStream_t st);
void rt_order_shifts_single(const rt_scene::OrderTable* t, int64_t N, int* shifts, hipStream_t st);
void rt_order_shifts_multi(const rt_scene::OrderTable* t, const TxDesc* txs, int n_tx, int64_t max_chunks,
                           int* shifts, hipStream_t st);
