// rt_capi.cpp -- the extern "C" entry points of librtmap.so: argument
// validation (all on the host, before any device work is queued), object
// ownership, launch descriptors and the thread-local error channel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rt_internal.h"

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

void rt_set_error(const std::string& m) { g_err = m; }
rt_status rt_fail(rt_status st, const std::string& m) {
    g_err = m;
    return st;
}
rt_status rt_hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE;
}

extern "C" const char* rt_last_error(void) { return g_err.c_str(); }

#define CHECK_ARG(cond, msg)                      \
    do {                                          \
        if (!(cond)) return rt_fail(RT_EINVAL, msg); \
    } while (0)

static bool finite_d(double v) { return std::isfinite(v); }

// ------------------------------------------------------------------- scene
extern "C" rt_status rt_build_scene(const float* vertices, int64_t n_vertices, const int32_t* triangles,
                                    int64_t n_triangles, const int32_t* tri_material, int32_t n_materials,
                                    void* stream, rt_scene** out) {
    CHECK_ARG(out != nullptr, "rt_build_scene: out is NULL");
    *out = nullptr;
    CHECK_ARG(n_vertices >= 0 && n_triangles >= 0, "rt_build_scene: negative size");
    CHECK_ARG(n_triangles < (int64_t)1 << 30, "rt_build_scene: more than 2^30 triangles");
    CHECK_ARG(n_materials >= 1 && n_materials <= 65536, "rt_build_scene: n_materials must be in [1, 65536]");
    if (n_triangles > 0) {
        CHECK_ARG(vertices && triangles && tri_material, "rt_build_scene: NULL input pointer");
        CHECK_ARG(n_vertices > 0, "rt_build_scene: triangles given but no vertices");
    }
    hipStream_t st = (hipStream_t)stream;
    rt_scene* s = new rt_scene();
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return rt_hip_fail(e, "hipGetDevice");
    }
    s->n_tri = n_triangles;
    s->n_mat = n_materials;
    e = hipMalloc(&s->counters, sizeof(unsigned long long) * (RT_QUEUES + 1) * RT_QUEUE_STRIDE);
    if (e != hipSuccess) {
        delete s;
        return rt_hip_fail(e, "hipMalloc(counters)");
    }
    rt_status r = rt_build_lbvh(s, vertices, n_vertices, triangles, tri_material, st);
    if (r != RT_OK) {
        std::string m = g_err;
        rt_scene_destroy(s);
        return rt_fail(r, m);
    }
    // traversal spill: (depth + 1 - RT_STACK_LDS) entries for every lane of
    // the largest persistent grid (a fixed number of lanes per CU)
    int64_t need_depth = std::max<int64_t>(0, rt_stack_need(s) - RT_STACK_LDS);
    int64_t lanes = (int64_t)rt_persistent_blocks(64, s->device) * 64;
    s->spill_entries = (size_t)(need_depth * lanes);
    if (s->spill_entries) {
        e = hipMalloc(&s->spill, sizeof(int) * s->spill_entries);
        if (e != hipSuccess) {
            rt_scene_destroy(s);
            return rt_hip_fail(e, "hipMalloc(spill)");
        }
    }
    s->bytes += sizeof(int) * s->spill_entries + sizeof(unsigned long long) * 8;
    *out = s;
    return RT_OK;
}

extern "C" rt_status rt_scene_destroy(rt_scene* s) {
    if (!s) return RT_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(s->nodes);
    (void)hipFree(s->tris);
    (void)hipFree(s->normals);
    (void)hipFree(s->wide);
    (void)hipFree(s->morton);
    (void)hipFree(s->counters);
    (void)hipFree(s->spill);
    (void)hipFree(s->tx_desc);
    (void)hipFree(s->grad_ws);
    for (int i = 0; i < s->n_otab; i++) {
        (void)hipFree(s->otab[i].perm);
        (void)hipFree(s->otab[i].az);
    }
    (void)hipFree(s->shifts);
    (void)hipFree(s->geom_ws);
    (void)hipFree(s->bgrad_ws);
    if (s->tx_desc_host) (void)hipHostFree(s->tx_desc_host);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    delete s;
    return RT_OK;
}

extern "C" rt_status rt_scene_info_get(const rt_scene* s, rt_scene_info* out) {
    CHECK_ARG(s && out, "rt_scene_info_get: NULL argument");
    out->n_triangles = s->n_tri;
    out->n_materials = s->n_mat;
    out->bvh_depth = s->depth;
    out->n_nodes = std::max<int64_t>(0, s->n_tri - 1);
    out->device_bytes = (int64_t)s->bytes;
    out->build_ms = s->build_ms;
    out->tuned_block = s->tuned_block;
    out->tuned_deposit = s->tuned_deposit;
    out->tuned_refill = s->tuned_refill;
    out->tuned_order = s->tuned_order;
    out->tuned_width = s->tuned_width;
    for (int a = 0; a < 3; a++) {
        out->lo[a] = s->lo[a];
        out->hi[a] = s->hi[a];
    }
    return RT_OK;
}

extern "C" rt_status rt_scene_export(const rt_scene* s, uint64_t* morton, float* nodes, float* wide, float* tris,
                                     int64_t* n_wide, void* stream) {
    CHECK_ARG(s != nullptr, "rt_scene_export: NULL scene");
    if (n_wide) *n_wide = s->wide ? s->n_wide : 0;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = s->n_tri, n_int = std::max<int64_t>(0, n - 1);
    hipError_t e = hipSuccess;
    if (morton && n > 0 && e == hipSuccess)
        e = hipMemcpyAsync(morton, s->morton, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, st);
    if (nodes && n_int > 0 && e == hipSuccess)
        e = hipMemcpyAsync(nodes, s->nodes, sizeof(float4) * 4 * n_int, hipMemcpyDeviceToHost, st);
    if (wide && s->wide && s->n_wide > 0 && e == hipSuccess)
        e = hipMemcpyAsync(wide, s->wide, sizeof(float4) * 8 * s->n_wide, hipMemcpyDeviceToHost, st);
    if (tris && n > 0 && e == hipSuccess)
        e = hipMemcpyAsync(tris, s->tris, sizeof(float4) * 3 * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return rt_hip_fail(e, "rt_scene_export");
    return RT_OK;
}

extern "C" rt_status rt_set_launch_config(rt_scene* s, int32_t width, int32_t order, int32_t block,
                                         int32_t deposit, int32_t refill) {
    CHECK_ARG(s != nullptr, "rt_set_launch_config: NULL scene");
    CHECK_ARG(width == 0 || width == 2 || width == 4, "rt_set_launch_config: width must be 0, 2 or 4");
    CHECK_ARG(width != 4 || s->wide != nullptr, "rt_set_launch_config: this scene has no 4-wide tree");
    CHECK_ARG(order >= 0 && order <= 2, "rt_set_launch_config: order must be 0, 1 or 2");
    CHECK_ARG(block == 0 || block == 64 || block == 128 || block == 256 || block == 512,
              "rt_set_launch_config: block must be 0, 64, 128, 256 or 512");
    CHECK_ARG(deposit >= 0 && deposit <= 2, "rt_set_launch_config: deposit must be 0, 1 or 2");
    CHECK_ARG(refill >= 0 && refill <= 64, "rt_set_launch_config: refill must be in [0, 64]");
    s->tuned_width = width;
    s->tuned_order = order;
    s->tuned_block = block;
    s->tuned_deposit = deposit;
    s->tuned_refill = refill;
    return RT_OK;
}

// ------------------------------------------------------------ descriptors
static rt_status check_tx(const rt_tx* tx, bool allow_dual) {
    CHECK_ARG(tx != nullptr, "tx is NULL");
    for (int a = 0; a < 3; a++) CHECK_ARG(finite_d(tx->pos[a]), "tx position is not finite");
    CHECK_ARG(finite_d(tx->yaw) && finite_d(tx->pitch) && finite_d(tx->roll), "tx orientation is not finite");
    CHECK_ARG(tx->pattern == RT_PATTERN_ISO || tx->pattern == RT_PATTERN_DIRECTIONAL, "tx pattern must be 0 or 1");
    CHECK_ARG(std::isfinite(tx->pattern_q) && tx->pattern_q >= 0.0f, "tx pattern_q must be finite and >= 0");
    CHECK_ARG(tx->pol == RT_POL_V || tx->pol == RT_POL_H || (allow_dual && tx->pol == RT_POL_DUAL),
              allow_dual ? "tx pol must be 0 (V), 1 (H) or 2 (dual)" : "tx pol must be 0 (V) or 1 (H) here");
    CHECK_ARG(tx->n_ant >= 0 && tx->n_ant <= 65536, "tx n_ant must be in [0, 65536]");
    CHECK_ARG(tx->n_ant == 0 || (tx->ant_pos != nullptr && tx->precoding != nullptr),
              "tx ant_pos and precoding must be set when n_ant > 0");
    return RT_OK;
}

static rt_status check_plane(const rt_plane* p) {
    CHECK_ARG(p != nullptr, "plane is NULL");
    CHECK_ARG(finite_d(p->z) && finite_d(p->x0) && finite_d(p->y0), "plane origin is not finite");
    CHECK_ARG(finite_d(p->dx) && finite_d(p->dy) && p->dx > 0 && p->dy > 0, "plane cell size must be > 0");
    CHECK_ARG(p->W >= 1 && p->H >= 1, "plane must have W >= 1 and H >= 1 cells");
    CHECK_ARG((int64_t)p->W * p->H <= ((int64_t)1 << 30), "plane has more than 2^30 cells");
    return RT_OK;
}

static rt_status check_params(const rt_sbr_params* p, int64_t* b, int64_t* e) {
    CHECK_ARG(p != nullptr, "params is NULL");
    CHECK_ARG(finite_d(p->freq_hz) && p->freq_hz > 0, "freq_hz must be > 0");
    CHECK_ARG(p->n_rays >= 1 && p->n_rays <= ((int64_t)1 << 40), "n_rays must be in [1, 2^40]");
    CHECK_ARG(p->max_depth >= 0 && p->max_depth <= 64, "max_depth must be in [0, 64]");
    CHECK_ARG(std::isfinite(p->t_min) && p->t_min >= 0.0f, "t_min must be finite and >= 0");
    CHECK_ARG(p->accel >= RT_ACCEL_BVH && p->accel <= RT_ACCEL_BVH4, "accel must be 0, 1, 2 or 3");
    CHECK_ARG(p->deposit >= RT_DEPOSIT_AUTO && p->deposit <= RT_DEPOSIT_WAVE, "deposit must be 0, 1 or 2");
    CHECK_ARG(p->block_size == 0 || p->block_size == 64 || p->block_size == 128 || p->block_size == 256 ||
                  p->block_size == 512,
              "block_size must be 0, 64, 128, 256 or 512");
    CHECK_ARG(p->accumulate == 0 || p->accumulate == 1, "accumulate must be 0 or 1");
    CHECK_ARG(std::isfinite(p->rr_p_max) && p->rr_p_max >= 0.0f && p->rr_p_max <= 1.0f,
              "rr_p_max must be in [0, 1]");
    CHECK_ARG(std::isfinite(p->gain_threshold) && p->gain_threshold >= 0.0f, "gain_threshold must be >= 0");
    CHECK_ARG(p->refraction == 0 || p->refraction == 1, "refraction must be 0 or 1");
    int64_t begin = p->ray_begin, end = p->ray_end <= 0 ? p->n_rays : p->ray_end;
    CHECK_ARG(begin >= 0 && begin <= end && end <= p->n_rays, "ray range must satisfy 0 <= begin <= end <= n_rays");
    *b = begin;
    *e = end;
    return RT_OK;
}

static void fill_plane(const rt_plane* p, double freq, PlaneDesc* d) {
    d->z = (float)p->z;
    d->x0 = (float)p->x0;
    d->y0 = (float)p->y0;
    d->inv_dx = (float)(1.0 / p->dx);
    d->inv_dy = (float)(1.0 / p->dy);
    d->W = p->W;
    d->H = p->H;
    d->inv_eps0_omega = (float)(1.0 / (RT_EPS0 * 2.0 * RT_PI * freq));
}

static void fill_tx(const rt_tx* t, int64_t n_rays, const rt_plane* p, double freq, TxDesc* d) {
    for (int a = 0; a < 3; a++) d->pos[a] = (float)t->pos[a];
    d->pattern = t->pattern;
    d->q = t->pattern_q;
    d->pol = t->pol;
    d->yaw = t->yaw;
    d->pitch = t->pitch;
    d->roll = t->roll;
    double ca = cos(t->yaw), sa = sin(t->yaw), cb = cos(t->pitch), sb = sin(t->pitch), cg = cos(t->roll),
           sg = sin(t->roll);
    // R = Rz(yaw) Ry(pitch) Rx(roll) (eq. rotation) and its partial derivatives
    double R[9] = {ca * cb, ca * sb * sg - sa * cg, ca * sb * cg + sa * sg,
                   sa * cb, sa * sb * sg + ca * cg, sa * sb * cg - ca * sg,
                   -sb,     cb * sg,                cb * cg};
    double dy[9] = {-sa * cb, -sa * sb * sg - ca * cg, -sa * sb * cg + ca * sg,
                    ca * cb,  ca * sb * sg - sa * cg,  ca * sb * cg + sa * sg,
                    0.0,      0.0,                     0.0};
    double dp[9] = {-ca * sb, ca * cb * sg, ca * cb * cg,
                    -sa * sb, sa * cb * sg, sa * cb * cg,
                    -cb,      -sb * sg,     -sb * cg};
    double dr[9] = {0.0, ca * sb * cg + sa * sg, -ca * sb * sg + sa * cg,
                    0.0, sa * sb * cg - ca * sg, -sa * sb * sg - ca * cg,
                    0.0, cb * cg,                -cb * sg};
    d->ax[0] = R[0];
    d->ax[1] = R[3];
    d->ax[2] = R[6];
    for (int i = 0; i < 9; i++) {
        d->R[i] = (float)R[i];
        d->dR[0][i] = (float)dy[i];
        d->dR[1][i] = (float)dp[i];
        d->dR[2][i] = (float)dr[i];
    }
    d->n_rays = n_rays;
    double lam = RT_C0 / freq;
    d->kappa = (float)(lam * lam / (4.0 * RT_PI * (double)n_rays * p->dx * p->dy));
    d->n_ant = t->n_ant;
    d->ant_pos = t->ant_pos;
    d->precoding = t->precoding;
    d->four_inv_lambda = 4.0 / lam;
}

static uint64_t mix(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) h = (h ^ c[i]) * 1099511628211ull;   // FNV-1a
    return h;
}

static uint64_t call_key(const rt_scene* s, rt_materials m, const rt_tx* tx, const rt_plane* pl,
                         const rt_sbr_params* p, int64_t b, int64_t e) {
    uint64_t h = 1469598103934665603ull;
    h = mix(h, &s, sizeof(s));
    h = mix(h, &m.eps_r, sizeof(m.eps_r));
    h = mix(h, &m.sigma, sizeof(m.sigma));
    h = mix(h, &m.thickness, sizeof(m.thickness));
    h = mix(h, &m.scattering, sizeof(m.scattering));
    h = mix(h, &m.xpd, sizeof(m.xpd));
    h = mix(h, &p->refraction, sizeof(int32_t));
    h = mix(h, &p->seed, sizeof(uint32_t));
    h = mix(h, &p->rr_depth, sizeof(int32_t));
    h = mix(h, &p->rr_p_max, sizeof(float));
    h = mix(h, &p->gain_threshold, sizeof(float));
    h = mix(h, tx, sizeof(rt_tx));
    h = mix(h, pl, sizeof(rt_plane));
    h = mix(h, &p->freq_hz, sizeof(double));
    h = mix(h, &p->n_rays, sizeof(int64_t));
    h = mix(h, &b, sizeof(b));
    h = mix(h, &e, sizeof(e));
    h = mix(h, &p->max_depth, sizeof(int32_t));
    h = mix(h, &p->t_min, sizeof(float));
    return h;
}

static int pick_block(const rt_scene* s, const rt_sbr_params* p) {
    if (p->block_size) return p->block_size;
    if (s->tuned_block) return s->tuned_block;
    return 256;
}

// Untuned defaults (from a sweep on the Manhattan workload): same-cell
// summation across the wavefront, refill once the whole wavefront is idle,
// coherent launch order, 4-wide tree.
static int pick_deposit(const rt_scene* s, const rt_sbr_params* p) {
    if (p->deposit) return p->deposit;
    if (s->tuned_deposit) return s->tuned_deposit;
    return RT_DEPOSIT_WAVE;
}

static int pick_refill(const rt_scene* s) {
    int r = s->tuned_refill ? s->tuned_refill : 64;
    if (const char* env = getenv("RTMAP_REFILL")) r = atoi(env);
    return std::max(1, std::min(64, r));
}

static bool want_order(const rt_scene* s) {
    const char* env = getenv("RTMAP_ORDER");
    if (env) return env[0] != '0';
    return s->tuned_order != 2;
}

// Launch-order table for an N-ray lattice and room for its chunk rotations
// (synchronous on first use of a chunk size or a larger lattice).
static rt_status prepare_order(rt_scene* s, int64_t N, size_t chunks_total, int log2m, hipStream_t st,
                               const rt_scene::OrderTable** out) {
    *out = nullptr;
    if (!want_order(s) || N < 4096) return RT_OK;
    rt_status r = rt_order_table(s, log2m, st, out);
    if (r != RT_OK) return r;
    return rt_order_reserve(s, chunks_total, st);
}

static rt_status check_device(const rt_scene* s) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rt_hip_fail(e, "hipGetDevice");
    CHECK_ARG(dev == s->device, "the current device is not the scene's device");
    return RT_OK;
}

// ----------------------------------------------------------------- forward
extern "C" rt_status rt_radio_map(const rt_scene* scene, rt_materials materials, const rt_tx* tx,
                                  const rt_plane* plane, const rt_sbr_params* params, float* out_map,
                                  rt_tape* tape, const rt_records* records, void* stream) {
    CHECK_ARG(scene != nullptr, "rt_radio_map: scene is NULL");
    CHECK_ARG(out_map != nullptr, "rt_radio_map: out_map is NULL");
    CHECK_ARG(materials.eps_r && materials.sigma, "rt_radio_map: material pointers are NULL");
    rt_status r;
    if ((r = check_tx(tx, true)) != RT_OK) return r;
    if ((r = check_plane(plane)) != RT_OK) return r;
    int64_t b, e;
    if ((r = check_params(params, &b, &e)) != RT_OK) return r;
    if (tape) {
        CHECK_ARG(tape->n_rays == e - b && tape->max_depth == params->max_depth,
                  "rt_radio_map: tape was created for another ray range or depth");
    }
    CHECK_ARG(!params->refraction || materials.thickness,
              "rt_radio_map: refraction needs the slab thickness of every material");
    CHECK_ARG((materials.scattering == nullptr) == (materials.xpd == nullptr),
              "rt_radio_map: scattering and xpd must both be given or both be NULL");
    CHECK_ARG(!materials.scatter_pattern || materials.scattering,
              "rt_radio_map: scatter_pattern needs scattering and xpd");
    if (materials.scattering && tx->pol == RT_POL_DUAL)
        return rt_fail(RT_EUNSUPPORTED, "rt_radio_map: diffuse reflection takes one polarisation");
    if ((r = check_device(scene)) != RT_OK) return r;
    FwdLaunch f{};
    f.scene = scene;
    f.eps_r = materials.eps_r;
    f.sigma = materials.sigma;
    fill_tx(tx, params->n_rays, plane, params->freq_hz, &f.tx);
    fill_plane(plane, params->freq_hz, &f.pl);
    f.ray_begin = b;
    f.ray_end = e;
    f.L = params->max_depth;
    f.t_min = params->t_min;
    f.accel = params->accel;
    f.deposit = pick_deposit(scene, params);
    f.block = pick_block(scene, params);
    f.refill = pick_refill(scene);
    {
        int l = rt_order_log2m(params->n_rays);
        rt_status ro = prepare_order(const_cast<rt_scene*>(scene), params->n_rays,
                                     (size_t)(params->n_rays >> l), l, (hipStream_t)stream, &f.order);
        if (ro != RT_OK) return ro;
    }
    f.zero_map = params->accumulate == 0;
    f.map = out_map;
    f.tape = tape;
    f.rr_depth = std::max(1, params->rr_depth);
    f.rr_p_max = params->rr_p_max;
    f.gain_threshold = params->gain_threshold;
    f.seed = params->seed;
    {
        const double lam = RT_C0 / params->freq_hz;
        f.gain_scale = (float)(lam * lam / (16.0 * RT_PI * RT_PI));
    }
    f.thickness = materials.thickness;
    f.scattering = materials.scattering;
    f.xpd = materials.xpd;
    f.pattern = materials.scatter_pattern;
    f.refraction = params->refraction;
    f.k0 = (float)(2.0 * RT_PI * params->freq_hz / RT_C0);
    if (records) {
        f.hits = records->hits;
        f.cells = records->cells;
        f.weights = records->weights;
        f.stats = records->stats;
    }
    r = rt_launch_forward(f, (hipStream_t)stream);
    if (r != RT_OK) return r;
    if (tape) {
        tape->key = call_key(scene, materials, tx, plane, params, b, e);
        tape->filled = true;
    }
    return RT_OK;
}

// -------------------------------------------------------------------- tape
extern "C" size_t rt_tape_bytes(const rt_sbr_params* p) {
    if (!p) return 0;
    int64_t b, e;
    if (check_params(p, &b, &e) != RT_OK) return 0;
    size_t n = (size_t)(e - b);
    return n * (size_t)(p->max_depth + 1) * 4 * sizeof(float4) + n * sizeof(int);
}

extern "C" rt_status rt_tape_create(const rt_sbr_params* p, rt_tape** out) {
    CHECK_ARG(out != nullptr, "rt_tape_create: out is NULL");
    *out = nullptr;
    int64_t b, e;
    rt_status r = check_params(p, &b, &e);
    if (r != RT_OK) return r;
    rt_tape* t = new rt_tape();
    t->n_rays = e - b;
    t->max_depth = p->max_depth;
    size_t segb = (size_t)t->n_rays * (size_t)(p->max_depth + 1) * 4 * sizeof(float4);
    hipError_t he = hipMalloc(&t->seg, std::max<size_t>(16, segb));
    if (he == hipSuccess) he = hipMalloc(&t->nseg, std::max<size_t>(4, sizeof(int) * (size_t)t->n_rays));
    if (he != hipSuccess) {
        rt_tape_destroy(t);
        return rt_hip_fail(he, "rt_tape_create: hipMalloc");
    }
    t->bytes = segb + sizeof(int) * (size_t)t->n_rays;
    *out = t;
    return RT_OK;
}

extern "C" rt_status rt_tape_destroy(rt_tape* t) {
    if (!t) return RT_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(t->seg);
    (void)hipFree(t->nseg);
    delete t;
    return RT_OK;
}

// ---------------------------------------------------------------- backward
// `noalloc`: the per-block partial sums go to this GPU's static workspace
// instead of the scene's (which is allocated on first use).
static rt_status backward_call(const rt_scene* scene, rt_materials materials, const rt_tx* tx,
                               const rt_plane* plane, const rt_sbr_params* params, const rt_tape* tape,
                               const float* grad_map, float* grad_eps_r, float* grad_sigma, float* grad_orient,
                               void* stream, bool noalloc) {
    CHECK_ARG(scene != nullptr, "rt_radio_map_backward: scene is NULL");
    CHECK_ARG(tape != nullptr, "rt_radio_map_backward: tape is NULL");
    CHECK_ARG(grad_map != nullptr, "rt_radio_map_backward: grad_map is NULL");
    CHECK_ARG(materials.eps_r && materials.sigma, "rt_radio_map_backward: material pointers are NULL");
    rt_status r;
    if ((r = check_tx(tx, true)) != RT_OK) return r;
    if ((r = check_plane(plane)) != RT_OK) return r;
    int64_t b, e;
    if ((r = check_params(params, &b, &e)) != RT_OK) return r;
    CHECK_ARG(tape->filled && tape->key == call_key(scene, materials, tx, plane, params, b, e),
              "rt_radio_map_backward: the tape was not filled by a forward call with these arguments");
    if ((r = check_device(scene)) != RT_OK) return r;
    BwdLaunch bl{};
    bl.scene = scene;
    bl.eps_r = materials.eps_r;
    bl.sigma = materials.sigma;
    fill_tx(tx, params->n_rays, plane, params->freq_hz, &bl.tx);
    fill_plane(plane, params->freq_hz, &bl.pl);
    bl.ray_begin = b;
    bl.ray_end = e;
    bl.L = params->max_depth;
    bl.tape = tape;
    bl.grad_map = grad_map;
    bl.grad_eps = grad_eps_r;
    bl.grad_sigma = grad_sigma;
    bl.grad_orient = grad_orient;
    bl.thickness = materials.thickness;
    bl.refraction = params->refraction;
    bl.k0 = (float)(2.0 * RT_PI * params->freq_hz / RT_C0);
    bl.rr_depth = std::max(1, params->rr_depth);
    bl.rr_p_max = params->rr_p_max;
    bl.scattering = materials.scattering;
    bl.xpd = materials.xpd;
    bl.seed = params->seed;
    if (noalloc) {
        if ((r = rt_backward_scratch(&bl.workspace)) != RT_OK) return r;
        bl.workspace_bytes = rt_backward_scratch_bytes();
    }
    return rt_launch_backward(bl, (hipStream_t)stream);
}

extern "C" rt_status rt_radio_map_backward(const rt_scene* scene, rt_materials materials, const rt_tx* tx,
                                           const rt_plane* plane, const rt_sbr_params* params,
                                           const rt_tape* tape, const float* grad_map, float* grad_eps_r,
                                           float* grad_sigma, float* grad_orient, void* stream) {
    return backward_call(scene, materials, tx, plane, params, tape, grad_map, grad_eps_r, grad_sigma, grad_orient,
                         stream, false);
}

extern "C" rt_status rt_radio_map_backward_noalloc(const rt_scene* scene, rt_materials materials, const rt_tx* tx,
                                                   const rt_plane* plane, const rt_sbr_params* params,
                                                   const rt_tape* tape, const float* grad_map, float* grad_eps_r,
                                                   float* grad_sigma, float* grad_orient, void* stream) {
    return backward_call(scene, materials, tx, plane, params, tape, grad_map, grad_eps_r, grad_sigma, grad_orient,
                         stream, true);
}

// ----------------------------------------------------------------- batched
extern "C" rt_status rt_radio_map_batched(const rt_scene* scene, rt_materials materials, int32_t n_samples,
                                          const rt_tx* txs, const int64_t* rays_per_tx, int32_t n_tx,
                                          const rt_plane* plane, const rt_sbr_params* params, float* out_maps,
                                          const float* grad_maps, float* grads, void* stream) {
    CHECK_ARG(scene != nullptr, "rt_radio_map_batched: scene is NULL");
    CHECK_ARG(out_maps != nullptr, "rt_radio_map_batched: out_maps is NULL");
    CHECK_ARG(materials.eps_r && materials.sigma, "rt_radio_map_batched: material pointers are NULL");
    CHECK_ARG(n_samples >= 1 && n_samples <= 64, "rt_radio_map_batched: n_samples must be in [1, 64]");
    CHECK_ARG(n_tx >= 1 && n_tx <= 4096, "rt_radio_map_batched: n_tx must be in [1, 4096]");
    CHECK_ARG(txs && rays_per_tx, "rt_radio_map_batched: txs / rays_per_tx are NULL");
    CHECK_ARG((grad_maps == nullptr) == (grads == nullptr),
              "rt_radio_map_batched: grad_maps and grads must both be given or both be NULL");
    rt_status r;
    // one material set without gradients runs the single-transmitter kernel
    // over all transmitters and takes all its extensions; material samples
    // and gradients share one traversal per ray, so they take only what
    // leaves the path unchanged (transmit arrays, slab walls without
    // refraction)
    const bool shared_paths = n_samples > 1 || grad_maps != nullptr;
    for (int i = 0; i < n_tx; i++) {
        if ((r = check_tx(&txs[i], false)) != RT_OK) return r;
        CHECK_ARG(rays_per_tx[i] >= 1 && rays_per_tx[i] <= ((int64_t)1 << 40),
                  "rt_radio_map_batched: rays_per_tx must be in [1, 2^40]");
    }
    if ((r = check_plane(plane)) != RT_OK) return r;
    int64_t b, e;
    rt_sbr_params p = *params;
    p.n_rays = 1;
    p.ray_begin = 0;
    p.ray_end = 0;
    if ((r = check_params(&p, &b, &e)) != RT_OK) return r;
    const bool path_changes = p.rr_p_max > 0.0f || p.gain_threshold > 0.0f || p.refraction ||
                              materials.scattering || materials.xpd || materials.scatter_pattern;
    if (shared_paths && path_changes)
        return rt_fail(RT_EUNSUPPORTED, "rt_radio_map_batched: early termination, refraction and diffuse "
                                        "reflection need one material sample and no gradients");
    CHECK_ARG(!p.refraction || materials.thickness,
              "rt_radio_map_batched: refraction needs the slab thickness of every material");
    CHECK_ARG((materials.scattering == nullptr) == (materials.xpd == nullptr),
              "rt_radio_map_batched: scattering and xpd must both be given or both be NULL");
    CHECK_ARG(!materials.scatter_pattern || materials.scattering,
              "rt_radio_map_batched: scatter_pattern needs scattering and xpd");
    if ((r = check_device(scene)) != RT_OK) return r;
    rt_scene* s = const_cast<rt_scene*>(scene);
    hipStream_t hs = (hipStream_t)stream;
    // order transmitters largest budget first so that the long lattices start early
    std::vector<int> order(n_tx);
    for (int i = 0; i < n_tx; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rays_per_tx[x] > rays_per_tx[y]; });
    // device tables: descriptors, budget prefix, wavefront prefix, slots
    static_assert(sizeof(TxDesc) % 8 == 0, "TxDesc must keep the int64 tables after it aligned");
    size_t need = sizeof(TxDesc) * n_tx + 2 * sizeof(int64_t) * (n_tx + 1) + sizeof(int32_t) * n_tx;
    std::vector<char> hb(need, 0);
    TxDesc* hd = (TxDesc*)hb.data();
    int64_t* hp = (int64_t*)(hb.data() + sizeof(TxDesc) * n_tx);
    int64_t* hw = hp + (n_tx + 1);
    int32_t* hslot = (int32_t*)(hw + (n_tx + 1));
    int64_t total = 0;
    // one launch-order chunk size for the whole batch (from the largest lattice)
    const int olog2m = rt_order_log2m(rays_per_tx[order[0]]);
    int64_t chunks_total = 0, max_chunks = 0;
    for (int i = 0; i < n_tx; i++) {
        int t = order[i];
        fill_tx(&txs[t], rays_per_tx[t], plane, params->freq_hz, &hd[i]);
        hd[i].n_chunks = rays_per_tx[t] >> olog2m;
        hd[i].shift0 = chunks_total;
        chunks_total += hd[i].n_chunks;
        max_chunks = std::max(max_chunks, hd[i].n_chunks);
        hp[i] = total;
        hslot[i] = t;
        total += rays_per_tx[t];
    }
    hp[n_tx] = total;
    // wavefronts of 64 consecutive global ray indices that hold rays of each
    // ordered transmitter: the batched gradients keep one partial sum per
    // (transmitter, wavefront) and add them in order
    hw[0] = 0;
    for (int i = 0; i < n_tx; i++) hw[i + 1] = hw[i] + (hp[i + 1] - 1) / 64 - hp[i] / 64 + 1;
    const rt_scene::OrderTable* otab = nullptr;
    {
        rt_status ro = prepare_order(s, rays_per_tx[order[0]], (size_t)chunks_total, olog2m, hs, &otab);
        if (ro != RT_OK) return ro;
        if (!otab) {
            for (int i = 0; i < n_tx; i++) hd[i].n_chunks = 0;
            max_chunks = 0;
        }
    }
    BatchLaunch bl{};
    bl.scene = scene;
    bl.eps_r = materials.eps_r;
    bl.sigma = materials.sigma;
    bl.n_samples = n_samples;
    bl.n_tx = n_tx;
    bl.total_rays = total;
    bl.total_waves = hw[n_tx];
    fill_plane(plane, params->freq_hz, &bl.pl);
    bl.L = params->max_depth;
    bl.t_min = params->t_min;
    bl.block = pick_block(scene, params);
    bl.deposit = pick_deposit(scene, params);
    bl.refill = pick_refill(scene);
    bl.order = otab;
    bl.max_chunks = max_chunks;
    bl.maps = out_maps;
    bl.grad_maps = grad_maps;
    bl.grads = grads;
    bl.ext.thickness = materials.thickness;
    bl.ext.scattering = materials.scattering;
    bl.ext.xpd = materials.xpd;
    bl.ext.pattern = materials.scatter_pattern;
    bl.ext.refraction = params->refraction;
    bl.ext.k0 = (float)(2.0 * RT_PI * params->freq_hz / RT_C0);
    bl.ext.rr_depth = std::max(1, params->rr_depth);
    bl.ext.rr_p_max = params->rr_p_max;
    bl.ext.gain_threshold = params->gain_threshold;
    {
        const double lam = RT_C0 / params->freq_hz;
        bl.ext.gain_scale = (float)(lam * lam / (16.0 * RT_PI * RT_PI));
    }
    bl.ext.seed = params->seed;
    bl.has_arrays = false;
    for (int i = 0; i < n_tx; i++) bl.has_arrays = bl.has_arrays || txs[i].n_ant > 0;
    // identity of the whole step: descriptors, pointers (including the
    // library workspaces the captured kernels read) and sizes
    uint64_t key = 1469598103934665603ull;
    key = mix(key, hb.data(), hb.size());
    const void* ptrs[9] = {materials.eps_r, materials.sigma, out_maps, grad_maps, grads, materials.thickness,
                           materials.scattering, materials.xpd, materials.scatter_pattern};
    key = mix(key, ptrs, sizeof(ptrs));
    key = mix(key, &bl.ext.refraction, sizeof(bl.ext.refraction));
    key = mix(key, &bl.ext.rr_depth, sizeof(bl.ext.rr_depth));
    key = mix(key, &bl.ext.rr_p_max, sizeof(bl.ext.rr_p_max));
    key = mix(key, &bl.ext.gain_threshold, sizeof(bl.ext.gain_threshold));
    key = mix(key, &bl.ext.seed, sizeof(bl.ext.seed));
    key = mix(key, plane, sizeof(rt_plane));
    key = mix(key, &bl.L, sizeof(bl.L));
    key = mix(key, &bl.t_min, sizeof(bl.t_min));
    key = mix(key, &bl.block, sizeof(bl.block));
    key = mix(key, &n_samples, sizeof(n_samples));
    key = mix(key, &params->freq_hz, sizeof(double));
    key = mix(key, &bl.deposit, sizeof(int));
    key = mix(key, &bl.refill, sizeof(int));
    const void* ws[6] = {otab, s->shifts, s->tx_desc, s->geom_ws, s->bgrad_ws, s->wide};
    key = mix(key, ws, sizeof(ws));
    int width = s->tuned_width;
    if (const char* env = getenv("RTMAP_WIDTH")) width = atoi(env);
    key = mix(key, &width, sizeof(width));
    const bool use_graph = getenv("RTMAP_NO_GRAPH") == nullptr;
    if (use_graph && s->graph_exec && s->graph_key == key) {
        hipError_t he = hipGraphLaunch(s->graph_exec, hs);
        if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: graph launch");
        return RT_OK;
    }
    // descriptors: pinned staging, then one upload on the caller's stream
    if (s->tx_desc_bytes < need) {
        (void)hipStreamSynchronize(hs);
        (void)hipFree(s->tx_desc);
        if (s->tx_desc_host) (void)hipHostFree(s->tx_desc_host);
        s->tx_desc = nullptr;
        s->tx_desc_host = nullptr;
        s->tx_desc_bytes = 0;
        hipError_t he = hipMalloc(&s->tx_desc, need);
        if (he == hipSuccess) he = hipHostMalloc(&s->tx_desc_host, need, hipHostMallocDefault);
        if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: staging allocation");
        s->tx_desc_bytes = need;
    } else {
        // the staging buffer may still be read by the previous call's upload
        (void)hipStreamSynchronize(hs);
    }
    memcpy(s->tx_desc_host, hb.data(), need);
    hipError_t he = hipMemcpyAsync(s->tx_desc, s->tx_desc_host, need, hipMemcpyHostToDevice, hs);
    if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: descriptor upload");
    char* db = (char*)s->tx_desc;
    bl.tx_dev = (const TxDesc*)db;
    bl.prefix_dev = (const int64_t*)(db + sizeof(TxDesc) * n_tx);
    bl.woff_dev = bl.prefix_dev + (n_tx + 1);
    bl.tx_slot_dev = (const int32_t*)(bl.woff_dev + (n_tx + 1));
    r = rt_batched_workspace(bl, hs);
    if (r != RT_OK) return r;
    if (!use_graph) return rt_launch_batched(bl, hs);
    // capture the step once on a library stream, then replay it on the caller's
    if (!s->capture_stream) {
        he = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
        if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: capture stream");
    }
    if (s->graph_exec) {
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
        s->graph_key = 0;
    }
    hipGraph_t graph = nullptr;
    he = hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: begin capture");
    r = rt_launch_batched(bl, s->capture_stream);
    hipError_t he2 = hipStreamEndCapture(s->capture_stream, &graph);
    if (r != RT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (he2 != hipSuccess) return rt_hip_fail(he2, "rt_radio_map_batched: end capture");
    he = hipGraphInstantiate(&s->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (he != hipSuccess) {
        s->graph_exec = nullptr;
        return rt_hip_fail(he, "rt_radio_map_batched: instantiate");
    }
    s->graph_key = key;
    he = hipGraphLaunch(s->graph_exec, hs);
    if (he != hipSuccess) return rt_hip_fail(he, "rt_radio_map_batched: graph launch");
    return RT_OK;
}

// ---------------------------------------------------------------- autotune
extern "C" rt_status rt_tune(rt_scene* scene, rt_materials materials, const rt_tx* tx, const rt_plane* plane,
                             const rt_sbr_params* params, int64_t n_probe_rays, float* scratch_map,
                             void* stream, int32_t* chosen_block, int32_t* chosen_deposit) {
    CHECK_ARG(scene != nullptr && scratch_map != nullptr, "rt_tune: NULL argument");
    CHECK_ARG(n_probe_rays >= 1, "rt_tune: n_probe_rays must be >= 1");
    int64_t b0, e0r;
    rt_status r = check_params(params, &b0, &e0r);
    if (r != RT_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    // probe: eight sub-ranges spread evenly over the lattice, aligned to the
    // launch-order chunks, so that every direction band is represented
    const int64_t N = params->n_rays;
    const int64_t M = (int64_t)1 << rt_order_log2m(N);
    const int n_sub = 8;
    int64_t sub = std::min<int64_t>(N, std::max<int64_t>(M, ((n_probe_rays / n_sub + M - 1) / M) * M));
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int i = 0; i < n_sub; i++) {
        int64_t b = ((N - sub) * i / std::max(1, n_sub - 1)) / M * M;
        ranges.push_back({b, std::min(N, b + sub)});
        if (sub >= N) break;
    }
    hipEvent_t ev0, ev1;
    hipError_t he = hipEventCreate(&ev0);
    if (he == hipSuccess) he = hipEventCreate(&ev1);
    if (he != hipSuccess) return rt_hip_fail(he, "rt_tune: hipEventCreate");
    rt_sbr_params p = *params;
    p.accel = RT_ACCEL_BVH;
    auto run_once = [&]() -> rt_status {
        for (size_t i = 0; i < ranges.size(); i++) {
            p.ray_begin = ranges[i].first;
            p.ray_end = ranges[i].second;
            p.accumulate = i ? 1 : 0;
            rt_status q = rt_radio_map(scene, materials, tx, plane, &p, scratch_map, nullptr, nullptr, stream);
            if (q != RT_OK) return q;
        }
        return RT_OK;
    };
    // search: tree width x launch order x workgroup size x deposit strategy x
    // wavefront refill threshold ("rays per wave" taken at once); the LDS part
    // of the traversal stack is fixed at compile time and spills beyond it
    const int blocks[] = {128, 256, 512};
    const int deps[] = {RT_DEPOSIT_ATOMIC, RT_DEPOSIT_WAVE};
    const int refills[] = {48, 56, 64};
    const int orders[] = {1, 2};
    const int widths[] = {4, 2};
    float best = 1e30f;
    int bb = 256, bd = RT_DEPOSIT_WAVE, br = 48, bo = 1, bw = 4;
    const int saved[5] = {scene->tuned_block, scene->tuned_deposit, scene->tuned_refill, scene->tuned_order,
                          scene->tuned_width};
    for (int wi : widths)
        for (int oi : orders)
            for (int bi : blocks)
                for (int di : deps)
                    for (int ri : refills) {
                        if (r != RT_OK) break;
                        if (wi == 4 && !scene->wide) continue;
                        p.block_size = bi;
                        p.deposit = di;
                        scene->tuned_refill = ri;
                        scene->tuned_order = oi;
                        scene->tuned_width = wi;
                        r = run_once();   // warm-up (also builds order tables)
                        if (r != RT_OK) break;
                        float ts[3] = {0, 0, 0};
                        for (int rep = 0; rep < 3 && r == RT_OK; rep++) {
                            (void)hipEventRecord(ev0, st);
                            r = run_once();
                            (void)hipEventRecord(ev1, st);
                            (void)hipEventSynchronize(ev1);
                            (void)hipEventElapsedTime(&ts[rep], ev0, ev1);
                        }
                        std::sort(ts, ts + 3);
                        if (r == RT_OK && ts[1] < best) {
                            best = ts[1];
                            bb = bi;
                            bd = di;
                            br = ri;
                            bo = oi;
                            bw = wi;
                        }
                    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (r != RT_OK) {
        scene->tuned_block = saved[0];
        scene->tuned_deposit = saved[1];
        scene->tuned_refill = saved[2];
        scene->tuned_order = saved[3];
        scene->tuned_width = saved[4];
        return r;
    }
    scene->tuned_block = bb;
    scene->tuned_deposit = bd;
    scene->tuned_refill = br;
    scene->tuned_order = bo;
    scene->tuned_width = bw;
    if (chosen_block) *chosen_block = bb;
    if (chosen_deposit) *chosen_deposit = bd;
    return RT_OK;
}
