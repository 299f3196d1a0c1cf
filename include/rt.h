/*
 * rt.h -- C ABI of librtmap.so, the MI355X (gfx950) SBR radio-map library.
 *
 * What the library computes: the radio map of a point source over a
 * horizontal measurement plane by shooting and bouncing rays (SBR), by
 * default for specular reflection only; the optional extensions (slab walls
 * and refraction, diffuse reflection, transmit arrays, early termination)
 * are described with the fields that enable them.  Citations are to
 * "Sionna RT: Technical Report"
 * (arXiv 2504.21719, v2.1):
 *   - rays leave the source on a spherical Fibonacci lattice of N_S points
 *     (Sec. "Sampling Initial Ray Directions");
 *   - each ray finds its closest hit in a triangle scene (Sec. "Scene Objects
 *     and Meshes"; Sec. "Generating Candidates by SBR");
 *   - at every hit it is specularly reflected (eq. path-solver-scatter-dir) and
 *     its 2x2 complex field transfer matrix is multiplied by the Fresnel
 *     reflection matrix of the hit material (eq. fresnel_in_vectors,
 *     eq. fresnel_out_vectors, eq. fresnel_vac, with eta from eq. eta);
 *   - every traced segment l = 0..L that crosses the plane adds
 *         lambda^2 ||T C_T||^2 / (4 pi N_S |M_i| |k_z|)
 *     to its cell i: this is the estimator eq. radio-map-solver-ci-all-2-
 *     estimator for specular chains (interaction probability 1; with the
 *     extensions, T also carries the 1/sqrt(Pr) sampling factors and the
 *     per-diffuse-point scale), where
 *     the squared ray-tube length of the change of variables dA = r^2/|n^T k|
 *     d(omega) cancels the spherical spreading of the path gain eq. radio-map-
 *     solver-path-gain (Sec. "Definition of Radio Map").
 *   - C_T is the transmit antenna pattern C = sqrt(G) F (eq. C) of a rotated
 *     antenna (eq. rotation, eq. theta_phi_prime, eq. F_prime_2_F).
 *
 * Conventions shared by every call:
 *   - SI units (metres, hertz, siemens per metre, radians).
 *   - "device" pointers point to memory of the current HIP device (for
 *     example torch CUDA tensors); "host" pointers point to CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on `stream` unless stated otherwise; outputs are
 *     valid after the stream is synchronised.
 *   - Every call returns an rt_status; on failure rt_last_error() returns a
 *     thread-local message.  No exception crosses the ABI.  Argument checks
 *     happen on the host before any device work is queued, so a rejected call
 *     writes no output.
 *   - The library never takes ownership of caller memory.  Objects it creates
 *     (rt_scene, rt_tape) are released only by their destroy calls.
 *   - Calls on one rt_scene share its device work state (work-queue
 *     counters, traversal spill area, launch-order tables, workspaces and
 *     the captured batched graph): queue them on one stream, or order them
 *     across streams and host threads; calls on different scenes are
 *     independent.  Likewise a tape belongs to one forward-backward pair at
 *     a time.
 *   - Environment overrides of the launch configuration, for experiments
 *     (each changes results only up to FP32 summation order):
 *     RTMAP_WIDTH (2: binary tree, else 4-wide), RTMAP_ORDER (0: lattice
 *     launch order, else coherent), RTMAP_REFILL (idle lanes a wavefront
 *     waits for before it takes new rays, 1..64), RTMAP_QUEUES (number of
 *     work queues, 1..256), RTMAP_CLAIM (rays per claim, 64..4096),
 *     RTMAP_NO_GRAPH (set: rt_radio_map_batched launches its kernels instead
 *     of replaying the captured graph).  They override rt_tune's choice and
 *     rt_set_launch_config.
 */
#ifndef RTMAP_RT_H
#define RTMAP_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_EINVAL = 1,        /* invalid argument (message says which)             */
    RT_ENOMEM = 2,        /* device allocation failed                          */
    RT_EDEVICE = 3,       /* HIP runtime error                                 */
    RT_EOVERFLOW = 4,     /* traversal stack overflow (map not written)        */
    RT_EUNSUPPORTED = 5   /* feature not supported by this build/device        */
} rt_status;

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* rt_last_error(void);

/* ------------------------------------------------------------------ scene */
typedef struct rt_scene rt_scene;

typedef struct {
    int64_t n_triangles;
    int32_t n_materials;
    int32_t bvh_depth;        /* deepest leaf of the LBVH (root = depth 0)    */
    int64_t n_nodes;          /* internal nodes (n_triangles - 1)             */
    int64_t device_bytes;     /* device memory held by the scene              */
    double build_ms;          /* device time of the last build                 */
    int32_t tuned_block;      /* launch configuration chosen by rt_tune (0 =   */
    int32_t tuned_deposit;    /* not tuned): workgroup size, deposit strategy, */
    int32_t tuned_refill;     /* wavefront refill threshold (lanes), launch    */
    int32_t tuned_order;      /* order (1 coherent patches, 2 lattice order)   */
    int32_t tuned_width;      /* and tree width (2 or 4)                       */
    float lo[3], hi[3];       /* bounds of the triangle AABB centres           */
} rt_scene_info;

/*
 * rt_build_scene -- build the device-resident scene and its LBVH
 * (Sec. "Scene Objects and Meshes": triangles with one radio material each).
 *   vertices     device float32 [n_vertices][3]
 *   triangles    device int32   [n_triangles][3]  vertex indices
 *   tri_material device int32   [n_triangles]     material index in [0, n_materials)
 * Hit ids reported by the library are indices into `triangles`.
 * The library copies what it needs; the inputs may be freed after return.
 * This call synchronises `stream` (it reads back validation flags).
 * Errors: RT_EINVAL for negative sizes, NULL pointers with n > 0, vertex
 * indices or material ids out of range, or non-finite vertex coordinates;
 * RT_ENOMEM; RT_EDEVICE.  Zero triangles is a valid (empty) scene.
 * Zero-area triangles are accepted and can never be hit.
 */
rt_status rt_build_scene(const float* vertices, int64_t n_vertices,
                         const int32_t* triangles, int64_t n_triangles,
                         const int32_t* tri_material, int32_t n_materials,
                         void* stream, rt_scene** out);

/* Release a scene (NULL is accepted).  Synchronises the device. */
rt_status rt_scene_destroy(rt_scene* scene);

/* Host-side description of a built scene. */
rt_status rt_scene_info_get(const rt_scene* scene, rt_scene_info* out);

/*
 * rt_scene_export -- copy the built acceleration structure to caller-owned
 * host memory, for structural checks of the builder (the LBVH is this
 * library's own design; the paper delegates intersection to its renderer).
 * Every buffer may be NULL to skip it:
 *   morton  uint64 [n_triangles]    63-bit Morton codes of the triangle AABB
 *                                   centres (21 bits per axis, one scale for
 *                                   all axes: 2^21 - 1 over the largest
 *                                   extent of the centres' box), in sorted
 *                                   (slot) order
 *   nodes   float  [n_nodes][16]    binary internal nodes, four float4 each:
 *                                   (L.lo.x, L.hi.x, L.lo.y, L.hi.y),
 *                                   (R.lo.x, R.hi.x, R.lo.y, R.hi.y),
 *                                   (L.lo.z, L.hi.z, R.lo.z, R.hi.z),
 *                                   (left ref, right ref, -, -) as int bits;
 *                                   a ref r >= 0 is an internal node, r < 0
 *                                   the leaf of triangle slot ~r; node 0 is
 *                                   the root
 *   wide    float  [n_wide][32]     4-wide nodes, eight float4 each: x_lo,
 *                                   x_hi, y_lo, y_hi, z_lo, z_hi of children
 *                                   0..3, then the four child refs as int bits
 *                                   (>= 0 wide node, < 0 leaf slot ~r,
 *                                   0x7fffffff empty), then unused; node 0 is
 *                                   the root
 *   tris    float  [n_triangles][12] triangles in slot order: (v0, original
 *                                   id bits), (v1, material bits), (v2, 0)
 *   n_wide  out (may be NULL): number of 4-wide nodes, 0 if the scene has no
 *           4-wide tree (call first with NULL buffers to size `wide`).
 * Synchronises `stream`.  Errors: RT_EINVAL for a NULL scene; RT_EDEVICE.
 */
rt_status rt_scene_export(const rt_scene* scene, uint64_t* morton, float* nodes, float* wide, float* tris,
                          int64_t* n_wide, void* stream);

/* ------------------------------------------------------- call parameters */
/*
 * Radio materials, device float32 arrays.  eps_r and sigma are the real
 * relative permittivity and the conductivity of eq. eta, indexed by material
 * (and, for batched calls, [n_samples][n_materials]).
 * thickness (optional, NULL = half-space walls): slab thickness d >= 0 in
 * metres per material.  Every interaction then uses the single-layer slab
 * coefficients of eq. fresnel_slab with eq. q_fresnel_slab (Sec.
 * "Single-Layer Slab") instead of the half-space ones of eq. fresnel_vac.
 * The array is read by the kernels of the call and must stay valid until it
 * completes; a negative or non-finite entry gives undefined results.  A tape
 * and rt_radio_map_backward take it (the backward needs the same array; the
 * sampling probabilities of refraction are held constant in the gradient);
 * rt_radio_map_batched takes it (one array shared by the material samples;
 * with refraction, one material sample and no gradients only).
 * scattering, xpd (optional, both or neither; NULL = no diffuse reflection):
 * scattering coefficient S in [0, 1] and cross-polarisation share K_x in
 * [0, 1] (eq. xpd) per material.  A hit on a material with S > 0 samples a
 * diffuse reflection with probability q(S) = S^2 A / (A + B) (A the
 * reflected and B the transmitted power share of the hit, B = 0 without
 * refraction; eq. path-solver-used-dist-event), specular reflection with
 * q(R) = (1 - S^2) A / (A + B) and coefficients times R = sqrt(1 - S^2)
 * (eq. R).  The diffuse ray leaves the hit point in a direction drawn
 * uniformly over the hemisphere of the incident side (polar cosine from
 * word 0 and azimuth from word 1 of the Philox4x32-10 block at counter
 * (ray index, l, 2), in the frame t1 = (a x n)/|a x n|, t2 = n x t1, a the
 * coordinate axis least aligned with the normal n), with the Lambertian
 * pattern (eq. lambertian_model): its field is the incident one in the
 * theta/phi bases of the two directions, mixed by the matrix of
 * eq. scattered_field with phases 2 pi times words 2 and 3, times
 * sqrt(2 cos(theta_s) S^2 Gamma^2 / q(S)).  One polarisation per call
 * (Gamma depends on the field): dual polarisation gives RT_EUNSUPPORTED, and
 * so does rt_radio_map_batched with several material samples or gradients.  A taped call is differentiable: the backward takes
 * the same scattering and xpd arrays.  Entries outside [0, 1] give
 * undefined results.
 * scatter_pattern (optional, needs scattering; NULL = Lambertian for every
 * material): device float32 [n_materials][4] = (kind, alpha_R, alpha_I,
 * Lambda) with kind 0 Lambertian (eq. lambertian_model), 1 directive
 * (eq. directive_model, lobe width alpha_R), 2 backscattering
 * (eq. backscattering_model, lobe widths alpha_R and alpha_I, share
 * Lambda); the diffuse factor 2 cos(theta_s) becomes 2 pi f_s.  alpha_R and
 * alpha_I are integers in [1, 64], Lambda in [0, 1]; other values give
 * undefined results.
 */
typedef struct {
    const float* eps_r;
    const float* sigma;
    const float* thickness;
    const float* scattering;
    const float* xpd;
    const float* scatter_pattern;
} rt_materials;

enum { RT_PATTERN_ISO = 0, RT_PATTERN_DIRECTIONAL = 1 };
enum { RT_POL_V = 0, RT_POL_H = 1, RT_POL_DUAL = 2 };

/*
 * Transmitter (host struct).  Orientation R = Rz(yaw) Ry(pitch) Rx(roll)
 * (eq. rotation).  Patterns, in local antenna coordinates:
 *   RT_PATTERN_ISO          G = 1
 *   RT_PATTERN_DIRECTIONAL  G(alpha) = (q+1) ((1 + cos alpha)/2)^q, alpha the
 *                           angle to the local +x axis (integrates to 4 pi).
 * pol: V puts C' = sqrt(G) theta_hat', H puts C' = sqrt(G) phi_hat'; DUAL
 * computes both, into two maps.
 */
typedef struct {
    double pos[3];
    double yaw, pitch, roll;
    int32_t pattern;
    float pattern_q;
    int32_t pol;
    /* Optional synthetic transmit array with a precoding vector (Sec.
     * "Handling Multiple Transmit Antennas"): rays start at `pos`; a ray of
     * departure direction k carries alpha = sum_i u_i exp(j 2 pi/lambda k.d_i)
     * (the array response vector, eq. path-solver-array-response-vector,
     * times the precoding vector) and its map weight is scaled by |alpha|^2.
     *   n_ant      number of elements; 0 = a single element at `pos`
     *   ant_pos    device float64 [n_ant][3]: element offsets d_i from `pos`
     *              in metres, global frame (not rotated with the antenna)
     *   precoding  device float32 [n_ant][2]: u_i as (re, im)
     * Both arrays are read by the kernels of the call and must stay valid
     * until it completes.  rt_radio_map_batched takes arrays, also with
     * material samples and gradients. */
    int32_t n_ant;
    const double* ant_pos;
    const float* precoding;
} rt_tx;

/*
 * Horizontal measurement plane z = z, W x H cells of dx x dy starting at
 * (x0, y0); cell (i, j) covers [x0 + i dx, x0 + (i+1) dx) x [y0 + j dy, ...)
 * and is stored at map[j * W + i] (row-major, j along +y).  The plane does
 * not interact with rays and is two-sided (Sec. "Radio Map Solver").
 */
typedef struct {
    double z, x0, y0, dx, dy;
    int32_t W, H;
} rt_plane;

enum { RT_ACCEL_BVH = 0, RT_ACCEL_BRUTE = 1, RT_ACCEL_BVH2 = 2, RT_ACCEL_BVH4 = 3 };
enum { RT_DEPOSIT_AUTO = 0, RT_DEPOSIT_ATOMIC = 1, RT_DEPOSIT_WAVE = 2 };

/*
 * SBR parameters (host struct).
 *   freq_hz     carrier frequency f (lambda = c0/f, omega = 2 pi f)
 *   n_rays      N_S: size of the Fibonacci lattice and normaliser of the estimator
 *   ray_begin, ray_end
 *               lattice indices traced by this call, [ray_begin, ray_end);
 *               ray_end <= 0 means N_S.  Disjoint sub-ranges of one lattice
 *               add up (with accumulate = 1) to the full map.
 *   max_depth   L: segments l = 0..L are traced (L reflections at most)
 *   accumulate  0: the map is overwritten; 1: contributions are added to it
 *   t_min       spawned rays accept hits at t > t_min (metres); the triangle
 *               just hit is always excluded
 *   accel       RT_ACCEL_BVH (tuned tree width), RT_ACCEL_BVH2 (binary LBVH),
 *               RT_ACCEL_BVH4 (4-wide tree collapsed from it), or
 *               RT_ACCEL_BRUTE (every triangle is tested with the same
 *               intersection test, for validation).  All four give
 *               identical hits.
 *   deposit     plane deposit strategy: AUTO (tuned), ATOMIC (one FP32 atomic
 *               per crossing) or WAVE (same-cell crossings of a wavefront are
 *               summed before one atomic)
 */
typedef struct {
    double freq_hz;
    int64_t n_rays;
    int64_t ray_begin, ray_end;
    int32_t max_depth;
    int32_t accumulate;
    float t_min;
    int32_t accel;
    int32_t deposit;
    int32_t block_size;   /* 0 = tuned default; else 64, 128, 256 or 512 */
    /* Early termination (Sec. "Practical Notes", eq. radio-map-solver-rr-prob),
     * applied before tracing every segment l >= max(rr_depth, 1):
     *   gain_threshold  > 0: drop the path when its path gain at the current
     *                   ray-tube length r, (lambda/(4 pi r))^2 ||E||^2, is
     *                   below it (biased); 0 = off
     *   rr_p_max        in (0, 1]: Russian roulette, keep the path with
     *                   p = min(||E||^2, rr_p_max) and divide its field by
     *                   sqrt(p) (unbiased); 0 = off
     *   seed            key of the per-ray random stream (Philox4x32-10 at
     *                   counter (ray index, l))
     * ||E||^2 is the distance-normalised gain of polarisation 0 (times
     * |alpha|^2 with a transmit array).  A taped call records the surviving
     * paths (a dropped path's tape ends at its last traced segment) for
     * rt_radio_map_backward.  rt_radio_map_batched takes it with one
     * material sample and no gradients (RT_EUNSUPPORTED otherwise). */
    int32_t rr_depth;
    float rr_p_max;
    float gain_threshold;
    uint32_t seed;
    /* Refraction (Sec. "Sampling Interaction Types"): 0 = specular
     * reflection only (q(R) = 1); 1 = at the end of every segment l that
     * hits a triangle one interaction is sampled, reflection with
     * q(R) = (|r_perp|^2 + |r_par|^2) / (|r_perp|^2 + |r_par|^2 + |t_perp|^2
     * + |t_par|^2), else transmission (eq. path-solver-used-dist-event with
     * no diffuse reflection or diffraction), from the draw at Philox4x32-10
     * counter (ray index, l, 1) with key (seed, 0); the field of the
     * sampled branch is divided by sqrt(q), the Pr(chi)^-1 factor of the
     * estimator.  A transmitted ray keeps its direction (Sec. "Interactions
     * with Scene Objects") and its TE/TM basis.  Needs materials.thickness
     * (RT_EINVAL otherwise).  A tape records the sampled branches; the
     * adjoint differentiates the sampled coefficients with q held constant.
     * rt_radio_map_batched takes it with one material sample and no
     * gradients (RT_EUNSUPPORTED otherwise). */
    int32_t refraction;
} rt_sbr_params;

/*
 * Optional per-segment records (device pointers, each may be NULL), indexed
 * [ray - ray_begin][l] with l = 0..L:
 *   hits     int32: id of the triangle that ends segment l, -1 if the
 *            segment escapes, -2 if it was not traced
 *   cells    int32: plane cell crossed by segment l (j*W + i), or -1
 *   weights  float: weight deposited by segment l (polarisation 0), or 0
 *   stats    uint64[5], accumulated (not reset): traced segments, plane
 *            crossings, BVH node visits, ray-triangle tests, traversal
 *            faults: stack overflows or references outside the tree, each of
 *            which ends that query (always 0: the spill area is sized from
 *            the tree depth, and a well-formed tree has no bad references)
 */
typedef struct {
    int32_t* hits;
    int32_t* cells;
    float* weights;
    unsigned long long* stats;
} rt_records;

/* --------------------------------------------------------------- forward */
typedef struct rt_tape rt_tape;

/*
 * rt_radio_map -- the SBR radio map (estimator eq. radio-map-solver-ci-all-2-
 * estimator, specular chains only).
 *   out_map   device float32 [H][W] (pol V or H) or [2][H][W] (RT_POL_DUAL)
 *   tape      NULL, or a tape from rt_tape_create for the same ray range and
 *             depth: records what rt_radio_map_backward needs
 *   records   NULL, or optional per-segment records (see rt_records)
 * Errors: RT_EINVAL (bad sizes, ranges, NULL map, tape of another shape),
 * RT_EOVERFLOW (a traversal stack overflowed; the map content is undefined),
 * RT_EDEVICE.
 */
rt_status rt_radio_map(const rt_scene* scene, rt_materials materials,
                       const rt_tx* tx, const rt_plane* plane,
                       const rt_sbr_params* params, float* out_map,
                       rt_tape* tape, const rt_records* records, void* stream);

/* ------------------------------------------------------------------ tape */
/*
 * A tape holds, per traced segment, the hit index, the crossed cell, the
 * direction and polarisation basis of the segment and the field transfer
 * matrix T (the per-bounce checkpoint).  Library-owned device memory.
 * rt_tape_bytes: bytes a tape for these params needs.
 */
size_t rt_tape_bytes(const rt_sbr_params* params);
rt_status rt_tape_create(const rt_sbr_params* params, rt_tape** out);
rt_status rt_tape_destroy(rt_tape* tape);

/*
 * rt_radio_map_backward -- vector-Jacobian product of the radio map.
 * Given grad_map = dLoss/dMap (device float32, same shape as out_map), writes
 *   grad_eps_r  device float32 [n_materials]  dLoss/d eps_r
 *   grad_sigma  device float32 [n_materials]  dLoss/d sigma
 *   grad_orient device float32 [3]            dLoss/d (yaw, pitch, roll)
 * (each may be NULL; non-NULL outputs are overwritten).  It replays the tape
 * filled by the rt_radio_map call with the same scene, materials, tx, plane
 * and params; it traces nothing.  Derivatives follow eq. fresnel_vac,
 * eq. eta (d eta/d eps_r = 1, d eta/d sigma = -j/(eps0 omega)) and
 * eq. rotation; with slab walls, eq. fresnel_slab (quotient and chain rules
 * through x = exp(-j q)); with refraction, the sampled branch (a transmitted
 * segment keeps its direction) with its probability held constant; with
 * Russian roulette, the surviving paths with their 1/sqrt(p) factors, p held
 * constant (the factor is recovered from the taped transfer matrices); with
 * diffuse reflection, eq. scattered_field with the direction and phases
 * redrawn from the forward's streams, q(S) held constant and Gamma^2
 * differentiated through both the coefficients and the incident field.  Partial
 * sums are reduced in a fixed order, so results are run-to-run
 * deterministic.
 * Errors: RT_EINVAL if the tape was not filled by a matching forward call
 * (same scene, material arrays including thickness, scattering and xpd,
 * transmitter, plane and parameters).
 */
rt_status rt_radio_map_backward(const rt_scene* scene, rt_materials materials,
                                const rt_tx* tx, const rt_plane* plane,
                                const rt_sbr_params* params, const rt_tape* tape,
                                const float* grad_map, float* grad_eps_r,
                                float* grad_sigma, float* grad_orient, void* stream);

/*
 * rt_radio_map_backward_noalloc -- rt_radio_map_backward for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as rt_radio_map_backward; the caller still provides the tape, the
 * upstream gradient and the outputs.  The per-block partial sums (512 blocks
 * x 19 FP64 values = 77,824 bytes, independent of the ray count and of the
 * number of materials, which are processed in chunks of 8) go to a static
 * device array, one per GPU, held until the process ends, instead of the
 * scene's workspace.  The call allocates nothing; its first call on a device
 * resolves that device's array (that device must be current).  Every call on
 * one GPU shares that array: calls that overlap in time on one GPU (other
 * streams, other threads) race and give wrong gradients; calls ordered on one
 * stream are safe.  Errors as rt_radio_map_backward, plus RT_EOVERFLOW if
 * the partial sums would not fit the array (they always do) and RT_EDEVICE
 * if the device index is 64 or above.
 */
rt_status rt_radio_map_backward_noalloc(const rt_scene* scene, rt_materials materials,
                                        const rt_tx* tx, const rt_plane* plane,
                                        const rt_sbr_params* params, const rt_tape* tape,
                                        const float* grad_map, float* grad_eps_r,
                                        float* grad_sigma, float* grad_orient, void* stream);

/* --------------------------------------------------------------- batched */
/*
 * rt_radio_map_batched -- many transmitters and/or many material samples in
 * one call ("radio maps for multiple sources in parallel", Sec. "Radio Map
 * Solver").
 *   materials   device float32 [n_samples][n_materials]
 *   n_samples   1..64 material samples
 *   txs         host [n_tx] transmitters, n_tx 1..4096 (pol V or H; DUAL is
 *               rejected)
 *   rays_per_tx host int64 [n_tx]: N_S of each transmitter's lattice
 *   params      n_rays, ray_begin and ray_end are ignored
 *   out_maps    device float32 [n_tx][n_samples][H][W]
 *   grad_maps   NULL (forward only) or device float32 [n_tx][n_samples][H][W]
 *               upstream gradients: the call then also returns the
 *               vector-Jacobian products
 *   grads       device float32 [n_tx][n_samples][2*n_materials + 3]
 *               (eps_r[m]..., sigma[m]..., yaw, pitch, roll), overwritten,
 *               required iff grad_maps != NULL
 * Every ray is traced once and serves all material samples.  Work over
 * (transmitter, ray) is scheduled from a device work counter by a persistent
 * kernel.
 * With one material sample and no gradients the call runs the
 * single-transmitter kernel over all transmitters and takes what
 * rt_radio_map takes: transmit arrays, materials.thickness, scattering, xpd
 * and scatter_pattern, and params' refraction, early termination and seed.
 * A ray draws from the random streams of its own lattice index, so each
 * transmitter's map is the one rt_radio_map gives for it.  Several material
 * samples or gradients share one traversal per ray, so they take only what
 * leaves the paths unchanged: transmit arrays and slab walls without
 * refraction (one thickness array for all samples); refraction, diffuse
 * reflection and early termination give RT_EUNSUPPORTED there, and so do
 * gradients with max_depth above 8 or more than 8 materials.  Out-of-range
 * counts give RT_EINVAL before any device work.
 */
rt_status rt_radio_map_batched(const rt_scene* scene, rt_materials materials,
                               int32_t n_samples, const rt_tx* txs,
                               const int64_t* rays_per_tx, int32_t n_tx,
                               const rt_plane* plane, const rt_sbr_params* params,
                               float* out_maps, const float* grad_maps,
                               float* grads, void* stream);

/* ------------------------------------------------------------- autotuner */
/*
 * rt_tune -- time the forward kernel variants (tree width, launch order,
 * workgroup size, deposit strategy, wavefront refill threshold) on this
 * scene, tx, plane and params, with about `n_probe_rays` rays taken from
 * eight sub-ranges spread over the lattice, and remember the fastest for
 * later calls on this scene (accel RT_ACCEL_BVH, deposit RT_DEPOSIT_AUTO,
 * block_size 0).
 * Writes the chosen block size and deposit strategy (host ints, may be NULL);
 * rt_scene_info_get reports the whole choice.
 * Launch order: by default each chunk of consecutive lattice indices is
 * launched sorted by azimuth, so that a wavefront starts on a small patch of
 * directions (results are unchanged up to FP32 summation order).
 * Synchronises `stream`; `scratch_map` is device float32 of the map's size
 * and is overwritten.
 */
rt_status rt_tune(rt_scene* scene, rt_materials materials, const rt_tx* tx,
                  const rt_plane* plane, const rt_sbr_params* params,
                  int64_t n_probe_rays, float* scratch_map, void* stream,
                  int32_t* chosen_block, int32_t* chosen_deposit);

/*
 * rt_set_launch_config -- apply a launch configuration reported earlier by
 * rt_scene_info_get after rt_tune (tree width 2 or 4, order 1 coherent or
 * 2 lattice, workgroup size, deposit strategy, refill threshold in lanes),
 * so that a caller can reuse a tuning result without timing again.  A zero
 * field selects the untuned default for that choice.  Results do not depend
 * on the configuration beyond FP32 summation order.  Host-only: no device
 * work, no synchronisation.
 * Errors: RT_EINVAL for a NULL scene, a value outside the ranges above, or
 * width 4 on a scene without a 4-wide tree (fewer than two triangles).
 */
rt_status rt_set_launch_config(rt_scene* scene, int32_t width, int32_t order,
                               int32_t block, int32_t deposit, int32_t refill);

#ifdef __cplusplus
}
#endif

#endif /* RTMAP_RT_H */
