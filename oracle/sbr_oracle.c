/*
 * sbr_oracle.c -- FP64 reference of the specular-only SBR radio map.
 *
 * TEST INFRASTRUCTURE.  This file is the correctness oracle of the project:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may build, load or call it.  The HIP library never links it, and the two
 * share no code, header, table or helper.
 *
 * It is deliberately plain and slow: one thread, double precision,
 * std C99 complex arithmetic, brute-force intersection against every
 * triangle, and a field representation that differs from the GPU path
 * (a complex 3-vector in global coordinates instead of a 2x2 transfer
 * matrix in per-ray local bases).
 *
 * What it computes (citations are to the Sionna RT technical report,
 * arXiv 2504.21719, v2.1):
 *   - ray directions on the spherical Fibonacci lattice
 *     (Sec. "Sampling Initial Ray Directions");
 *   - the transmitted field C_T = sqrt(G) F rotated into the global frame
 *     (App. A: eq. rotation, eq. theta_phi_prime, eq. F_prime_2_F, eq. C);
 *   - closest hit per segment by brute force (Sec. "Generating Candidates by
 *     SBR": intersect, deactivate on a miss);
 *   - specular reflection: reflected direction (eq. path-solver-scatter-dir,
 *     eq. reflected_refracted_vectors), TE/TM bases (eq. fresnel_in_vectors,
 *     eq. fresnel_out_vectors), vacuum Fresnel coefficients (eq. fresnel_vac)
 *     with the complex relative permittivity of eq. eta;
 *   - optional finite-thickness walls: the single-layer slab coefficients
 *     eq. fresnel_slab with eq. q_fresnel_slab (Sec. "Single-Layer Slab")
 *     replace the half-space ones, and optional refraction: at every hit one
 *     interaction type, reflection or transmission, is sampled with the
 *     probabilities of eq. path-solver-used-dist-event and the field is
 *     divided by the square root of the probability (the Pr(chi)^-1 factor of
 *     the estimator); transmitted rays keep their direction (Sec.
 *     "Interactions with Scene Objects");
 *   - optional diffuse reflection (Sec. "Definition of Radio Map",
 *     App. "Diffuse Reflection"): a material with scattering coefficient
 *     S > 0 scatters with probability q(S) of eq. path-solver-used-dist-event
 *     into a direction drawn uniformly over the hemisphere of the incident
 *     side (solid angle 2 pi), with the Lambertian, directive or
 *     backscattering pattern (eq. lambertian_model, eq. directive_model,
 *     eq. backscattering_model), the reflected power ratio Gamma^2 and the
 *     cross-polarisation matrix of eq. scattered_field with random phases;
 *     the specular coefficients are multiplied by R = sqrt(1 - S^2) (eq. R);
 *   - an optional synthetic transmit array with a precoding vector
 *     (Sec. "Handling Multiple Transmit Antennas"): the launch field of a ray
 *     is multiplied by alpha = a_tx^T u_P of its departure direction;
 *   - the Monte-Carlo radio-map estimator eq. radio-map-solver-ci-all-2-
 *     estimator for specular chains only (no diffuse reflection, so n_S = 0 and
 *     the interaction probability is 1), in which the squared ray-tube length
 *     r^2 of the change of variables dA = r^2/|n^T k| d(omega) cancels the
 *     1/r^2 of the spherical spreading of the path gain eq. radio-map-solver-
 *     path-gain; every depth l = 0..L that crosses the plane contributes.
 *
 * Parity aids: per-segment hit ids, per-segment ambiguity flags (edge, tie,
 * grazing, near-origin, polar ray) and per-crossing records.
 *
 * Gradients: forward-mode tangents of the field w.r.t. (eps_r[m], sigma[m]
 * for every material, yaw, pitch, roll).  Fresnel derivatives are taken by the
 * quotient rule on eq. fresnel_vac with d(eta)/d(eps_r) = 1 and
 * d(eta)/d(sigma) = -j/(eps0 omega) from eq. eta; transmitter-angle
 * derivatives use dual numbers through eq. rotation and eq. theta_phi_prime.
 * Sampling probabilities (interaction type, Russian roulette) are held
 * constant.  At a diffuse point the tangent includes the change of Gamma^2,
 * which depends on the coefficients and on the incident field itself.
 *
 * Readings where the paper is silent (stated once here, used throughout):
 *   - by default only specular reflection is enabled, so q(R) = 1 and
 *     Pr(chi) = 1; with refraction, diffuse reflection and diffraction stay
 *     off (S = 0, R = 1, q(D) = 0), so q(T) = 1 - q(R);
 *   - half-space (vacuum-incidence) Fresnel coefficients unless a slab
 *     thickness is given; a transmitted ray keeps the TE/TM basis of the
 *     incident side (k_t = k_i gives e_t,par = e_i,par in
 *     eq. fresnel_out_vectors);
 *   - the interaction at the end of segment l of ray n reflects iff the
 *     uniform draw at Philox counter (n, l, 1) is below q(R), scatters
 *     diffusely iff it is below q(R) + q(S), and is transmitted otherwise;
 *     without refraction the transmission share is 0;
 *   - a diffuse reflection takes its four draws from Philox counter (n, l, 2):
 *     cos(theta_s) = u0, azimuth 2 pi u1 in the frame (t1, t2, n) with
 *     t1 = (a x n)/|a x n|, a the coordinate axis least aligned with n, and
 *     t2 = n x t1; the phases chi_1 = 2 pi u2, chi_2 = 2 pi u3.  The field
 *     components refer to theta_hat and phi_hat of the incident and the
 *     scattered direction (phi = 0 on the z axis).  With the change of
 *     variables of eq. radio-map-solver-ci-all-2 the footprint dA, r^2 and
 *     cos(theta_i) cancel, so the scattered distance-normalised field is the
 *     incident one times sqrt(2 pi f_s S^2 Gamma^2 / q(S)) (for the
 *     Lambertian pattern 2 pi f_s = 2 cos(theta_s)), and the ray-tube length
 *     starts again at 0 (gain thresholding uses the current tube);
 *   - c0 = 299792458 m/s, eps0 = 8.8541878128e-12 F/m, phi_g = (1+sqrt 5)/2;
 *   - the plane is two-sided and non-occluding; a segment contributes iff
 *     0 < t_plane < t_hit (t_hit = inf on a miss); cells are half-open;
 *   - segments l = 0..L are traced; segment L is traced to its first hit (or
 *     infinity) for the crossing test and is not reflected;
 *   - spawned rays exclude the primitive just hit and accept t > t_min;
 *   - equal-t ties go to the smallest primitive index;
 *   - the normal is flipped toward the incident side;
 *   - at normal incidence the TE direction is k x a, with a the coordinate
 *     axis least aligned with k;
 *   - the complex square root is the principal branch.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_C0 299792458.0
#define OR_EPS0 8.8541878128e-12
#define OR_PI 3.14159265358979323846

/* flag bits per (ray, segment) */
#define OR_FLAG_EDGE 1u
#define OR_FLAG_TIE 2u
#define OR_FLAG_GRAZING 4u
#define OR_FLAG_NEAR 8u
#define OR_FLAG_POLAR 16u
#define OR_FLAG_TERM 32u     /* early-termination decision within 1e-5 of its threshold */
#define OR_FLAG_CHOICE 64u   /* interaction-type draw within 1e-5 of a class boundary */

#define OR_MAX_PARAMS 64
#define OR_MAX_DEPTH 64   /* largest max_depth L (L + 1 segments), as the library accepts */

/* ---------------------------------------------------------------- vectors */
typedef struct { double x, y, z; } vec3;
typedef struct { cplx x, y, z; } cvec3;

static vec3 mk(double x, double y, double z) { vec3 r = {x, y, z}; return r; }
static vec3 vsub(vec3 a, vec3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static vec3 vadd(vec3 a, vec3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static vec3 vscale(vec3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double vdot(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec3 vcross(vec3 a, vec3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vnorm(vec3 a) { return sqrt(vdot(a, a)); }
static vec3 vunit(vec3 a) { return vscale(a, 1.0 / vnorm(a)); }

static cvec3 cv_zero(void) { cvec3 r = {0, 0, 0}; return r; }
static cplx cv_dot_real(vec3 e, cvec3 E) { return e.x * E.x + e.y * E.y + e.z * E.z; }
static cvec3 cv_axpy(cvec3 acc, cplx a, vec3 e) {
    acc.x += a * e.x; acc.y += a * e.y; acc.z += a * e.z; return acc;
}
static cvec3 cv_scale(cvec3 E, cplx a) { cvec3 r = {a * E.x, a * E.y, a * E.z}; return r; }
static double cv_norm2(cvec3 E) {
    return creal(E.x * conj(E.x) + E.y * conj(E.y) + E.z * conj(E.z));
}
/* Re(E^H dE) */
static double cv_re_inner(cvec3 E, cvec3 dE) {
    return creal(conj(E.x) * dE.x + conj(E.y) * dE.y + conj(E.z) * dE.z);
}

/* ------------------------------------------------ one specular interaction */
/* eq. fresnel_vac: r_perp and r_par at incidence cos(theta_1) = c on a
 * medium of relative permittivity eta (vacuum on the incident side), their
 * eta-derivatives (quotient rule, ds/deta = 1/(2 s)), and
 * s = sqrt(eta - sin^2 theta_1) (principal branch). */
static void fresnel_half_space(cplx eta, double c, cplx* s_out, cplx* r_perp, cplx* r_par,
                               cplx* dr_perp, cplx* dr_par)
{
    double s2 = 1.0 - c * c;                  /* sin^2(theta_1) */
    cplx s = csqrt(eta - s2);
    cplx den_p = c + s, den_l = eta * c + s;
    *r_perp = (c - s) / den_p;
    *r_par = (eta * c - s) / den_l;
    cplx ds = 1.0 / (2.0 * s);
    *dr_perp = ((-ds) * den_p - (c - s) * ds) / (den_p * den_p);
    *dr_par = ((c - ds) * den_l - (eta * c - s) * (c + ds)) / (den_l * den_l);
    *s_out = s;
}

/* eq. fresnel_in_vectors, eq. fresnel_out_vectors: the TE direction e_perp
 * (any unit vector normal to k at normal incidence: k x a, a the axis least
 * aligned with k), the incident TM direction e_par = e_perp x k, the
 * reflected direction k_r and its TM direction er_par = e_perp x k_r.  The
 * normal n points to the incident side. */
static void reflection_bases(vec3 k, vec3 nrm, vec3* e_perp_out, vec3* e_par, vec3* kr_out, vec3* er_par)
{
    vec3 kn = vcross(k, nrm);
    vec3 e_perp;
    if (vnorm(kn) > 1e-12) {
        e_perp = vunit(kn);
    } else {
        double ax = fabs(k.x), ay = fabs(k.y), az = fabs(k.z);
        vec3 a = (ax <= ay && ax <= az) ? mk(1, 0, 0) : (ay <= az ? mk(0, 1, 0) : mk(0, 0, 1));
        e_perp = vunit(vcross(k, a));
    }
    *e_par = vcross(e_perp, k);
    vec3 kr = vsub(k, vscale(nrm, 2.0 * vdot(k, nrm)));
    kr = vunit(kr);
    *er_par = vunit(vcross(e_perp, kr));
    *e_perp_out = e_perp;
    *kr_out = kr;
}

/* The field leaving an interaction (eq. fresnel_out_vectors): the TE part
 * e_perp^T E scaled by c_perp along e_perp, the TM part e_par^T E scaled by
 * c_par along out_par (real basis vectors, no conjugation), both times
 * inv_sqrt_q. */
static cvec3 specular_field(cvec3 E, vec3 e_perp, vec3 e_par, vec3 out_par, cplx c_perp, cplx c_par,
                            double inv_sqrt_q)
{
    cplx a_perp = cv_dot_real(e_perp, E);
    cplx a_par = cv_dot_real(e_par, E);
    cvec3 En = cv_zero();
    En = cv_axpy(En, c_perp * a_perp * inv_sqrt_q, e_perp);
    En = cv_axpy(En, c_par * a_par * inv_sqrt_q, out_par);
    return En;
}

/* ------------------------------------------------------- dual numbers (3) */
/* value + derivatives w.r.t. (yaw, pitch, roll) */
typedef struct { double v, d[3]; } dual;

static dual dc(double v) { dual r; r.v = v; r.d[0] = r.d[1] = r.d[2] = 0; return r; }
static dual dvar(double v, int i) { dual r = dc(v); r.d[i] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < 3; i++) r.d[i] = a.d[i] + b.d[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < 3; i++) r.d[i] = a.d[i] - b.d[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < 3; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static dual dneg(dual a) { dual r; r.v = -a.v; for (int i = 0; i < 3; i++) r.d[i] = -a.d[i]; return r; }
static dual dfun(dual a, double f, double fp) { dual r; r.v = f; for (int i = 0; i < 3; i++) r.d[i] = fp * a.d[i]; return r; }
static dual dsin(dual a) { return dfun(a, sin(a.v), cos(a.v)); }
static dual dcos(dual a) { return dfun(a, cos(a.v), -sin(a.v)); }
static dual dacos(dual a) {
    double s = sqrt(fmax(0.0, 1.0 - a.v * a.v));
    return dfun(a, acos(fmax(-1.0, fmin(1.0, a.v))), s > 0 ? -1.0 / s : 0.0);
}
static dual datan2(dual y, dual x) {
    dual r; double q = x.v * x.v + y.v * y.v;
    r.v = atan2(y.v, x.v);
    for (int i = 0; i < 3; i++) r.d[i] = q > 0 ? (x.v * y.d[i] - y.v * x.d[i]) / q : 0.0;
    return r;
}
static dual dpow(dual a, double p) {
    double f = pow(a.v, p);
    double fp = (a.v > 0) ? p * pow(a.v, p - 1.0) : 0.0;
    return dfun(a, f, fp);
}
static dual dsqrt(dual a) { double s = sqrt(fmax(0.0, a.v)); return dfun(a, s, s > 0 ? 0.5 / s : 0.0); }

/* ----------------------------------------------------------------- inputs */
typedef struct {
    double pos[3];
    double yaw, pitch, roll;
    int32_t pattern;     /* 0 isotropic, 1 directional (q) */
    double q;
    int32_t pol;         /* 0 V, 1 H, 2 dual (V and H) */
    int32_t n_ant;       /* synthetic transmit array: number of elements, 0 = none */
    const double* ant_pos;   /* [n_ant][3] element offsets from pos (m, global frame) */
    const double* precoding; /* [n_ant][2] complex precoding vector u_P (re, im) */
} or_tx;

typedef struct {
    double z, x0, y0, dx, dy;
    int32_t W, H;
} or_plane;

typedef struct {
    double freq;
    int64_t n_rays;
    int32_t max_depth;
    double t_min;
    int32_t rr_depth;       /* early termination before every segment l >= rr_depth */
    double rr_p_max;        /* Russian roulette: maximum keep probability, 0 = off */
    double gain_threshold;  /* gain thresholding: path-gain floor, 0 = off */
    uint32_t seed;          /* key of the random stream */
    int32_t refraction;     /* 1: sample reflection or transmission at every hit */
} or_params;

typedef struct {
    /* all outputs optional (NULL) */
    double* map;          /* [npol][H][W], accumulated into                  */
    int64_t* counts;      /* [H][W] crossings, accumulated into              */
    int32_t* hits;        /* [n_rays_run][L+1]                              */
    uint8_t* flags;       /* [n_rays_run][L+1]                              */
    int64_t rec_cap;      /* capacity of the crossing-record arrays          */
    int64_t rec_n;        /* out: number of crossings (may exceed rec_cap)  */
    int64_t* rec_ray;
    int32_t* rec_depth;
    int32_t* rec_cell;
    double* rec_w;        /* weight of polarisation 0                        */
    double* rec_border;   /* distance to the nearest decision boundary (m)   */
    double* rec_len;      /* unfolded length from the source (m)             */
    const double* grad_map; /* [npol][H][W] upstream gradient, or NULL       */
    double* grad;         /* [2*n_mat+3] accumulated: eps_r[m], sigma[m], yaw, pitch, roll */
    const int32_t* replay_hits; /* [n_rays_run][L+1]: force these hits (no search) */
    int64_t tri_tests;    /* out: number of ray-triangle tests */
    int64_t segments;     /* out: number of traced segments */
} or_out;

/* ------------------------------------------------------- random numbers */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): a counter-based generator.  Each of the ten
 * rounds multiplies words 0 and 2 by two fixed odd constants, keeps the low
 * halves, and XORs the high halves with the other two words and the round
 * key; the key is advanced by two Weyl constants between rounds. */
void or_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in [0, 1) for ray n, index l and stream s: the top 24 bits of the
 * first output word of Philox4x32-10 at counter (n_lo, n_hi, l, s) with key
 * (seed, 0), exactly representable in single precision.  Stream 0 is early
 * termination before segment l, stream 1 the interaction type at the end of
 * segment l. */
static double rr_uniform(uint32_t seed, int64_t n, int l, uint32_t stream)
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)n & 0xffffffffu), (uint32_t)((uint64_t)n >> 32), (uint32_t)l, stream};
    uint32_t key[2] = {seed, 0u};
    uint32_t out[4];
    or_philox4x32(ctr, key, out);
    return (double)(out[0] >> 8) * (1.0 / 16777216.0);
}

/* The four uniforms of one Philox4x32-10 block at counter (n_lo, n_hi, l,
 * stream), key (seed, 0), each from the top 24 bits of its word. */
static void uniform4(uint32_t seed, int64_t n, int l, uint32_t stream, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)n & 0xffffffffu), (uint32_t)((uint64_t)n >> 32), (uint32_t)l, stream};
    uint32_t key[2] = {seed, 0u};
    uint32_t out[4];
    or_philox4x32(ctr, key, out);
    for (int i = 0; i < 4; i++) u[i] = (double)(out[i] >> 8) * (1.0 / 16777216.0);
}

/* theta_hat and phi_hat of direction k (eq. spherical_vecs); phi = 0 on the
 * z axis. */
static void sph_basis(vec3 k, vec3* th, vec3* ph)
{
    double rho = sqrt(k.x * k.x + k.y * k.y);
    double cp = rho > 0.0 ? k.x / rho : 1.0, sp = rho > 0.0 ? k.y / rho : 0.0;
    *th = mk(k.z * cp, k.z * sp, -rho);
    *ph = mk(-sp, cp, 0.0);
}

/* Scattering pattern f_s (App. "Diffuse Reflection"): pp = (kind, alpha_R,
 * alpha_I, Lambda) with kind 0 Lambertian (eq. lambertian_model), 1
 * directive (eq. directive_model), 2 backscattering
 * (eq. backscattering_model); n is the unit normal on the incident side,
 * ki the incident and ks the scattered direction, kr the specular one. */
static double lobe_norm(int alpha, double ci)
{
    /* F_alpha(theta_i) = 2^-alpha sum_k C(alpha, k) I_k, with
     * I_k = 2 pi/(k+1) (k even) or 2 pi/(k+1) cos(theta_i) sum_{w <= (k-1)/2}
     * C(2w, w) sin^{2w}(theta_i) / 2^{2w} (k odd) */
    double s2 = fmax(0.0, 1.0 - ci * ci), F = 0.0, binom = 1.0;
    for (int k = 0; k <= alpha; k++) {
        if (k > 0) binom = binom * (double)(alpha - k + 1) / (double)k;
        double Ik = 2.0 * OR_PI / (double)(k + 1);
        if (k % 2 == 1) {
            double sum = 0.0, cw = 1.0, p = 1.0;
            for (int w = 0; w <= (k - 1) / 2; w++) {
                if (w > 0) cw = cw * (double)(2 * w) * (double)(2 * w - 1) / ((double)w * (double)w);
                sum += cw * p / pow(4.0, (double)w);
                p *= s2;
            }
            Ik *= ci * sum;
        }
        F += binom * Ik;
    }
    return F / pow(2.0, (double)alpha);
}

static double scatter_pattern(const double* pp, vec3 ki, vec3 ks, vec3 n, vec3 kr)
{
    int kind = pp ? (int)pp[0] : 0;
    if (kind == 0) return vdot(n, ks) / OR_PI;
    int aR = (int)pp[1], aI = (int)pp[2];
    double lam = kind == 1 ? 1.0 : pp[3];
    double ci = -vdot(ki, n);
    double num = lam * pow(0.5 * (1.0 + vdot(kr, ks)), (double)aR);
    double F = lam * lobe_norm(aR, ci);
    if (kind == 2) {
        num += (1.0 - lam) * pow(0.5 * (1.0 - vdot(ki, ks)), (double)aI);
        F += (1.0 - lam) * lobe_norm(aI, ci);
    }
    return num / F;
}

/* f_s for tests: pp as above, directions as 3-vectors. */
double or_scatter_pattern(const double* pp, const double* ki, const double* ks, const double* n)
{
    vec3 vi = mk(ki[0], ki[1], ki[2]), vs = mk(ks[0], ks[1], ks[2]), vn = mk(n[0], n[1], n[2]);
    vec3 kr = vsub(vi, vscale(vn, 2.0 * vdot(vi, vn)));
    return scatter_pattern(pp, vi, vs, vn, kr);
}

/* ------------------------------------------------- synthetic transmit array */
/* Sec. "Handling Multiple Transmit Antennas": paths start at the array centre;
 * element i adds the phase of the array response vector
 * (eq. path-solver-array-response-vector), exp(j 2 pi/lambda k^T d_i), and
 * the precoded array radiates alpha = a_tx^T u_P times the single-element
 * field, so a path contributes ||E alpha||^2 to the map. */
static cplx array_alpha(const or_tx* tx, vec3 k, double lam)
{
    if (tx->n_ant <= 0) return 1.0;
    cplx alpha = 0.0;
    for (int32_t i = 0; i < tx->n_ant; i++) {
        const double* d = tx->ant_pos + 3 * (int64_t)i;
        double phase = 2.0 * OR_PI / lam * (k.x * d[0] + k.y * d[1] + k.z * d[2]);
        cplx u = tx->precoding[2 * (int64_t)i] + I * tx->precoding[2 * (int64_t)i + 1];
        alpha += u * cexp(I * phase);
    }
    return alpha;
}

/* ------------------------------------------------------------- slab */
/* Single-layer slab (Sec. "Single-Layer Slab", eq. fresnel_slab): with
 * x = exp(-j q) and q = (2 pi d / lambda) s, s = sqrt(eta - sin^2 theta_1)
 * (eq. q_fresnel_slab), each half-space coefficient r' of eq. fresnel_vac
 * becomes r = r' (1 - x^2) / (1 - r'^2 x^2), and the slab passes
 * t = (1 - r'^2) x / (1 - r'^2 x^2).  k_d = 2 pi d / lambda.  The r's are
 * replaced in place. */
static void slab(cplx s, double k_d, cplx* r_perp, cplx* r_par, cplx* t_perp, cplx* t_par)
{
    cplx x1 = cexp(-I * (k_d * s)), x2 = x1 * x1;
    cplx rp2 = *r_perp * *r_perp, rl2 = *r_par * *r_par;
    *t_perp = (1.0 - rp2) * x1 / (1.0 - rp2 * x2);
    *t_par = (1.0 - rl2) * x1 / (1.0 - rl2 * x2);
    *r_perp = *r_perp * (1.0 - x2) / (1.0 - rp2 * x2);
    *r_par = *r_par * (1.0 - x2) / (1.0 - rl2 * x2);
}

/* Derivatives of the slab coefficients of one polarisation with respect to
 * eta, by the quotient and chain rules: r = r' (1 - x^2) / D and
 * t = (1 - r'^2) x / D with D = 1 - r'^2 x^2, x = exp(-j k_d s),
 * dx/d(eta) = -j k_d x / (2 s), and dr'/d(eta) = dr1 of the half-space
 * coefficient r1. */
static void slab_deriv(cplx s, double k_d, cplx r1, cplx dr1, cplx* dr, cplx* dt)
{
    cplx x = cexp(-I * (k_d * s)), x2 = x * x;
    cplx dx = -I * k_d * x / (2.0 * s);
    cplx D = 1.0 - r1 * r1 * x2;
    cplx dD = -(2.0 * r1 * dr1 * x2 + 2.0 * r1 * r1 * x * dx);
    cplx r = r1 * (1.0 - x2) / D, t = (1.0 - r1 * r1) * x / D;
    *dr = (dr1 * (1.0 - x2) - 2.0 * r1 * x * dx - r * dD) / D;
    *dt = (-2.0 * r1 * dr1 * x + (1.0 - r1 * r1) * dx - t * dD) / D;
}

/* ------------------------------------------------------ lattice and launch */
/* Spherical Fibonacci lattice (Sec. "Sampling Initial Ray Directions"). */
void or_fibonacci(int64_t n, int64_t N, double* theta, double* phi)
{
    if (N == 1) { *theta = OR_PI / 2; *phi = OR_PI; return; }
    double u = 1.0 - 2.0 * (double)n / (double)(N - 1);
    *theta = acos(u);
    /* frac(n / phi_g) = frac(n (phi_g - 1)), evaluated in extended precision */
    long double g1 = (sqrtl(5.0L) - 1.0L) / 2.0L;
    long double x = (long double)n * g1;
    long double fr = x - floorl(x);
    *phi = 2.0 * OR_PI * (double)fr;
}

static vec3 lattice_dir(int64_t n, int64_t N)
{
    double th, ph;
    or_fibonacci(n, N, &th, &ph);
    double u = (N == 1) ? 0.0 : 1.0 - 2.0 * (double)n / (double)(N - 1);
    double st = sqrt(fmax(0.0, (1.0 - u) * (1.0 + u)));
    return mk(st * cos(ph), st * sin(ph), u);
}

/* R(yaw, pitch, roll) = Rz(yaw) Ry(pitch) Rx(roll), eq. rotation, with duals */
static void rotation_dual(double yaw, double pitch, double roll, dual R[3][3])
{
    dual a = dvar(yaw, 0), b = dvar(pitch, 1), g = dvar(roll, 2);
    dual ca = dcos(a), sa = dsin(a), cb = dcos(b), sb = dsin(b), cg = dcos(g), sg = dsin(g);
    dual Rz[3][3] = {{ca, dneg(sa), dc(0)}, {sa, ca, dc(0)}, {dc(0), dc(0), dc(1)}};
    dual Ry[3][3] = {{cb, dc(0), sb}, {dc(0), dc(1), dc(0)}, {dneg(sb), dc(0), cb}};
    dual Rx[3][3] = {{dc(1), dc(0), dc(0)}, {dc(0), cg, dneg(sg)}, {dc(0), sg, cg}};
    dual T[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            dual s = dc(0);
            for (int k = 0; k < 3; k++) s = dadd(s, dmul(Rz[i][k], Ry[k][j]));
            T[i][j] = s;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            dual s = dc(0);
            for (int k = 0; k < 3; k++) s = dadd(s, dmul(T[i][k], Rx[k][j]));
            R[i][j] = s;
        }
}

/*
 * Transmitted field in global coordinates for direction k (a real 3-vector,
 * with derivatives w.r.t. yaw/pitch/roll).  The local direction is u = R^T k
 * (eq. theta_phi_prime); the local pattern C' = (C_theta', C_phi') multiplies
 * the local spherical unit vectors (eq. spherical_vecs) and the vector is
 * rotated back by R, which is eq. F_prime_2_F written as a 3-vector.
 * pol_index: 0 -> C' = sqrt(G) theta_hat', 1 -> C' = sqrt(G) phi_hat'.
 */
static void launch_field(vec3 k, const or_tx* tx, int pol_index, dual E[3])
{
    dual R[3][3];
    rotation_dual(tx->yaw, tx->pitch, tx->roll, R);
    double kk[3] = {k.x, k.y, k.z};
    dual u[3];
    for (int i = 0; i < 3; i++) {           /* u = R^T k */
        dual s = dc(0);
        for (int j = 0; j < 3; j++) s = dadd(s, dmul(R[j][i], dc(kk[j])));
        u[i] = s;
    }
    dual th = dacos(u[2]);
    dual ph = datan2(u[1], u[0]);
    dual ct = dcos(th), st = dsin(th), cp = dcos(ph), sp = dsin(ph);
    dual thv[3] = {dmul(ct, cp), dmul(ct, sp), dneg(st)};
    dual phv[3] = {dneg(sp), cp, dc(0)};
    dual amp;
    if (tx->pattern == 1) {
        /* G(alpha) = (q+1) ((1 + cos alpha)/2)^q, alpha = angle to local +x */
        dual half = dmul(dadd(dc(1.0), u[0]), dc(0.5));
        amp = dsqrt(dmul(dc(tx->q + 1.0), dpow(half, tx->q)));
    } else {
        amp = dc(1.0);
    }
    dual f[3];
    for (int i = 0; i < 3; i++) f[i] = dmul(amp, pol_index == 0 ? thv[i] : phv[i]);
    for (int i = 0; i < 3; i++) {           /* E = R f */
        dual s = dc(0);
        for (int j = 0; j < 3; j++) s = dadd(s, dmul(R[i][j], f[j]));
        E[i] = s;
    }
}

/* --------------------------------------------------------- intersection */
typedef struct {
    const float* V; const int32_t* F; int64_t n_tri;
} or_mesh;

static void tri_verts(const or_mesh* m, int64_t t, vec3* a, vec3* b, vec3* c)
{
    const int32_t* f = m->F + 3 * t;
    const float* p0 = m->V + 3 * (int64_t)f[0];
    const float* p1 = m->V + 3 * (int64_t)f[1];
    const float* p2 = m->V + 3 * (int64_t)f[2];
    *a = mk(p0[0], p0[1], p0[2]);
    *b = mk(p1[0], p1[1], p1[2]);
    *c = mk(p2[0], p2[1], p2[2]);
}

/* Moeller-Trumbore in double: returns 1 if the supporting plane is hit at
 * finite t, with barycentrics (u, v) and t; inside-ness is decided by caller. */
static int tri_plane_hit(vec3 o, vec3 k, vec3 a, vec3 b, vec3 c, double* t, double* bu, double* bv)
{
    vec3 e1 = vsub(b, a), e2 = vsub(c, a);
    vec3 p = vcross(k, e2);
    double det = vdot(e1, p);
    if (det == 0.0 || !isfinite(det)) return 0;
    double inv = 1.0 / det;
    vec3 s = vsub(o, a);
    double u = vdot(s, p) * inv;
    vec3 q = vcross(s, e1);
    double v = vdot(k, q) * inv;
    *t = vdot(e2, q) * inv;
    *bu = u; *bv = v;
    return 1;
}

typedef struct {
    double t; int64_t prim; double t2; uint8_t flags;
} hit_info;

static hit_info closest_hit(const or_mesh* m, vec3 o, vec3 k, int64_t last, double t_min, int64_t* tests)
{
    hit_info h = {INFINITY, -1, INFINITY, 0};
    double t_edge = INFINITY;   /* smallest t of a triangle hit/missed within 1e-5 of an edge */
    double t_any = INFINITY;    /* smallest positive t of any (nearly) inside triangle */
    for (int64_t i = 0; i < m->n_tri; i++) {
        if (i == last) continue;
        vec3 a, b, c;
        tri_verts(m, i, &a, &b, &c);
        double t, u, v;
        (*tests)++;
        if (!tri_plane_hit(o, k, a, b, c, &t, &u, &v)) continue;
        double w = 1.0 - u - v;
        double mb = fmin(u, fmin(v, w));
        if (t > 0.0 && mb > -1e-5 && t < t_any) t_any = t;
        if (!(t > t_min)) continue;
        if (fabs(mb) < 1e-5 && t < t_edge) t_edge = t;
        if (mb < 0.0) continue;
        if (t < h.t || (t == h.t && i < h.prim)) {
            h.t2 = h.t;
            h.t = t;
            h.prim = i;
        } else if (t < h.t2) {
            h.t2 = t;
        }
    }
    if (isfinite(t_edge) && t_edge <= h.t * (1.0 + 1e-6)) h.flags |= OR_FLAG_EDGE;
    if (h.prim >= 0 && h.t2 <= h.t * (1.0 + 1e-5)) h.flags |= OR_FLAG_TIE;
    if (t_any < 1e-2) h.flags |= OR_FLAG_NEAR;
    return h;
}

/* ------------------------------------------------------------- main loop */
/*
 * or_radio_map: trace rays [ray_begin, ray_end) of an N_S-ray lattice (or the
 * explicit list ray_ids[0..n_ids) when ray_ids != NULL) and accumulate the
 * radio map and the optional parity / gradient outputs.
 * Returns 0 on success, nonzero on invalid arguments.
 */
int or_radio_map(const float* V, int64_t n_v, const int32_t* F, int64_t n_tri,
                 const int32_t* tri_mat, int32_t n_mat,
                 const double* eps_r, const double* sigma, const double* thickness,
                 const double* scattering, const double* xpd, const double* pattern,
                 const or_tx* tx, const or_plane* pl, const or_params* prm,
                 const int64_t* ray_ids, int64_t n_ids, int64_t ray_begin, int64_t ray_end,
                 or_out* out)
{
    if (prm->n_rays < 1 || prm->max_depth < 0 || prm->max_depth > OR_MAX_DEPTH) return 1;
    if (pl->W < 1 || pl->H < 1 || !(pl->dx > 0) || !(pl->dy > 0)) return 1;
    if (n_mat < 1 || 2 * n_mat + 3 > OR_MAX_PARAMS) return 1;
    if (prm->refraction && !thickness) return 1;
    if (thickness) {
        for (int32_t i = 0; i < n_mat; i++)
            if (!(thickness[i] >= 0.0)) return 1;
    }
    if (scattering) {
        for (int32_t i = 0; i < n_mat; i++)
            if (!(scattering[i] >= 0.0 && scattering[i] <= 1.0) || !(xpd && xpd[i] >= 0.0 && xpd[i] <= 1.0))
                return 1;
        if (tx->pol == 2) return 1;                 /* Gamma depends on the field */
        if (pattern)
            for (int32_t i = 0; i < n_mat; i++) {
                const double* pp = pattern + 4 * (int64_t)i;
                if (!(pp[0] == 0.0 || pp[0] == 1.0 || pp[0] == 2.0)) return 1;
                if (pp[0] != 0.0 && !(pp[1] >= 1.0 && pp[1] <= 64.0 && pp[1] == floor(pp[1]))) return 1;
                if (pp[0] == 2.0 && !(pp[2] >= 1.0 && pp[2] <= 64.0 && pp[2] == floor(pp[2]) &&
                                      pp[3] >= 0.0 && pp[3] <= 1.0)) return 1;
            }
    }
    for (int64_t i = 0; i < n_tri; i++) {
        for (int j = 0; j < 3; j++)
            if (F[3 * i + j] < 0 || F[3 * i + j] >= n_v) return 1;
        if (tri_mat[i] < 0 || tri_mat[i] >= n_mat) return 1;
    }
    const int L = prm->max_depth;
    const int64_t N = prm->n_rays;
    const int npol = tx->pol == 2 ? 2 : 1;
    const int P = 2 * n_mat + 3;
    const double lam = OR_C0 / prm->freq;
    const double omega = 2.0 * OR_PI * prm->freq;
    const double area = pl->dx * pl->dy;
    const double kappa = lam * lam / (4.0 * OR_PI * (double)N * area);
    const cplx deta_dsigma = -I / (OR_EPS0 * omega);
    or_mesh mesh = {V, F, n_tri};
    const int want_grad = out->grad_map != NULL && out->grad != NULL;
    int64_t n_run = ray_ids ? n_ids : (ray_end - ray_begin);
    if (!ray_ids && (ray_begin < 0 || ray_end > N || ray_begin > ray_end)) return 1;
    out->rec_n = 0;
    out->tri_tests = 0;
    out->segments = 0;

    cvec3 E[2];
    static cvec3 dE[2][OR_MAX_PARAMS];

    for (int64_t r = 0; r < n_run; r++) {
        int64_t n = ray_ids ? ray_ids[r] : ray_begin + r;
        if (n < 0 || n >= N) return 1;
        vec3 k = lattice_dir(n, N);
        const cplx alpha = array_alpha(tx, k, lam);   /* 1 without an array */
        for (int p = 0; p < npol; p++) {
            dual Ed[3];
            launch_field(k, tx, tx->pol == 1 ? 1 : p, Ed);
            E[p].x = Ed[0].v; E[p].y = Ed[1].v; E[p].z = Ed[2].v;
            for (int q = 0; q < P; q++) dE[p][q] = cv_zero();
            for (int a = 0; a < 3; a++) {
                dE[p][2 * n_mat + a].x = Ed[0].d[a];
                dE[p][2 * n_mat + a].y = Ed[1].d[a];
                dE[p][2 * n_mat + a].z = Ed[2].d[a];
            }
            /* the element offsets are global, so alpha depends on no parameter */
            if (tx->n_ant > 0) {
                E[p] = cv_scale(E[p], alpha);
                for (int q = 0; q < P; q++) dE[p][q] = cv_scale(dE[p][q], alpha);
            }
        }
        vec3 o = mk(tx->pos[0], tx->pos[1], tx->pos[2]);
        int64_t last = -1;
        double run_len = 0.0;   /* unfolded length from the source */
        double tube_len = 0.0;  /* length of the current ray tube */
        int32_t* hrow = out->hits ? out->hits + r * (L + 1) : NULL;
        uint8_t* frow = out->flags ? out->flags + r * (L + 1) : NULL;
        if (hrow) for (int l = 0; l <= L; l++) hrow[l] = -2;
        if (frow) for (int l = 0; l <= L; l++) frow[l] = 0;

        for (int l = 0; l <= L; l++) {
            hit_info h;
            if (out->replay_hits) {
                int32_t pr = out->replay_hits[r * (L + 1) + l];
                if (pr == -2) break;
                h.prim = pr; h.t = INFINITY; h.t2 = INFINITY; h.flags = 0;
                if (pr >= 0) {
                    vec3 a, b, c; double t, u, v;
                    tri_verts(&mesh, pr, &a, &b, &c);
                    if (!tri_plane_hit(o, k, a, b, c, &t, &u, &v)) return 2;
                    h.t = t;
                }
            } else {
                h = closest_hit(&mesh, o, k, last, prm->t_min, &out->tri_tests);
            }
            out->segments++;
            uint8_t fl = h.flags;
            if (N > 1 && (n == 0 || n == N - 1)) fl |= OR_FLAG_POLAR;

            /* grazing incidence on the hit surface */
            vec3 nrm = mk(0, 0, 0);
            if (h.prim >= 0) {
                vec3 a, b, c;
                tri_verts(&mesh, h.prim, &a, &b, &c);
                nrm = vunit(vcross(vsub(b, a), vsub(c, a)));
                if (vdot(nrm, k) > 0) nrm = vscale(nrm, -1.0);
                if (fabs(vdot(nrm, k)) < 1e-5) fl |= OR_FLAG_GRAZING;
                if (h.t < 1e-2) fl |= OR_FLAG_NEAR;
            }
            if (hrow) hrow[l] = (int32_t)h.prim;
            if (frow) frow[l] = fl;

            /* measurement-plane crossing of this segment */
            if (k.z != 0.0) {
                double tm = (pl->z - o.z) / k.z;
                if (tm > 0.0 && tm < h.t) {
                    double x = o.x + tm * k.x, y = o.y + tm * k.y;
                    double fx = (x - pl->x0) / pl->dx, fy = (y - pl->y0) / pl->dy;
                    double fi = floor(fx), fj = floor(fy);
                    if (fi >= 0 && fi < pl->W && fj >= 0 && fj < pl->H) {
                        int64_t i = (int64_t)fi, j = (int64_t)fj;
                        int64_t cell = j * pl->W + i;
                        double g = kappa / fabs(k.z);
                        for (int p = 0; p < npol; p++) {
                            double w = g * cv_norm2(E[p]);
                            if (out->map) out->map[(int64_t)p * pl->W * pl->H + cell] += w;
                            if (want_grad) {
                                double G = out->grad_map[(int64_t)p * pl->W * pl->H + cell];
                                if (G != 0.0)
                                    for (int q = 0; q < P; q++)
                                        out->grad[q] += G * g * 2.0 * cv_re_inner(E[p], dE[p][q]);
                            }
                        }
                        if (out->counts) out->counts[cell] += 1;
                        int64_t ri = out->rec_n++;
                        if (ri < out->rec_cap) {
                            double bx = fmin(x - (pl->x0 + fi * pl->dx), pl->x0 + (fi + 1) * pl->dx - x);
                            double by = fmin(y - (pl->y0 + fj * pl->dy), pl->y0 + (fj + 1) * pl->dy - y);
                            double bz = fmin(tm * fabs(k.z), isfinite(h.t) ? (h.t - tm) * fabs(k.z) : INFINITY);
                            if (out->rec_ray) out->rec_ray[ri] = n;
                            if (out->rec_depth) out->rec_depth[ri] = l;
                            if (out->rec_cell) out->rec_cell[ri] = (int32_t)cell;
                            if (out->rec_w) out->rec_w[ri] = g * cv_norm2(E[0]);
                            if (out->rec_border) out->rec_border[ri] = fmin(fmin(bx, by), bz);
                            if (out->rec_len) out->rec_len[ri] = run_len + tm;
                        }
                    }
                }
            }
            if (h.prim < 0 || l == L) break;

            /* interaction at primitive h.prim */
            int m = tri_mat[h.prim];
            cplx eta = eps_r[m] - I * sigma[m] / (OR_EPS0 * omega);
            double c = -vdot(nrm, k);                 /* cos(theta_1) >= 0 */
            cplx s, r_perp, r_par, dr_perp, dr_par;
            fresnel_half_space(eta, c, &s, &r_perp, &r_par, &dr_perp, &dr_par);

            cplx t_perp = 0.0, t_par = 0.0, dt_perp = 0.0, dt_par = 0.0;
            if (thickness) {
                const double k_d = 2.0 * OR_PI * thickness[m] / lam;
                cplx dsp, dsl;
                slab_deriv(s, k_d, r_perp, dr_perp, &dsp, &dt_perp);
                slab_deriv(s, k_d, r_par, dr_par, &dsl, &dt_par);
                dr_perp = dsp;
                dr_par = dsl;
                slab(s, k_d, &r_perp, &r_par, &t_perp, &t_par);
            }

            vec3 e_perp, e_par, kr, er_par;
            reflection_bases(k, nrm, &e_perp, &e_par, &kr, &er_par);

            /* interaction type (eq. path-solver-used-dist-event with
             * q(D) = 0): with A = |r_perp|^2 + |r_par|^2 and B = |t_perp|^2 +
             * |t_par|^2 (0 without refraction), q(R) = R^2 A / (A + B),
             * q(S) = S^2 A / (A + B), q(T) = B / (A + B); the field of the
             * sampled branch is divided by sqrt(q) so that ||E||^2 carries the
             * Pr(chi)^-1 factor of eq. radio-map-solver-ci-all-2-estimator */
            const double Sm = scattering ? scattering[m] : 0.0;
            int kind = 0;                             /* 0 reflect, 1 diffuse, 2 transmit */
            double qk = 1.0;
            if (prm->refraction || Sm > 0.0) {
                double ar = creal(r_perp * conj(r_perp)) + creal(r_par * conj(r_par));
                double at = prm->refraction ? creal(t_perp * conj(t_perp)) + creal(t_par * conj(t_par)) : 0.0;
                double fa = (ar + at > 0.0) ? ar / (ar + at) : 1.0;
                double qr = (1.0 - Sm * Sm) * fa, qs = Sm * Sm * fa;
                double qt = (ar + at > 0.0) ? at / (ar + at) : 0.0;
                double u = rr_uniform(prm->seed, n, l, 1u);
                if (frow && (fabs(u - qr) <= 1e-5 || (Sm > 0.0 && fabs(u - (qr + qs)) <= 1e-5)))
                    frow[l] |= OR_FLAG_CHOICE;
                kind = u < qr ? 0 : (u < qr + qs ? 1 : 2);
                qk = kind == 0 ? qr : (kind == 1 ? qs : qt);
            }
            const double inv_sqrt_q = 1.0 / sqrt(qk);

            vec3 k_new = kr;
            if (kind == 1) {
                /* diffuse reflection: Lambertian direction over the
                 * hemisphere of the incident side (n points there) */
                double u4[4];
                uniform4(prm->seed, n, l, 2u, u4);
                double cs = u4[0], ss = sqrt(fmax(0.0, 1.0 - cs * cs));
                double phs = 2.0 * OR_PI * u4[1];
                double ax = fabs(nrm.x), ay = fabs(nrm.y), az = fabs(nrm.z);
                vec3 a = (ax <= ay && ax <= az) ? mk(1, 0, 0) : (ay <= az ? mk(0, 1, 0) : mk(0, 0, 1));
                vec3 t1 = vunit(vcross(a, nrm)), t2 = vcross(nrm, t1);
                k_new = vunit(vadd(vadd(vscale(t1, ss * cos(phs)), vscale(t2, ss * sin(phs))), vscale(nrm, cs)));
                vec3 thi, phi_i, ths, phs_v;
                sph_basis(k, &thi, &phi_i);
                sph_basis(k_new, &ths, &phs_v);
                const double K = xpd[m];
                const cplx e1 = cexp(I * (2.0 * OR_PI * u4[2])), e2 = cexp(I * (2.0 * OR_PI * u4[3]));
                for (int p = 0; p < npol; p++) {
                    cplx a_perp = cv_dot_real(e_perp, E[p]);
                    cplx a_par = cv_dot_real(e_par, E[p]);
                    double en2 = cv_norm2(E[p]);
                    /* Gamma^2: reflected share of the incident power, with
                     * the Fresnel (or slab) coefficients before R */
                    double g2 = en2 > 0.0 ? (creal(r_perp * a_perp * conj(r_perp * a_perp)) +
                                             creal(r_par * a_par * conj(r_par * a_par))) / en2 : 0.0;
                    cplx eth = cv_dot_real(thi, E[p]), eph = cv_dot_real(phi_i, E[p]);
                    cplx sth = e1 * (sqrt(1.0 - K) * eth - sqrt(K) * eph);
                    cplx sph = e2 * (sqrt(K) * eth + sqrt(1.0 - K) * eph);
                    /* 2 pi f_s S^2 Gamma^2 / q(S) */
                    double fs = scatter_pattern(pattern ? pattern + 4 * (int64_t)m : NULL, k, k_new, nrm, kr);
                    double sc = sqrt(2.0 * OR_PI * fs * Sm * Sm * g2) * inv_sqrt_q;
                    if (want_grad) {
                        /* E' = sc(E, eta) X P E with sc^2 = cf Gamma^2 and cf =
                         * 2 pi f_s S^2 / q(S) held constant: dE' = dsc X P E +
                         * sc X P dE, where dGamma^2 takes both the change of
                         * the coefficients (d eta) and of the incident field
                         * (Gamma^2 is a ratio of its powers) */
                        const double cf = 2.0 * OR_PI * fs * Sm * Sm / qk;
                        for (int q = 0; q < P; q++) {
                            const cvec3 dq = dE[p][q];
                            cplx deta = 0.0;
                            if (q == m) deta = 1.0;
                            else if (q == n_mat + m) deta = deta_dsigma;
                            const cplx dap = r_perp * cv_dot_real(e_perp, dq) + dr_perp * deta * a_perp;
                            const cplx dal = r_par * cv_dot_real(e_par, dq) + dr_par * deta * a_par;
                            double dg2 = 0.0;
                            if (en2 > 0.0)
                                dg2 = (2.0 * creal(conj(r_perp * a_perp) * dap) + 2.0 * creal(conj(r_par * a_par) * dal) -
                                       g2 * 2.0 * cv_re_inner(E[p], dq)) / en2;
                            const double dsc = sc > 0.0 ? cf * dg2 / (2.0 * sc) : 0.0;
                            const cplx dth = cv_dot_real(thi, dq), dph = cv_dot_real(phi_i, dq);
                            const cplx dsth = e1 * (sqrt(1.0 - K) * dth - sqrt(K) * dph);
                            const cplx dsph = e2 * (sqrt(K) * dth + sqrt(1.0 - K) * dph);
                            cvec3 nd = cv_zero();
                            nd = cv_axpy(nd, dsc * sth + sc * dsth, ths);
                            nd = cv_axpy(nd, dsc * sph + sc * dsph, phs_v);
                            dE[p][q] = nd;
                        }
                    }
                    cvec3 En = cv_zero();
                    En = cv_axpy(En, sc * sth, ths);
                    En = cv_axpy(En, sc * sph, phs_v);
                    E[p] = En;
                }
            } else {
                const double Rr = sqrt(1.0 - Sm * Sm);   /* eq. R: specular share */
                cplx c_perp = kind == 2 ? t_perp : Rr * r_perp;
                cplx c_par = kind == 2 ? t_par : Rr * r_par;
                /* derivatives w.r.t. eta; the sampling probability q is held
                 * constant (its draw decides the branch, not the value) */
                cplx dc_perp = (kind == 2 ? dt_perp : Rr * dr_perp) * inv_sqrt_q;
                cplx dc_par = (kind == 2 ? dt_par : Rr * dr_par) * inv_sqrt_q;
                vec3 out_par = kind == 2 ? e_par : er_par;
                if (kind == 2) k_new = k;

                for (int p = 0; p < npol; p++) {
                    cplx a_perp = cv_dot_real(e_perp, E[p]);
                    cplx a_par = cv_dot_real(e_par, E[p]);
                    if (want_grad) {
                        for (int q = 0; q < P; q++) {
                            cplx b_perp = cv_dot_real(e_perp, dE[p][q]);
                            cplx b_par = cv_dot_real(e_par, dE[p][q]);
                            cvec3 nd = cv_zero();
                            nd = cv_axpy(nd, c_perp * inv_sqrt_q * b_perp, e_perp);
                            nd = cv_axpy(nd, c_par * inv_sqrt_q * b_par, out_par);
                            cplx deta = 0.0;
                            if (q == m) deta = 1.0;                   /* d eta / d eps_r[m] */
                            else if (q == n_mat + m) deta = deta_dsigma; /* d eta / d sigma[m] */
                            if (deta != 0.0) {
                                nd = cv_axpy(nd, dc_perp * deta * a_perp, e_perp);
                                nd = cv_axpy(nd, dc_par * deta * a_par, out_par);
                            }
                            dE[p][q] = nd;
                        }
                    }
                    E[p] = specular_field(E[p], e_perp, e_par, out_par, c_perp, c_par, inv_sqrt_q);
                }
            }
            o = vadd(o, vscale(k, h.t));
            run_len += h.t;
            tube_len = kind == 1 ? 0.0 : tube_len + h.t;
            k = k_new;
            last = h.prim;

            /* Early termination before segment l + 1 (Sec. "Practical Notes",
             * eq. radio-map-solver-rr-prob), from depth rr_depth on.  The
             * distance-normalised gain r^2 ||E||^2 is ||E||^2 here (E carries
             * no spreading); polarisation 0 decides for both.  Gain
             * thresholding drops the path when its path gain at the current
             * ray-tube length, (lambda / (4 pi r))^2 ||E||^2, is below the
             * threshold; Russian roulette keeps it with probability
             * p = min(||E||^2, p_max) and then divides the field by sqrt(p). */
            const int next = l + 1;
            if (next >= prm->rr_depth && (prm->gain_threshold > 0.0 || prm->rr_p_max > 0.0)) {
                const double gn = cv_norm2(E[0]);
                if (prm->gain_threshold > 0.0 && tube_len > 0.0) {
                    const double thr = prm->gain_threshold;
                    const double gain = lam * lam / (16.0 * OR_PI * OR_PI * tube_len * tube_len) * gn;
                    if (frow && fabs(gain - thr) <= 1e-5 * thr) frow[next] |= OR_FLAG_TERM;
                    if (gain < thr) break;
                }
                if (prm->rr_p_max > 0.0) {
                    const double p = fmin(gn, prm->rr_p_max);
                    const double u = rr_uniform(prm->seed, n, next, 0u);
                    if (frow && fabs(u - p) <= 1e-5 * p) frow[next] |= OR_FLAG_TERM;
                    if (!(u < p)) break;
                    const double sc = 1.0 / sqrt(p);     /* p is held constant for gradients */
                    for (int p2 = 0; p2 < npol; p2++) {
                        E[p2] = cv_scale(E[p2], sc);
                        for (int q = 0; q < P; q++) dE[p2][q] = cv_scale(dE[p2][q], sc);
                    }
                }
            }
        }
    }
    return 0;
}

/* Field transport along a given specular chain, for tests (reciprocity):
 * pts [n_pts][3] are the source, the reflection points and the end point;
 * nrms [n_pts-2][3], eps_r and sigma [n_pts-2] describe the surface at each
 * reflection point.  The complex field E0 (E0[2 i], E0[2 i + 1] = Re, Im of
 * component i), transverse to the first segment, is carried through every
 * reflection with the interaction step of the radio map (half-space
 * eq. fresnel_vac, the bases of eq. fresnel_in_vectors and
 * eq. fresnel_out_vectors); the directions after each reflection are the
 * reflected ones, not re-derived from the points.  out[0..5] is the field at
 * the end point, out[6..8] the direction of the last segment.
 * Returns 1 for bad sizes. */
int or_path_field(const double* pts, int32_t n_pts, const double* nrms, const double* eps_r,
                  const double* sigma, double freq, const double* E0, double* out)
{
    if (n_pts < 2) return 1;
    const double omega = 2.0 * OR_PI * freq;
    vec3 k = vunit(vsub(mk(pts[3], pts[4], pts[5]), mk(pts[0], pts[1], pts[2])));
    cvec3 E = {E0[0] + I * E0[1], E0[2] + I * E0[3], E0[4] + I * E0[5]};
    for (int32_t i = 0; i + 2 < n_pts; i++) {
        vec3 nrm = vunit(mk(nrms[3 * i], nrms[3 * i + 1], nrms[3 * i + 2]));
        if (vdot(nrm, k) > 0.0) nrm = vscale(nrm, -1.0);
        const cplx eta = eps_r[i] - I * sigma[i] / (OR_EPS0 * omega);
        cplx sq, r_perp, r_par, dr_perp, dr_par;
        fresnel_half_space(eta, -vdot(nrm, k), &sq, &r_perp, &r_par, &dr_perp, &dr_par);
        vec3 e_perp, e_par, kr, er_par;
        reflection_bases(k, nrm, &e_perp, &e_par, &kr, &er_par);
        E = specular_field(E, e_perp, e_par, er_par, r_perp, r_par, 1.0);
        k = kr;
    }
    out[0] = creal(E.x); out[1] = cimag(E.x);
    out[2] = creal(E.y); out[3] = cimag(E.y);
    out[4] = creal(E.z); out[5] = cimag(E.z);
    out[6] = k.x; out[7] = k.y; out[8] = k.z;
    return 0;
}

/* Fresnel coefficients for tests: eq. fresnel_vac at incidence cos(theta_1) = c. */
void or_fresnel(double eps_r, double sigma, double freq, double c,
                double* rperp_re, double* rperp_im, double* rpar_re, double* rpar_im)
{
    double omega = 2.0 * OR_PI * freq;
    cplx eta = eps_r - I * sigma / (OR_EPS0 * omega);
    cplx s = csqrt(eta - (1.0 - c * c));
    cplx a = (c - s) / (c + s), b = (eta * c - s) / (eta * c + s);
    *rperp_re = creal(a); *rperp_im = cimag(a);
    *rpar_re = creal(b); *rpar_im = cimag(b);
}

/* Slab coefficients for tests: eq. fresnel_slab at incidence cos(theta_1) = c
 * for a slab of thickness d (metres); out = (r_perp, r_par, t_perp, t_par) as
 * (re, im) pairs. */
void or_fresnel_slab(double eps_r, double sigma, double freq, double c, double d, double* out8)
{
    double omega = 2.0 * OR_PI * freq;
    cplx eta = eps_r - I * sigma / (OR_EPS0 * omega);
    cplx s = csqrt(eta - (1.0 - c * c));
    cplx rp = (c - s) / (c + s), rl = (eta * c - s) / (eta * c + s), tp, tl;
    slab(s, 2.0 * OR_PI * d * freq / OR_C0, &rp, &rl, &tp, &tl);
    out8[0] = creal(rp); out8[1] = cimag(rp); out8[2] = creal(rl); out8[3] = cimag(rl);
    out8[4] = creal(tp); out8[5] = cimag(tp); out8[6] = creal(tl); out8[7] = cimag(tl);
}

/* Uniform draw of the random stream, for tests. */
double or_uniform(uint32_t seed, int64_t n, int l, uint32_t stream)
{
    return rr_uniform(seed, n, l, stream);
}

/* Transmitted field (value only) for tests: E[3 complex as re,im pairs]. */
void or_launch_field(double kx, double ky, double kz, const or_tx* tx, int pol_index, double* E3, double* dE3x3)
{
    dual Ed[3];
    launch_field(mk(kx, ky, kz), tx, pol_index, Ed);
    for (int i = 0; i < 3; i++) {
        E3[i] = Ed[i].v;
        if (dE3x3) for (int a = 0; a < 3; a++) dE3x3[3 * a + i] = Ed[i].d[a];
    }
}

void or_lattice_dir(int64_t n, int64_t N, double* k3)
{
    vec3 k = lattice_dir(n, N);
    k3[0] = k.x; k3[1] = k.y; k3[2] = k.z;
}
