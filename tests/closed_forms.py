"""Closed-form reference values that pin the oracle (test-only, NumPy).

Nothing here is shared with the oracle or the HIP library.  Where a
reflection coefficient is needed it is taken from the general two-medium
Fresnel equations (eq. fresnel) with Snell's law for cos(theta_2), a different
route from the vacuum-incidence form (eq. fresnel_vac) that the oracle uses.

Radio maps are cell averages (Sec. "Definition of Radio Map", eq. radio-map-
solver-ci-ell), so point gains are integrated over each cell with 16 x 16
Gauss-Legendre points.
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0                 # m/s (exact)
EPS0 = 8.8541878128e-12            # F/m (CODATA 2018)


def wavelength(freq):
    return C0 / freq


def eta(eps_r, sigma, freq):
    """Complex relative permittivity, eq. eta."""
    return eps_r - 1j * sigma / (EPS0 * 2 * math.pi * freq)


def fresnel_general(eta2, cos_t1):
    """(r_perp, r_par) from eq. fresnel with eta1 = 1 and Snell's law."""
    cos_t1 = np.asarray(cos_t1, dtype=np.complex128)
    n2 = np.sqrt(eta2 + 0j)
    sin2 = 1.0 - cos_t1 ** 2
    cos_t2 = np.sqrt(1.0 - sin2 / eta2)
    r_perp = (cos_t1 - n2 * cos_t2) / (cos_t1 + n2 * cos_t2)
    r_par = (n2 * cos_t1 - cos_t2) / (n2 * cos_t1 + cos_t2)
    return r_perp, r_par


def slab_characteristic(eta2, cos_t1, d, lam):
    """(r_s, r_p, t_s, t_p) of a homogeneous layer in vacuum by the optical
    characteristic-matrix method (Born and Wolf, Principles of Optics,
    Sec. 1.6): the layer of index n = sqrt(eta2) and phase thickness
    delta = (2 pi / lambda) n d cos(theta_2) has the matrix
    [[cos delta, j sin delta / Y], [j Y sin delta, cos delta]], with the
    tilted admittance Y = n cos(theta_2) (TE) or n / cos(theta_2) (TM) and
    Y_0 = cos(theta_1) or 1 / cos(theta_1) in vacuum; with (B, C) = M (1, Y_0),
    r = (Y_0 B - C) / (Y_0 B + C) and t = 2 Y_0 / (Y_0 B + C).  r_p refers to
    the tangential field, so r_p = -r_par of eq. fresnel at one interface.
    The matrix is even in n cos(theta_2), so no square-root branch enters."""
    c = np.asarray(cos_t1, dtype=np.complex128)
    n2 = np.sqrt(eta2 + 0j)
    cos_t2 = np.sqrt(1.0 - (1.0 - c ** 2) / eta2)
    delta = 2 * math.pi / lam * d * n2 * cos_t2
    out = []
    for y0, y1 in ((c, n2 * cos_t2), (1.0 / c, n2 / cos_t2)):
        B = np.cos(delta) + 1j * np.sin(delta) / y1 * y0
        C = 1j * y1 * np.sin(delta) + np.cos(delta) * y0
        out.append(((y0 * B - C) / (y0 * B + C), 2 * y0 / (y0 * B + C)))
    (rs, ts), (rp, tp) = out
    return rs, rp, ts, tp


def normal_incidence_r(eta2):
    """Textbook normal-incidence reflection coefficient (1 - n)/(1 + n), n = sqrt(eta)."""
    n = np.sqrt(eta2 + 0j)
    return (1 - n) / (1 + n)


def brewster_angle(eps_r):
    return math.atan(math.sqrt(eps_r))


def free_space_gain(d, lam):
    """Friis gain (lambda/(4 pi d))^2 for unit antenna gains (Friis box, App. A)."""
    return (lam / (4 * math.pi * d)) ** 2


def cell_average(fn, plane, n=16):
    """(1/|M_i|) * integral of fn(x, y) over every cell, 16x16 Gauss-Legendre.

    Returns an array [H][W].
    """
    g, w = np.polynomial.legendre.leggauss(n)
    ux = (g + 1) / 2 * plane.dx           # offsets within a cell
    uy = (g + 1) / 2 * plane.dy
    wx = w / 2
    xs = plane.x0 + np.arange(plane.W)[:, None] * plane.dx + ux[None, :]   # [W][n]
    ys = plane.y0 + np.arange(plane.H)[:, None] * plane.dy + uy[None, :]   # [H][n]
    X = xs[None, :, None, :]                                               # [1][W][1][n]
    Y = ys[:, None, :, None]                                               # [H][1][n][1]
    F = fn(np.broadcast_to(X, (plane.H, plane.W, n, n)), np.broadcast_to(Y, (plane.H, plane.W, n, n)))
    return np.einsum("hwij,i,j->hw", F, wx, wx)


def friis_map(tx_pos, plane, lam):
    tx = np.asarray(tx_pos, dtype=np.float64)

    def f(x, y):
        d2 = (x - tx[0]) ** 2 + (y - tx[1]) ** 2 + (plane.z - tx[2]) ** 2
        return (lam / (4 * math.pi)) ** 2 / d2

    return cell_average(f, plane)


def two_ray_map(tx_pos, plane, lam, eta2, pol="V", ground_z=0.0):
    """Non-coherent two-ray map over a horizontal ground at z = ground_z.

    LoS term plus the image-source term weighted by |r|^2 at the incidence
    angle; V polarisation lies in the plane of incidence (r_par), H is
    perpendicular to it (r_perp).  pol = "sum" gives |r_perp|^2 + |r_par|^2.
    """
    tx = np.asarray(tx_pos, dtype=np.float64)
    ht = tx[2] - ground_z
    hr = plane.z - ground_z

    def f(x, y):
        rho2 = (x - tx[0]) ** 2 + (y - tx[1]) ** 2
        d_los2 = rho2 + (ht - hr) ** 2
        d_ref2 = rho2 + (ht + hr) ** 2
        cos_i = (ht + hr) / np.sqrt(d_ref2)
        rp, rl = fresnel_general(eta2, cos_i)
        if pol == "V":
            refl = np.abs(rl) ** 2
        elif pol == "H":
            refl = np.abs(rp) ** 2
        else:
            refl = np.abs(rp) ** 2 + np.abs(rl) ** 2
        return (lam / (4 * math.pi)) ** 2 * (1.0 / d_los2 + refl / d_ref2)

    return cell_average(f, plane)


def reflected_only_map(tx_pos, plane, lam, eta2, pol="V", ground_z=0.0):
    tx = np.asarray(tx_pos, dtype=np.float64)
    ht = tx[2] - ground_z
    hr = plane.z - ground_z

    def f(x, y):
        rho2 = (x - tx[0]) ** 2 + (y - tx[1]) ** 2
        d_ref2 = rho2 + (ht + hr) ** 2
        cos_i = (ht + hr) / np.sqrt(d_ref2)
        rp, rl = fresnel_general(eta2, cos_i)
        refl = np.abs(rl) ** 2 if pol == "V" else np.abs(rp) ** 2
        return (lam / (4 * math.pi)) ** 2 * refl / d_ref2

    return cell_average(f, plane)


def fibonacci_phase_exact(n: int) -> float:
    """frac(n / phi_g) with 60 significant digits (decimal arithmetic)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    phi = (Decimal(1) + Decimal(5).sqrt()) / 2
    x = Decimal(n) / phi
    return float(x - int(x))


def lattice_directions(ns, N: int) -> np.ndarray:
    """Unit directions of lattice points `ns` of an N-point spherical
    Fibonacci lattice (float64; fine for n below about 1e7)."""
    ns = np.asarray(ns, dtype=np.float64)
    golden = (1.0 + math.sqrt(5.0)) / 2.0
    z = 1.0 - 2.0 * ns / (N - 1)
    phi = 2.0 * math.pi * np.mod(ns * (golden - 1.0), 1.0)
    s = np.sqrt(np.maximum(0.0, (1.0 - z) * (1.0 + z)))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def dirichlet_gain(n: int, spacing_wl: float, c, c0: float) -> np.ndarray:
    """|alpha|^2 of an n-element uniform linear array, element spacing
    `spacing_wl` wavelengths, weights exp(-j 2 pi s i c0)/sqrt(n): the
    Dirichlet kernel sin^2(n pi s (c - c0)) / (n sin^2(pi s (c - c0))), with
    c the direction cosine along the array axis (limit n where the
    denominator vanishes)."""
    x = math.pi * spacing_wl * (np.asarray(c, dtype=np.float64) - c0)
    den = n * np.sin(x) ** 2
    num = np.sin(n * x) ** 2
    small = np.abs(np.sin(x)) < 1e-12
    return np.where(small, float(n), num / np.where(small, 1.0, den))


def directive_pattern(alpha, ki, ks, n, lobe2=None):
    """Scattering pattern of eq. directive_model (lobe2 = (alpha_I, Lambda):
    eq. backscattering_model) for arrays of unit vectors [..., 3]; the
    normalisation F_alpha(theta_i) is taken by numerical quadrature over the
    hemisphere (so that int f_s d(omega) = 1 holds by construction here and
    the closed-form F of the paper is what the oracle pins against)."""
    ci = -np.sum(ki * n, -1)
    kr = ki + 2.0 * ci[..., None] * n
    lobe = (0.5 * (1.0 + np.sum(kr * ks, -1))) ** alpha
    F = _lobe_norm_interp(alpha, "r", ci)
    if lobe2 is not None:
        aI, L = lobe2
        lobe = L * lobe + (1 - L) * (0.5 * (1.0 - np.sum(ki * ks, -1))) ** aI
        F = L * F + (1 - L) * _lobe_norm_interp(aI, "i", ci)
    return lobe / F


_LOBE_CACHE = {}


def _lobe_norm_interp(alpha, which, ci):
    """lobe_norm_quadrature on a 2,001-point grid of cos(theta_i), cubic
    interpolation in between (smooth in cos(theta_i))."""
    key = (alpha, which)
    if key not in _LOBE_CACHE:
        grid = np.linspace(0.0, 1.0, 2001)
        _LOBE_CACHE[key] = (grid, lobe_norm_quadrature(alpha, grid, which))
    grid, vals = _LOBE_CACHE[key]
    from scipy.interpolate import CubicSpline
    return CubicSpline(grid, vals)(np.clip(ci, 0.0, 1.0))


def lobe_norm_quadrature(alpha, ci, which, n_t=64, n_p=128):
    """int over the hemisphere of ((1 + k_r.k_s)/2)^alpha (which = "r") or
    ((1 - k_i.k_s)/2)^alpha ("i") d(omega), for incidence cosines ci, by
    Gauss-Legendre in cos(theta_s) and the midpoint rule in azimuth, in the
    frame n = z, incidence plane x-z."""
    ci = np.asarray(ci, dtype=np.float64)
    g, w = np.polynomial.legendre.leggauss(n_t)
    mu = (g + 1) / 2
    wm = w / 2
    ph = (np.arange(n_p) + 0.5) * 2 * math.pi / n_p
    si = np.sqrt(np.maximum(0.0, 1 - ci ** 2))[..., None, None]
    c = ci[..., None, None]
    st = np.sqrt(1 - mu ** 2)[:, None]
    # k_i = (si, 0, -ci), k_r = (si, 0, ci), k_s = (st cos ph, st sin ph, mu)
    dot_r = si * st * np.cos(ph)[None, :] + c * mu[:, None]
    dot_i = si * st * np.cos(ph)[None, :] - c * mu[:, None]
    base = 0.5 * (1 + dot_r) if which == "r" else 0.5 * (1 - dot_i)
    return np.sum(base ** alpha * wm[:, None], axis=(-2, -1)) * (2 * math.pi / n_p)


def lambertian_ground_map(tx_pos, plane, lam, eta_g, pol, half, ceiling=None, n_beta=48, n_psi=96, n_cell=2,
                          pattern=None):
    """Expected map of paths Tx -> Lambertian ground (S = 1) -> plane, or,
    with ceiling = (z_c, eta_c, "par" | "perp"), Tx -> ground -> specular
    ceiling -> plane, over a ground square |x|, |y| <= half at z = 0.

    The gain per ground element dA at q seen from a plane point t is
    (lambda/4 pi)^2 Gamma^2 (cos theta_s / pi) cos theta_i dA / (r0^2 d^2)
    (App. "Diffuse Reflection", eq. scattered_field with the Lambertian
    pattern); with dA cos theta_s / d^2 = d(omega) seen from t (or from its
    image above the ceiling) the integral runs over directions:
    (lambda/4 pi)^2 / pi * int Gamma^2 cos theta_i / r0^2 [|r_c|^2] d(omega).
    Gamma^2 is |r_par|^2 (V-pol: the field lies in the plane of incidence)
    or |r_perp|^2 (H-pol).  Directions: Gauss-Legendre in the polar angle up
    to the square's edge, uniform in azimuth; cells: n_cell^2 points.
    pattern(ki, ks, n) replaces the Lambertian cos(theta_s)/pi (no ceiling).
    """
    tx = np.asarray(tx_pos, dtype=np.float64)
    g, gw = np.polynomial.legendre.leggauss(n_beta)
    c, cw = np.polynomial.legendre.leggauss(n_cell)
    psi = (np.arange(n_psi) + 0.5) * 2 * math.pi / n_psi
    cp, sp = np.cos(psi), np.sin(psi)
    out = np.zeros((plane.H, plane.W))
    for j in range(plane.H):
        for i in range(plane.W):
            acc = 0.0
            for a, wa in zip(c, cw):
                for b, wb in zip(c, cw):
                    tx_ = plane.x0 + (i + (a + 1) / 2) * plane.dx
                    ty_ = plane.y0 + (j + (b + 1) / 2) * plane.dy
                    hz = plane.z if ceiling is None else 2 * ceiling[0] - plane.z
                    # distance along psi from (tx_, ty_) to the square's edge
                    with np.errstate(divide="ignore"):
                        rx = np.where(cp > 0, (half - tx_) / cp, np.where(cp < 0, (-half - tx_) / cp, np.inf))
                        ry = np.where(sp > 0, (half - ty_) / sp, np.where(sp < 0, (-half - ty_) / sp, np.inf))
                    bmax = np.arctan(np.minimum(rx, ry) / hz)                    # [n_psi]
                    beta = (g[None, :] + 1) / 2 * bmax[:, None]                 # [n_psi][n_beta]
                    wbeta = gw[None, :] / 2 * bmax[:, None]
                    rho = hz * np.tan(beta)
                    qx = tx_ + rho * cp[:, None]
                    qy = ty_ + rho * sp[:, None]
                    r0 = np.sqrt((qx - tx[0]) ** 2 + (qy - tx[1]) ** 2 + tx[2] ** 2)
                    ci = tx[2] / r0
                    rp, rl = fresnel_general(eta_g, ci)
                    gam = np.abs(rl) ** 2 if pol == "V" else np.abs(rp) ** 2
                    f = gam * ci / r0 ** 2
                    if pattern is not None:
                        # f_s / (cos(theta_s)/pi) at (incident q - tx, scattered t - q)
                        ki = np.stack([qx - tx[0], qy - tx[1], np.full_like(qx, -tx[2])], -1) / r0[..., None]
                        dvec = np.stack([tx_ - qx, ty_ - qy, np.full_like(qx, hz)], -1)
                        ks = dvec / np.linalg.norm(dvec, axis=-1)[..., None]
                        nz = np.zeros_like(ks)
                        nz[..., 2] = 1.0
                        f = f * pattern(ki, ks, nz) * math.pi / ks[..., 2]
                    if ceiling is not None:
                        cp_, cl_ = fresnel_general(ceiling[1], np.cos(beta))
                        f = f * (np.abs(cl_) ** 2 if ceiling[2] == "par" else np.abs(cp_) ** 2)
                    acc += wa * wb / 4 * np.sum(f * np.sin(beta) * wbeta) * (2 * math.pi / n_psi)
            out[j, i] = (lam / (4 * math.pi)) ** 2 / math.pi * acc
    return out
