"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins; together they are chosen so that a dropped
term, a wrong sign or index, or a transposed operand anywhere in the oracle
fails at least one of them.  CPU only.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import scenegen as sg

FREQ = 3.5e9
LAM = cf.wavelength(FREQ)


def _run(oracle_lib, scene, tx, plane, N, L, **kw):
    return oracle_lib.radio_map(scene, tx, plane, sg.Params(FREQ, N, L), **kw)


# ---------------------------------------------------------------- lattice
def test_fibonacci_lattice_invariants(oracle_lib):
    """Sec. 'Sampling Initial Ray Directions': z spacing, both poles, balance."""
    for N in (1000, 100_001):
        ks = np.array([oracle_lib.lattice(n, N) for n in range(N)])
        z = ks[:, 2]
        n = np.arange(N)
        assert np.max(np.abs(z - (1 - 2 * n / (N - 1)))) <= 2e-16
        assert np.allclose(np.linalg.norm(ks, axis=1), 1.0, atol=1e-15)
        assert z[0] == 1.0 and z[-1] == -1.0
        assert (z < 0).sum() == (n > (N - 1) / 2).sum()
        assert abs(z.sum()) < 1e-9
        assert np.linalg.norm(ks.sum(0)) < 1.0


def test_fibonacci_phase_exact(oracle_lib):
    """frac(n/phi_g) against 60-digit decimal arithmetic (n up to 1e9).

    The oracle evaluates n (phi_g - 1) in 64-bit-mantissa extended precision,
    so its phase error is bounded by a few units of n * 2^-64.
    """
    for n in (1, 2, 99_999, 9_999_999, 99_999_999, 123_456_789, 999_999_999):
        _, phi = oracle_lib.fibonacci_angles(n, 2 * n + 1)
        exact = cf.fibonacci_phase_exact(n)
        d = abs(phi / (2 * math.pi) - exact)
        assert min(d, 1 - d) < max(1e-15, 4.0 * n * 2.0 ** -64), (n, phi, exact)


def test_fibonacci_single_ray(oracle_lib):
    """N_S = 1: theta = pi/2, phi = pi."""
    th, ph = oracle_lib.fibonacci_angles(0, 1)
    assert th == pytest.approx(math.pi / 2) and ph == pytest.approx(math.pi)
    k = oracle_lib.lattice(0, 1)
    assert np.allclose(k, [-1.0, 0.0, 0.0], atol=1e-15)


# ---------------------------------------------------------- antenna field
def test_iso_vpol_field_is_theta_hat(oracle_lib):
    """Isotropic V-pol at zero orientation: C = theta_hat (eq. spherical_vecs, eq. C)."""
    tx = sg.Tx((0, 0, 0))
    for n in (3, 77, 500):
        k = oracle_lib.lattice(n, 1000)
        th, ph = math.acos(k[2]), math.atan2(k[1], k[0])
        theta_hat = [math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)]
        E, _ = oracle_lib.launch_field(k, tx, 0)
        assert np.allclose(E, theta_hat, atol=1e-14)
        Eh, _ = oracle_lib.launch_field(k, tx, 1)
        assert np.allclose(Eh, [-math.sin(ph), math.cos(ph), 0], atol=1e-14)


def test_directional_pattern_normalisation_and_pointing(oracle_lib):
    """int G dOmega = 4 pi (normalisation box, App. A) and the main lobe follows R x_hat.

    Facts of the right-handed yaw/pitch/roll rotation (eq. rotation): yaw = 90 deg
    turns +x to +y; pitch = +90 deg turns +x to -z.
    """
    N = 20000
    ks = np.array([oracle_lib.lattice(n, N) for n in range(N)])
    for yaw, pitch, roll, lobe in ((0, 0, 0, (1, 0, 0)), (90, 0, 0, (0, 1, 0)),
                                   (0, 90, 0, (0, 0, -1)), (30, -10, 25, None)):
        tx = sg.Tx((0, 0, 0), yaw=math.radians(yaw), pitch=math.radians(pitch), roll=math.radians(roll),
                   pattern=sg.PATTERN_DIRECTIONAL, pattern_q=2.0)
        G = np.array([np.sum(oracle_lib.launch_field(k, tx, 0)[0] ** 2) for k in ks])
        assert G.mean() * 4 * math.pi == pytest.approx(4 * math.pi, rel=2e-4)
        if lobe is not None:
            E, _ = oracle_lib.launch_field(np.array(lobe, float), tx, 0)
            assert np.sum(E ** 2) == pytest.approx(3.0, rel=1e-12)     # (q+1)
            E, _ = oracle_lib.launch_field(-np.array(lobe, float), tx, 0)
            assert np.sum(E ** 2) == pytest.approx(0.0, abs=1e-24)


def test_launch_field_transverse_and_derivatives(oracle_lib):
    """The field is transverse to k; dual-number derivatives match central differences."""
    tx = sg.Tx((0, 0, 0), yaw=0.4, pitch=-0.2, roll=0.3, pattern=sg.PATTERN_DIRECTIONAL)
    k = oracle_lib.lattice(1234, 5000)
    E, dE = oracle_lib.launch_field(k, tx, 0)
    assert abs(np.dot(E, k)) < 1e-14
    h = 1e-6
    for a, name in enumerate(("yaw", "pitch", "roll")):
        tp = sg.Tx(**{**tx.__dict__, name: getattr(tx, name) + h})
        tm = sg.Tx(**{**tx.__dict__, name: getattr(tx, name) - h})
        fd = (oracle_lib.launch_field(k, tp, 0)[0] - oracle_lib.launch_field(k, tm, 0)[0]) / (2 * h)
        assert np.allclose(dE[a], fd, atol=1e-8)


# ------------------------------------------------------------- Fresnel
def test_fresnel_special_cases(oracle_lib):
    """Normal incidence (textbook), Brewster zero (lossless), grazing -> -1, PEC limit."""
    e = cf.eta(5.24, 0.12, FREQ)
    rp, rl = oracle_lib.fresnel(5.24, 0.12, FREQ, 1.0)
    r0 = cf.normal_incidence_r(e)
    assert abs(rp - r0) < 1e-15 and abs(rl + r0) < 1e-15
    assert abs(r0) ** 2 == pytest.approx(0.1555877, abs=5e-8)
    tb = cf.brewster_angle(5.24)
    assert math.degrees(tb) == pytest.approx(66.4018, abs=1e-4)
    rp, rl = oracle_lib.fresnel(5.24, 0.0, FREQ, math.cos(tb))
    assert abs(rl) < 1e-15 and abs(rp) > 0.5
    rp, rl = oracle_lib.fresnel(5.24, 0.12, FREQ, 1e-9)
    assert abs(rp + 1) < 1e-8 and abs(rl + 1) < 1e-7
    rp, rl = oracle_lib.fresnel(1.0, 1e14, FREQ, math.cos(0.7))
    assert abs(rp + 1) < 1e-5 and abs(rl - 1) < 1e-5


def test_fresnel_matches_general_form(oracle_lib):
    """eq. fresnel_vac equals eq. fresnel with Snell's law (different algebraic route)."""
    for eps, sig in ((5.24, 0.12), (6.31, 0.05), (1.0, 1e7), (3.0, 0.0)):
        e = cf.eta(eps, sig, FREQ)
        for deg in np.linspace(0, 89.9, 37):
            c = math.cos(math.radians(deg))
            a, b = oracle_lib.fresnel(eps, sig, FREQ, c)
            ga, gb = cf.fresnel_general(e, c)
            assert abs(a - ga) < 1e-12 and abs(b - gb) < 1e-12, (eps, sig, deg)


# ----------------------------------------------------- radio-map closed forms
def test_friis_free_space(oracle_lib):
    """Empty scene: cell averages of (lambda/(4 pi d))^2 (Friis box)."""
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -20.0, -20.0, 1.0, 1.0, 40, 40)
    r = _run(oracle_lib, sg.empty_scene(), tx, pl, 1_000_000, 0)
    ref = cf.friis_map(tx.pos, pl, LAM)
    m = r.counts >= 400
    assert m.sum() > 150
    rel = np.abs(r.map[0] / ref - 1)
    assert np.all(rel[m] <= 3 / np.sqrt(r.counts[m]))
    assert abs(r.map[0][m].sum() / ref[m].sum() - 1) <= 2e-3


@pytest.mark.parametrize("pol", ["V", "H"])
def test_two_ray_ground_reflection(oracle_lib, pol):
    """Ground quad: LoS + image-source term with |r_par|^2 (V) or |r_perp|^2 (H)."""
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_V if pol == "V" else sg.POL_H)
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    r = _run(oracle_lib, sg.ground_quad(100.0), tx, pl, 2_000_000, 3)
    ref = cf.two_ray_map(tx.pos, pl, LAM, cf.eta(5.24, 0.12, FREQ), pol)
    m = r.counts >= 400
    assert m.sum() > 200
    rel = np.abs(r.map[0] / ref - 1)
    assert np.all(rel[m] <= 3 / np.sqrt(r.counts[m]))
    assert abs(r.map[0][m].sum() / ref[m].sum() - 1) <= 2e-3
    # V and H differ: swapping r_par and r_perp must be detectable
    other = cf.two_ray_map(tx.pos, pl, LAM, cf.eta(5.24, 0.12, FREQ), "H" if pol == "V" else "V")
    assert abs(r.map[0][m].sum() / other[m].sum() - 1) > 1e-2


def test_dual_pol_sum_is_basis_free(oracle_lib):
    """Dual-pol iso Tx on ground: map_V + map_H = LoS x 2 + (|r_perp|^2 + |r_par|^2) image term."""
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_DUAL)
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    r = _run(oracle_lib, sg.ground_quad(100.0), tx, pl, 1_000_000, 2)
    e = cf.eta(5.24, 0.12, FREQ)
    refv = cf.two_ray_map(tx.pos, pl, LAM, e, "V")
    refh = cf.two_ray_map(tx.pos, pl, LAM, e, "H")
    m = r.counts >= 200
    tot = r.map[0] + r.map[1]
    assert abs(tot[m].sum() / (refv + refh)[m].sum() - 1) <= 2e-3
    assert abs(r.map[0][m].sum() / refv[m].sum() - 1) <= 2e-3
    assert abs(r.map[1][m].sum() / refh[m].sum() - 1) <= 2e-3


def test_brewster_ring(oracle_lib):
    """Lossless ground (sigma = 0): the V-pol reflected part vanishes at rho_B = 11.5 tan(theta_B)."""
    sc = sg.ground_quad(200.0, (5.24, 0.0))
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, 0.0, -2.0, 0.5, 4.0, 120, 1)      # radial strip along +x
    N = 4_000_000
    r1 = _run(oracle_lib, sc, tx, pl, N, 1)
    r0 = _run(oracle_lib, sc, tx, pl, N, 0)
    refl = r1.map[0, 0] - r0.map[0, 0]
    rho = (np.arange(120) + 0.5) * 0.5
    rho_b = 11.5 * math.tan(cf.brewster_angle(5.24))
    assert rho_b == pytest.approx(26.32, abs=0.01)
    i_min = int(np.argmin(refl[10:]) + 10)
    assert abs(rho[i_min] - rho_b) <= 0.5
    i_half = int(rho_b / 2 / 0.5)
    assert refl[i_min] <= 1e-2 * refl[i_half]
    ref = cf.reflected_only_map(tx.pos, pl, LAM, cf.eta(5.24, 0.0, FREQ), "V")[0]
    cnt = r1.counts[0]
    ok = (cnt >= 400) & (ref > 0.05 * ref.max())
    assert np.all(np.abs(refl[ok] - ref[ok]) <= 3 / np.sqrt(cnt[ok]) * (r1.map[0, 0][ok]))


def test_normal_incidence_record(oracle_lib):
    """Ray N_S-1 goes straight down, reflects straight up: weight lambda^2|r(0)|^2/(4 pi N_S |M|)."""
    tx = sg.Tx((0.3, 0.7, 10.0))
    pl = sg.Plane(1.5, -50.0, -50.0, 1.0, 1.0, 100, 100)
    N = 10_001
    r = _run(oracle_lib, sg.ground_quad(100.0), tx, pl, N, 2, ray_ids=[N - 1], want_records=True)
    rec = r.records
    assert list(rec["depth"]) == [0, 1]
    cell = 50 * 100 + 50
    assert list(rec["cell"]) == [cell, cell]
    r0 = cf.normal_incidence_r(cf.eta(5.24, 0.12, FREQ))
    w_los = LAM ** 2 / (4 * math.pi * N * 1.0)
    assert rec["w"][0] == pytest.approx(w_los, rel=1e-12)
    assert rec["w"][1] == pytest.approx(w_los * abs(r0) ** 2, rel=1e-12)
    assert rec["length"][1] == pytest.approx(10.0 + 1.5, rel=1e-12)
    assert r.hits[0, 0] in (0, 1) and r.hits[0, 1] == -1 and r.hits[0, 2] == -2


def test_pec_image_source(oracle_lib):
    """Near-PEC ground: |r| -> 1 at every angle, map = LoS + image source."""
    sc = sg.ground_quad(100.0, (1.0, 1e14))
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    r = _run(oracle_lib, sc, tx, pl, 1_000_000, 1)
    lam = LAM

    def f(x, y):
        rho2 = x ** 2 + y ** 2
        return (lam / (4 * math.pi)) ** 2 * (1 / (rho2 + 8.5 ** 2) + 1 / (rho2 + 11.5 ** 2))

    ref = cf.cell_average(f, pl)
    m = r.counts >= 200
    assert abs(r.map[0][m].sum() / ref[m].sum() - 1) <= 2e-3
    assert np.all(np.abs(r.map[0] / ref - 1)[m] <= 3 / np.sqrt(r.counts[m]))


def test_pec_corner_four_images(oracle_lib):
    """Near-PEC ground + near-PEC wall: every reflection is norm-preserving, so the map is
    the sum of four image sources (direct, ground, wall, corner).  Paths of depth 2
    pin the reflected-basis bookkeeping: a field left non-transverse after the first
    bounce loses norm at the second."""
    mb = sg._MeshBuilder()
    mb.quad((-200.0, -200.0, 0.0), (200.0, -200.0, 0.0), (200.0, 200.0, 0.0), (-200.0, 200.0, 0.0), 0)
    mb.quad((20.0, -200.0, 0.0), (20.0, 200.0, 0.0), (20.0, 200.0, 100.0), (20.0, -200.0, 100.0), 0)
    sc = mb.build([(1.0, 1e14)], "corner")
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -20.0, -20.0, 2.0, 2.0, 19, 20)
    r = _run(oracle_lib, sc, tx, pl, 2_000_000, 3)
    lam = LAM
    images = [(0.0, 0.0, 10.0), (0.0, 0.0, -10.0), (40.0, 0.0, 10.0), (40.0, 0.0, -10.0)]

    def f(x, y):
        return sum((lam / (4 * math.pi)) ** 2 / ((x - a) ** 2 + (y - b) ** 2 + (1.5 - c) ** 2)
                   for a, b, c in images)

    ref = cf.cell_average(f, pl)
    m = r.counts >= 300
    assert m.sum() > 200
    assert abs(r.map[0][m].sum() / ref[m].sum() - 1) <= 2e-3
    assert np.all(np.abs(r.map[0] / ref - 1)[m] <= 3 / np.sqrt(r.counts[m]))


def test_depth_invariance_ground_only(oracle_lib):
    """Ground only: every reflected ray escapes, so L = 1 and L = 3 maps are identical."""
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    sc = sg.ground_quad(100.0)
    a = _run(oracle_lib, sc, tx, pl, 200_000, 1)
    b = _run(oracle_lib, sc, tx, pl, 200_000, 3)
    assert np.array_equal(a.map, b.map) and np.array_equal(a.counts, b.counts)
    c = _run(oracle_lib, sc, tx, pl, 200_000, 0)
    assert np.all(c.map <= a.map) and c.map.sum() < a.map.sum()


def test_yaw_invariance_iso(oracle_lib):
    """Iso V-pol: a yaw rotation about z leaves the field (and the map) unchanged."""
    cfg = sg.tiny_config(n_rays=20_000)
    a = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params)
    tx = sg.Tx(cfg.tx.pos, yaw=math.radians(40.0))
    G = np.ones((1, cfg.plane.H, cfg.plane.W))
    b = oracle_lib.radio_map(cfg.scene, tx, cfg.plane, cfg.params, grad_map=G)
    assert np.allclose(a.map, b.map, rtol=1e-12, atol=0)
    g = b.grad
    assert abs(g[2]) <= 1e-9 * max(abs(g[3]), 1e-30) or abs(g[2]) < 1e-20


def test_reciprocity_dual_pol(oracle_lib):
    """Swapping Tx and Rx leaves the dual-pol (Frobenius) path gain unchanged.

    Tiny scene (ground + building).  A = (0, 0, 10), B = (20, 30, 2): the map of
    Tx@A on the plane z = 2 at the cell around B equals the map of Tx@B on the
    plane z = 10 at the cell around A, within Monte-Carlo noise.
    """
    sc = sg.tiny_scene()
    A, B = (0.0, 0.0, 10.0), (20.0, 30.0, 2.0)
    N = 2_000_000
    plA = sg.Plane(B[2], B[0] - 1.5, B[1] - 1.5, 3.0, 3.0, 1, 1)
    plB = sg.Plane(A[2], A[0] - 1.5, A[1] - 1.5, 3.0, 3.0, 1, 1)
    ra = _run(oracle_lib, sc, sg.Tx(A, pol=sg.POL_DUAL), plA, N, 3)
    rb = _run(oracle_lib, sc, sg.Tx(B, pol=sg.POL_DUAL), plB, N, 3)
    ga = ra.map[:, 0, 0].sum()
    gb = rb.map[:, 0, 0].sum()
    n = min(ra.counts[0, 0], rb.counts[0, 0])
    assert n > 300
    assert abs(ga / gb - 1) <= 3 / math.sqrt(n)


def _mirror(p, q, n):
    return p - 2.0 * np.dot(p - q, n) * n


def _image_chain(A, B, planes):
    """Reflection points of the specular path A -> planes[0] -> ... -> B by
    the image method (planes: (point, unit normal)); None if a reflection
    point falls outside its segment."""
    imgs = [None] * len(planes)
    img = B
    for i in range(len(planes) - 1, -1, -1):
        img = _mirror(img, *planes[i])
        imgs[i] = img
    pts, cur = [A], A
    for i, (q, n) in enumerate(planes):
        d = imgs[i] - cur
        den = np.dot(d, n)
        if abs(den) < 1e-12:
            return None
        t = np.dot(q - cur, n) / den
        if not 1e-6 < t < 1 - 1e-6:
            return None
        cur = cur + t * d
        pts.append(cur)
    pts.append(B)
    return np.array(pts)


def _transfer(oracle_lib, pts, planes, mats):
    """3x2 transfer matrix of the chain on the two transverse unit fields at
    the source, and the direction of the last segment."""
    k0 = (pts[1] - pts[0]) / np.linalg.norm(pts[1] - pts[0])
    u1 = np.cross(k0, [0.3, 0.5, 0.8])
    u1 /= np.linalg.norm(u1)
    u2 = np.cross(k0, u1)
    nrm = [n for _, n in planes]
    cols = []
    for u in (u1, u2):
        E, k = oracle_lib.path_field(pts, nrm, [m[0] for m in mats], [m[1] for m in mats], 3.5e9,
                                     u.astype(complex))
        cols.append(E)
    return np.stack(cols, axis=1), k


def test_reciprocity_exact_per_path(oracle_lib):
    """Reciprocity of the field transport, path by path: for specular chains
    of one to three reflections on a ground (z = 0) and two walls (x = 30,
    y = 40), built by the image method between random points A and B with
    random materials, the transfer matrix of A -> B and that of the reverse
    chain B -> A have the same singular values (so the same Frobenius norm)
    to 1e-12; every reflected direction of the oracle reproduces the image
    geometry, and the field stays transverse to it."""
    rng = np.random.default_rng(3)
    ground = (np.zeros(3), np.array([0.0, 0.0, 1.0]))
    wall_x = (np.array([30.0, 0.0, 0.0]), np.array([-1.0, 0.0, 0.0]))
    wall_y = (np.array([0.0, 40.0, 0.0]), np.array([0.0, -1.0, 0.0]))
    sequences = [[ground], [wall_x], [ground, wall_x], [wall_x, ground], [wall_x, ground, wall_y],
                 [ground, wall_y, wall_x], [wall_y, wall_x, ground]]
    n_checked = 0
    for trial in range(60):
        seq = sequences[trial % len(sequences)]
        A = np.array([rng.uniform(-20, 25), rng.uniform(-20, 35), rng.uniform(1, 30)])
        B = np.array([rng.uniform(-20, 25), rng.uniform(-20, 35), rng.uniform(1, 30)])
        pts = _image_chain(A, B, seq)
        if pts is None:
            continue
        mats = [(rng.uniform(2.0, 10.0), 10 ** rng.uniform(-3, 0)) for _ in seq]
        M, k = _transfer(oracle_lib, pts, seq, mats)
        Mr, kr = _transfer(oracle_lib, pts[::-1].copy(), seq[::-1], mats[::-1])
        last = (pts[-1] - pts[-2]) / np.linalg.norm(pts[-1] - pts[-2])
        assert np.allclose(k, last, atol=1e-12) and np.allclose(kr, -(pts[1] - pts[0]) / np.linalg.norm(pts[1] - pts[0]),
                                                                 atol=1e-12)
        assert np.abs(k @ M).max() <= 1e-12 and np.abs(kr @ Mr).max() <= 1e-12
        sv, svr = np.linalg.svd(M, compute_uv=False), np.linalg.svd(Mr, compute_uv=False)
        assert np.allclose(sv, svr, rtol=0, atol=1e-12 * sv.max()), (seq, sv, svr)
        n_checked += 1
    assert n_checked >= 30


# ------------------------------------------------------------- gradients
def test_forward_mode_gradient_matches_central_fd(oracle_lib):
    """Oracle tangents vs FP64 central finite differences (h = 1e-4 relative) on a
    Manhattan sub-sample with the directional, rotated transmitter."""
    cfg = sg.diff_config(n_rays=3000, max_depth=4)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((1, 100, 100))
    base = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, grad_map=G, want_hits=True)
    hits = base.hits

    def loss(eps, sig, tx):
        r = oracle_lib.radio_map(cfg.scene, tx, cfg.plane, cfg.params, eps_r=eps, sigma=sig, replay_hits=hits)
        return float(np.sum(G * r.map))

    eps0, sig0 = cfg.scene.eps_r.copy(), cfg.scene.sigma.copy()
    nm = len(eps0)
    fd = []
    for p in range(2 * nm + 3):
        def at(sign):
            eps, sig, tx = eps0.copy(), sig0.copy(), sg.Tx(**cfg.tx.__dict__)
            if p < nm:
                h = 1e-4 * eps[p]; eps[p] += sign * h
            elif p < 2 * nm:
                h = 1e-4 * sig[p - nm]; sig[p - nm] += sign * h
            else:
                name = ("yaw", "pitch", "roll")[p - 2 * nm]
                v = getattr(tx, name)
                h = 1e-4 * abs(v) if v != 0 else 1e-4
                setattr(tx, name, v + sign * h)
            return loss(eps, sig, tx), h
        lp, h = at(+1)
        lm, _ = at(-1)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    g = base.grad
    scale = np.max(np.abs(fd))
    assert np.all(np.abs(g - fd) <= 1e-6 * np.abs(fd) + 1e-7 * scale), (g, fd)
    # replay reproduces the traced map exactly
    rr = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, replay_hits=hits)
    assert np.allclose(rr.map, base.map, rtol=1e-13, atol=0)


def test_two_ray_analytic_permittivity_derivative(oracle_lib):
    """d/d(eps_r) of the ground-reflected V-pol map vs the closed form.

    Closed form: d|r_par|^2/d(eps_r) from eq. fresnel (general form) by complex
    central differences in eta, integrated over each cell; the oracle's
    forward-mode gradient of sum(map over a set of cells) must agree within the
    Monte-Carlo tolerance of the map itself.
    """
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    sc = sg.ground_quad(100.0)
    G = np.ones((1, 30, 30))
    r = _run(oracle_lib, sc, tx, pl, 2_000_000, 1, grad_map=G)
    e0 = cf.eta(5.24, 0.12, FREQ)
    h = 1e-6
    dref = (cf.reflected_only_map(tx.pos, pl, LAM, e0 + h, "V") - cf.reflected_only_map(tx.pos, pl, LAM, e0 - h, "V")) / (2 * h)
    assert r.grad[0] == pytest.approx(dref.sum(), rel=3e-3)
    # d/d sigma = Re part through d eta/d sigma = -j/(eps0 omega)
    ds = -1j / (cf.EPS0 * 2 * math.pi * FREQ)
    dref_s = (cf.reflected_only_map(tx.pos, pl, LAM, e0 + h * ds, "V") - cf.reflected_only_map(tx.pos, pl, LAM, e0 - h * ds, "V")) / (2 * h)
    assert r.grad[1] == pytest.approx(dref_s.sum(), rel=3e-3)


# ----------------------------------------------------------- bookkeeping
def test_ray_ranges_and_lists_are_additive(oracle_lib):
    cfg = sg.tiny_config(n_rays=5000)
    full = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, want_hits=True)
    a = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_begin=0, ray_end=1777)
    b = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_begin=1777, ray_end=5000)
    assert np.allclose(a.map + b.map, full.map, rtol=1e-12, atol=0)
    assert np.array_equal(a.counts + b.counts, full.counts)
    ids = np.array([4999, 3, 1776, 1777])
    lst = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_ids=ids, want_hits=True)
    assert np.array_equal(lst.hits, full.hits[ids])


def test_flags_on_shared_edge_and_tie(oracle_lib):
    """The straight-down ray of the tiny scene lands on the ground-quad diagonal: edge-flagged.
    Two coincident triangles produce a tie that the smaller index wins."""
    cfg = sg.tiny_config(n_rays=101)
    r = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_ids=[100], want_hits=True)
    assert r.flags[0, 0] & oracle_lib.FLAG_EDGE
    assert r.flags[0, 0] & oracle_lib.FLAG_POLAR
    V = np.array([[-5, -5, 0], [5, -5, 0], [0, 5, 0]], np.float32)
    sc = sg.Scene(np.concatenate([V, V]), np.array([[0, 1, 2], [3, 4, 5]], np.int32),
                  np.zeros(2, np.int32), np.array([5.24]), np.array([0.12]))
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -1, -1, 1, 1, 2, 2)
    r = oracle_lib.radio_map(sc, tx, pl, sg.Params(FREQ, 101, 1), ray_ids=[100], want_hits=True)
    assert r.hits[0, 0] == 0 and r.flags[0, 0] & oracle_lib.FLAG_TIE


def test_degenerate_inputs(oracle_lib):
    """Empty scene, single ray, depth 0, rejection of invalid arguments."""
    pl = sg.Plane(1.5, -10, -10, 1, 1, 20, 20)
    r = oracle_lib.radio_map(sg.empty_scene(), sg.Tx((0, 0, 10)), pl, sg.Params(FREQ, 1, 0), want_hits=True)
    assert r.hits.shape == (1, 1) and r.hits[0, 0] == -1 and r.map.sum() == 0.0   # horizontal ray
    with pytest.raises(ValueError):
        oracle_lib.radio_map(sg.empty_scene(), sg.Tx((0, 0, 10)), pl, sg.Params(FREQ, 0, 0))
    bad = sg.tiny_scene()
    bad.tri_material = bad.tri_material.copy()
    bad.tri_material[3] = 7
    with pytest.raises(ValueError):
        oracle_lib.radio_map(bad, sg.Tx((0, 0, 10)), pl, sg.Params(FREQ, 10, 1))


# ------------------------------------------------- synthetic transmit array
def _steered_ula(n, spacing, c0):
    """Uniform linear array along x, weights steering toward x-cosine c0."""
    base = sg.linear_array(n, spacing)
    d = base.positions[:, 0]
    u = np.exp(-2j * math.pi * d / LAM * c0) / math.sqrt(n)
    return sg.TxArray(base.positions, u.astype(np.complex64))


def test_array_single_element_is_identity(oracle_lib):
    """One element at the array centre with a unit-modulus weight leaves the
    map unchanged (alpha = u, |alpha| = 1)."""
    cfg = sg.tiny_config(n_rays=20_000)
    base = _run(oracle_lib, cfg.scene, cfg.tx, cfg.plane, 20_000, 3)
    one = sg.TxArray(np.zeros((1, 3)), np.ones(1, np.complex64))
    r1 = _run(oracle_lib, cfg.scene, sg.Tx(cfg.tx.pos, array=one), cfg.plane, 20_000, 3)
    assert np.array_equal(r1.map, base.map)
    ph = sg.TxArray(np.zeros((1, 3)), np.array([np.exp(0.7j)], np.complex64))
    r2 = _run(oracle_lib, cfg.scene, sg.Tx(cfg.tx.pos, array=ph), cfg.plane, 20_000, 3)
    np.testing.assert_allclose(r2.map, base.map, rtol=1e-6)


def test_array_ula_dirichlet(oracle_lib):
    """Empty scene: every crossing's weight is the single-element weight times
    the Dirichlet kernel of a steered 8-element half-wavelength ULA evaluated
    at the ray's launch direction (closed form of eq. path-solver-array-
    response-vector with a steering precoding vector)."""
    N = 30_000
    n, c0 = 8, 0.3
    pl = sg.Plane(1.5, -40.0, -40.0, 1.0, 1.0, 80, 80)
    tx0 = sg.Tx((0.0, 0.0, 10.0))
    tx1 = sg.Tx((0.0, 0.0, 10.0), array=_steered_ula(n, 0.5 * LAM, c0))
    r0 = _run(oracle_lib, sg.empty_scene(), tx0, pl, N, 0, want_records=True)
    r1 = _run(oracle_lib, sg.empty_scene(), tx1, pl, N, 0, want_records=True)
    assert np.array_equal(r0.records["ray"], r1.records["ray"])
    assert r0.records["ray"].size > 5_000
    k = cf.lattice_directions(r0.records["ray"], N)
    ref = cf.dirichlet_gain(n, 0.5, k[:, 0], c0)
    ratio = r1.records["w"] / r0.records["w"]
    # weights are stored in float32: allow their rounding
    np.testing.assert_allclose(ratio, ref, rtol=2e-6, atol=2e-6 * n)
    assert ratio.max() > 0.9 * n and ratio.min() < 1e-2      # main lobe and nulls both sampled


def test_array_gain_applies_per_ray_at_every_depth(oracle_lib):
    """Ground-only scene: alpha depends only on the departure direction, so
    the direct and the ground-reflected crossing of one ray are scaled alike."""
    N = 40_000
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    ant = sg.random_array(6, 0.2, seed=11)
    r0 = _run(oracle_lib, sg.ground_quad(100.0), sg.Tx((0.0, 0.0, 10.0)), pl, N, 2, want_records=True)
    r1 = _run(oracle_lib, sg.ground_quad(100.0), sg.Tx((0.0, 0.0, 10.0), array=ant), pl, N, 2,
              want_records=True)
    assert np.array_equal(r0.records["ray"], r1.records["ray"])
    assert np.array_equal(r0.records["depth"], r1.records["depth"])
    ratio = r1.records["w"] / r0.records["w"]
    rays = r0.records["ray"]
    both = [n for n in np.unique(rays) if (rays == n).sum() == 2]
    assert len(both) > 1_000
    for n in both[:2000]:
        a, b = ratio[rays == n]
        assert abs(a - b) <= 1e-9 * max(a, b, 1e-12)


# ---------------------------------------- early termination (Russian roulette)
def test_philox_known_answers(oracle_lib):
    """The generator that drives Russian roulette reproduces the published
    Philox4x32-10 known-answer vectors (tests/golden/philox4x32_10_kat.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        out = oracle_lib.philox4x32(w[0:4], w[4:6])
        assert [int(v) for v in out] == w[6:10]
        n += 1
    assert n == 3


def _rr_params(N, L, **kw):
    return sg.Params(FREQ, N, L, **kw)


def test_roulette_depth_gating_and_threshold_limits(oracle_lib):
    """Termination from a depth beyond L changes nothing; a vanishing gain
    threshold changes nothing; an infinite one leaves only the direct (depth-0)
    contributions."""
    cfg = sg.tiny_config(n_rays=30_000)
    base = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(30_000, 3))
    off = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane,
                               _rr_params(30_000, 3, rr_depth=4, rr_p_max=0.5, gain_threshold=1.0))
    assert np.array_equal(off.map, base.map)
    tiny = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(30_000, 3, gain_threshold=1e-300))
    assert np.array_equal(tiny.map, base.map)
    d0 = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(30_000, 0))
    inf = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(30_000, 3, gain_threshold=1e300))
    assert np.array_equal(inf.map, d0.map)


def test_roulette_reweights_survivors_by_one_over_p(oracle_lib):
    """With p_max below every path's distance-normalised gain, p = p_max for
    all paths: a ray survives its roulette iff its uniform is below p_max, and
    each surviving crossing weighs exactly 1/p_max times the unterminated one."""
    N, pmax = 20_000, 0.02
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_H)     # |r_perp|^2 >= 0.155 on concrete: never below p_max
    scene = sg.ground_quad(100.0)
    r0 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1), want_records=True, want_hits=True)
    r1 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1, rr_p_max=pmax, seed=77), want_records=True,
                              want_hits=True)
    traced1 = r0.hits[:, 1] != -2            # rays that reach a second segment without roulette
    surv = r1.hits[:, 1] != -2
    assert np.all(surv <= traced1)
    # the decision follows the counter-based stream: uniform of (ray, depth 1)
    u = np.array([(int(oracle_lib.philox4x32([n & 0xffffffff, n >> 32, 1, 0], [77, 0])[0]) >> 8) / 2.0 ** 24
                  for n in np.nonzero(traced1)[0]])
    assert np.array_equal(surv[traced1], u < pmax)
    assert 0.5 * pmax < surv[traced1].mean() < 2.0 * pmax
    w0 = {(int(a), int(b)): w for a, b, w in zip(r0.records["ray"], r0.records["depth"], r0.records["w"])}
    n1 = 0
    for a, b, w in zip(r1.records["ray"], r1.records["depth"], r1.records["w"]):
        ref = w0[(int(a), int(b))]
        if b == 0:
            assert w == ref
        else:
            assert abs(w * pmax - ref) <= 1e-12 * ref
            n1 += 1
    assert n1 > 20


def test_roulette_is_unbiased(oracle_lib):
    """Russian roulette with p = min(||E||^2, p_max) keeps the estimator
    unbiased: the total reflected power with roulette matches the one without
    within four standard errors (seeded, so the outcome is fixed)."""
    N = 200_000
    cfg = sg.tiny_config(n_rays=N)
    r0 = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(N, 3), want_records=True)
    r1 = oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, _rr_params(N, 3, rr_p_max=0.9, seed=5),
                              want_records=True)
    def reflected_per_ray(r):
        m = r.records["depth"] >= 1
        return np.bincount(r.records["ray"][m], weights=r.records["w"][m], minlength=N)
    a, b = reflected_per_ray(r0), reflected_per_ray(r1)
    assert np.count_nonzero(b) < 0.9 * np.count_nonzero(a)      # roulette did remove paths
    se = np.std(b - a) * math.sqrt(N)
    assert abs(b.sum() - a.sum()) <= 4.0 * se
    assert abs(b.sum() / a.sum() - 1.0) < 0.05


def test_roulette_probability_is_the_normalised_gain(oracle_lib):
    """H-pol over a horizontal ground: after the bounce ||E||^2 = |r_perp|^2
    (textbook Fresnel via Snell's law at cos(theta_i) = |k_z|), so with
    p_max = 1 a ray survives its roulette iff its uniform is below that."""
    N = 20_000
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_H)
    scene = sg.ground_quad(100.0)
    r0 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1), want_hits=True)
    r1 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1, rr_p_max=1.0, seed=3), want_hits=True)
    rays = np.nonzero(r0.hits[:, 1] != -2)[0]
    k = cf.lattice_directions(rays, N)
    rp, _ = cf.fresnel_general(cf.eta(5.24, 0.12, FREQ), np.abs(k[:, 2]))
    p = np.abs(rp) ** 2
    u = np.array([(int(oracle_lib.philox4x32([int(n) & 0xffffffff, int(n) >> 32, 1, 0], [3, 0])[0]) >> 8) / 2.0 ** 24
                  for n in rays])
    clear = np.abs(u - p) > 1e-9
    surv = r1.hits[rays, 1] != -2
    assert clear.sum() > 0.99 * rays.size
    assert np.array_equal(surv[clear], (u < p)[clear])
    assert 0.1 < surv.mean() < 0.9


def _philox_word0(n, l, stream, seed):
    return (int(sg_philox(n, l, stream, seed)) >> 8) / 2.0 ** 24


def sg_philox(n, l, stream, seed):
    import oracle
    return oracle.philox4x32([int(n) & 0xffffffff, int(n) >> 32, l, stream], [seed, 0])[0]


def test_gain_threshold_specular_closed_form(oracle_lib):
    """Gain thresholding (Sec. "Practical Notes"): H-pol over a horizontal
    concrete ground (pure TE, ||E||^2 = |r_perp(theta_i)|^2 after the bounce,
    textbook Fresnel via Snell's law at cos(theta_i) = |k_z|).  Before segment
    1 the path gain at the tube length r = h/|k_z| (the distance from the
    source to the ground point) is (lambda / (4 pi r))^2 |r_perp|^2; with the
    threshold at the median of that gain a ray's reflected segment is traced
    iff its gain is at least the threshold.  With rr_depth = 2 the check
    never runs at L = 1.  A missing 1/(16 pi^2), lambda in place of lambda^2,
    or the check before another segment moves the set of survivors."""
    N, h = 20_000, 10.0
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    tx = sg.Tx((0.0, 0.0, h), pol=sg.POL_H)
    scene = sg.ground_quad(100.0)
    r0 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1), want_hits=True)
    rays = np.nonzero(r0.hits[:, 0] >= 0)[0]           # down-going rays that hit the ground
    assert rays.size > 0.45 * N
    k = cf.lattice_directions(rays, N)
    rp, _ = cf.fresnel_general(cf.eta(*CONCRETE_EPS_SIGMA, FREQ), np.abs(k[:, 2]))
    r = h / np.abs(k[:, 2])
    gain = (LAM / (4.0 * math.pi * r)) ** 2 * np.abs(rp) ** 2
    thr = float(np.median(gain))
    r1 = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1, gain_threshold=thr), want_hits=True)
    surv = r1.hits[rays, 1] != -2
    clear = np.abs(gain / thr - 1.0) > 1e-9
    assert clear.sum() > rays.size - 4
    assert np.array_equal(surv[clear], (gain >= thr)[clear])
    assert 0.4 < surv.mean() < 0.6
    # rays that miss the ground are never thresholded (they have no bounce)
    assert np.all(r1.hits[r0.hits[:, 0] < 0, 1] == -2)
    gated = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 1, gain_threshold=thr, rr_depth=2), want_hits=True)
    assert np.array_equal(gated.hits, r0.hits)


CONCRETE_EPS_SIGMA = (5.24, 0.12)
METAL_EPS_SIGMA = (1.0, 1.0e7)


def test_gain_threshold_restarts_at_a_diffuse_point(oracle_lib):
    """A diffuse point starts a new ray tube (Sec. "Definition of Radio Map":
    the scattered field is that of a new source at the diffuse point), so the
    gain threshold measures the tube from there.  Fully diffuse concrete ground
    (S = 1, K_x = 0, Lambertian) under a metal ceiling at z = 20 m, H-pol
    source at 10 m: a down-going ray scatters at the ground in the direction
    whose polar cosine u0 is word 0 of the Philox block at (ray, 0, 2) (no
    check right after the diffuse point), reaches the ceiling after
    r2 = 20/u0, and before segment 2 its path gain is
        (lambda / (4 pi r2))^2 * 2 u0 |r_perp,ground(theta_i)|^2 |r_perp,metal(theta_s)|^2
    (the scattered field stays TE with K_x = 0; 2 cos(theta_s) Gamma^2 is the
    Lambertian field factor with q(S) = 1).  With the threshold at its median,
    segment 2 is traced iff the gain reaches it; measuring from the source
    (r1 + r2) instead would keep a different set."""
    N, seed = 20_000, 21
    mb = sg._MeshBuilder()
    mb.quad((-100.0, -100.0, 0.0), (100.0, -100.0, 0.0), (100.0, 100.0, 0.0), (-100.0, 100.0, 0.0), 0)
    mb.quad((-100.0, -100.0, 20.0), (100.0, -100.0, 20.0), (100.0, 100.0, 20.0), (-100.0, 100.0, 20.0), 1)
    scene = sg.with_diffuse(mb.build([CONCRETE_EPS_SIGMA, METAL_EPS_SIGMA], "ground+ceiling"), [1.0, 0.0], [0.0, 0.0])
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_H)
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    base = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 2, seed=seed), want_hits=True)
    n = np.arange(N)
    k = cf.lattice_directions(n, N)
    down = k[:, 2] < -0.05
    u0 = np.array([_philox_word0(i, 0, 2, seed) for i in n])
    tan_i = np.sqrt(1.0 - k[:, 2] ** 2) / np.abs(np.where(down, k[:, 2], 1.0))
    tan_s = np.sqrt(np.maximum(0.0, 1.0 - u0 ** 2)) / np.maximum(u0, 1e-12)
    reach = 10.0 * tan_i + 20.0 * tan_s                  # horizontal distance to the ceiling point
    sel = down & (u0 > 0.05) & (reach < 90.0)
    rays = n[sel]
    assert rays.size > 0.2 * N
    assert np.all(np.isin(base.hits[rays, 0], [0, 1]))      # the ground quad
    assert np.all(np.isin(base.hits[rays, 1], [2, 3]))      # the ceiling quad
    rg, _ = cf.fresnel_general(cf.eta(*CONCRETE_EPS_SIGMA, FREQ), np.abs(k[sel, 2]))
    rm, _ = cf.fresnel_general(cf.eta(*METAL_EPS_SIGMA, FREQ), u0[sel])
    r2 = 20.0 / u0[sel]
    r1 = 10.0 / np.abs(k[sel, 2])
    amp = 2.0 * u0[sel] * np.abs(rg) ** 2 * np.abs(rm) ** 2
    gain = (LAM / (4.0 * math.pi * r2)) ** 2 * amp
    thr = float(np.median(gain))
    th = oracle_lib.radio_map(scene, tx, pl, _rr_params(N, 2, seed=seed, gain_threshold=thr), want_hits=True)
    # no check right at the diffuse point: every ray that first meets the
    # ground traces its next segment (rays that first meet the specular
    # ceiling are checked there, with their tube measured from the source)
    gnd = np.isin(base.hits[:, 0], [0, 1])
    assert np.array_equal(th.hits[gnd, :2], base.hits[gnd, :2])
    assert np.any(th.hits[~gnd, 1] != base.hits[~gnd, 1])
    surv = th.hits[rays, 2] != -2
    clear = np.abs(gain / thr - 1.0) > 1e-9
    assert clear.sum() > rays.size - 4
    assert np.array_equal(surv[clear], (gain >= thr)[clear])
    unfolded = (LAM / (4.0 * math.pi * (r1 + r2))) ** 2 * amp >= thr
    assert np.count_nonzero(unfolded != (gain >= thr)) > 0.1 * rays.size
