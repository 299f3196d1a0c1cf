"""Pins of the oracle's diffuse reflection (App. "Diffuse Reflection",
eq. scattered_field with the Lambertian pattern eq. lambertian_model; the
estimator eq. radio-map-solver-ci-all-2-estimator with its (2 pi)^n_S and
r^2 / |n^T k| factors; the interaction shares of
eq. path-solver-used-dist-event with R = sqrt(1 - S^2), eq. R).

* A fully diffuse ground (S = 1): the depth-1 map equals the closed-form
  scattering integral over the ground for V- and H-polarised sources
  (Gamma^2 = |r_par|^2 and |r_perp|^2), per cell within the Monte-Carlo
  error and in aggregate.
* Cross-polarisation: with a specular ceiling above the diffuse ground the
  ground -> ceiling -> plane paths weigh |r_par|^2 (K_x = 0) or |r_perp|^2
  (K_x = 1) of the ceiling, against the same integral seen from the image of
  the plane point, and every crossing for K_x = 1/2 is the mean of the two.
* Gradients: over a fully diffuse ground an H-polarised crossing weighs
  Gamma^2 = |r_perp|^2 of its incidence angle, so d w = w d ln|r_perp|^2 from
  eq. fresnel; on a two-material scene without refraction the draws do not
  depend on the parameters and the forward-mode gradient equals central
  differences of the oracle's own map.
* Shares: with S = 0.6 a ray reflects specularly iff its draw is below
  q(R) = 1 - S^2, and then its weights equal those of a non-diffuse ground
  (R^2 / q(R) = 1); S = 0 changes nothing.
CPU only.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import scenegen as sg

FREQ = 3.5e9
LAM = cf.wavelength(FREQ)
ETA_C = cf.eta(5.24, 0.12, FREQ)


def _cell_stats(res, plane, depth, rays=None):
    r = res.records
    sel = r["depth"] == depth
    if rays is not None:
        sel &= np.isin(r["ray"], rays)
    W = plane.W * plane.H
    s1 = np.bincount(r["cell"][sel], weights=r["w"][sel], minlength=W).reshape(plane.H, plane.W)
    s2 = np.bincount(r["cell"][sel], weights=r["w"][sel] ** 2, minlength=W).reshape(plane.H, plane.W)
    n = np.bincount(r["cell"][sel], minlength=W).reshape(plane.H, plane.W)
    return s1, s2, n


@pytest.mark.parametrize("pol", ["V", "H"])
def test_lambertian_ground_matches_scattering_integral(oracle_lib, pol):
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_V if pol == "V" else sg.POL_H)
    pl = sg.Plane(1.5, -30.0, -30.0, 4.0, 4.0, 15, 15)
    g = sg.with_diffuse(sg.ground_quad(100.0), 1.0, 0.0)
    res = oracle_lib.radio_map_parallel(g, tx, pl, sg.Params(FREQ, 2_000_000, 1, seed=4), workers=8,
                                        want_records=True)
    s1, s2, n = _cell_stats(res, pl, 1)
    ref = cf.lambertian_ground_map(tx.pos, pl, LAM, ETA_C, pol, 100.0, n_beta=96, n_psi=192, n_cell=3)
    assert n.min() >= 300
    z = (s1 - ref) / np.sqrt(s2)
    assert np.abs(z).max() <= 4.5, np.abs(z).max()
    assert abs(s1.sum() / ref.sum() - 1) <= 3e-3
    # V and H differ by more than the tolerance: Gamma follows the polarisation
    other = cf.lambertian_ground_map(tx.pos, pl, LAM, ETA_C, "H" if pol == "V" else "V", 100.0,
                                     n_beta=48, n_psi=96, n_cell=2)
    assert abs(s1.sum() / other.sum() - 1) > 0.05


def test_cross_polarisation_share(oracle_lib):
    mb = sg._MeshBuilder()
    mb.quad((-100.0, -100.0, 0.0), (100.0, -100.0, 0.0), (100.0, 100.0, 0.0), (-100.0, 100.0, 0.0), 0)
    mb.quad((-100.0, -100.0, 20.0), (-100.0, 100.0, 20.0), (100.0, 100.0, 20.0), (100.0, -100.0, 20.0), 1)
    base = mb.build([sg.CONCRETE, sg.CONCRETE], "ground+ceiling")
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 6.0, 6.0, 10, 10)
    p = sg.Params(FREQ, 2_000_000, 2, seed=6)
    runs = {}
    for K in (0.0, 1.0, 0.5):
        sc = sg.with_diffuse(base, [1.0, 0.0], [K, 0.0])
        runs[K] = oracle_lib.radio_map_parallel(sc, tx, pl, p, workers=8, want_hits=True, want_records=True)
    h = runs[0.0].hits
    rays = np.nonzero((h[:, 0] >= 0) & (h[:, 0] <= 1) & (h[:, 1] >= 2))[0]     # ground, then ceiling
    assert rays.size > 100_000
    for K, side in ((0.0, "par"), (1.0, "perp")):
        s1, s2, n = _cell_stats(runs[K], pl, 2, rays)
        ref = cf.lambertian_ground_map(tx.pos, pl, LAM, ETA_C, "V", 100.0, ceiling=(20.0, ETA_C, side),
                                       n_beta=96, n_psi=192, n_cell=3)
        z = (s1 - ref) / np.sqrt(s2)
        assert n.min() >= 300 and np.abs(z).max() <= 4.5, (K, np.abs(z).max())
        assert abs(s1.sum() / ref.sum() - 1) <= 5e-3, (K, s1.sum() / ref.sum())
    # per crossing: K = 1/2 splits the scattered power evenly between the two
    r0, r1, rh = runs[0.0].records, runs[1.0].records, runs[0.5].records
    assert np.array_equal(r0["ray"], rh["ray"]) and np.array_equal(r0["depth"], rh["depth"])
    d2 = r0["depth"] == 2
    np.testing.assert_allclose(rh["w"][d2], 0.5 * (r0["w"][d2] + r1["w"][d2]), rtol=1e-12)


def test_specular_share_of_a_partly_diffuse_ground(oracle_lib):
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -60.0, -60.0, 2.0, 2.0, 60, 60)
    N = 200_000
    g = sg.ground_quad(100.0)
    plain = oracle_lib.radio_map(g, tx, pl, sg.Params(FREQ, N, 1), want_records=True)
    zero = oracle_lib.radio_map(sg.with_diffuse(g, 0.0, 0.3), tx, pl, sg.Params(FREQ, N, 1, seed=2))
    np.testing.assert_array_equal(zero.map, plain.map)
    part = oracle_lib.radio_map(sg.with_diffuse(g, 0.6, 0.3), tx, pl, sg.Params(FREQ, N, 1, seed=2),
                                want_records=True)
    pk = dict(zip(plain.records["ray"][plain.records["depth"] == 1].tolist(),
                  plain.records["w"][plain.records["depth"] == 1].tolist()))
    cand = np.array(sorted(pk))
    u = np.array([oracle_lib.uniform(2, n, 0, 1) for n in cand])
    spec = cand[u < 0.64 - 1e-9]
    sel = (part.records["depth"] == 1) & np.isin(part.records["ray"], spec)
    got = dict(zip(part.records["ray"][sel].tolist(), part.records["w"][sel].tolist()))
    assert len(got) == spec.size
    np.testing.assert_allclose([got[k] for k in spec.tolist()], [pk[k] for k in spec.tolist()], rtol=1e-12)
    q = 0.64
    assert abs(spec.size - q * cand.size) <= 5 * math.sqrt(cand.size * q * (1 - q))
    # the diffuse rays carry S^2 / q(S) = 1 of the fully diffuse ground's
    # scattering: their crossings sum to S^2 times its integral
    pl2 = sg.Plane(1.5, -30.0, -30.0, 4.0, 4.0, 15, 15)
    N2 = 1_000_000
    d = oracle_lib.radio_map_parallel(sg.with_diffuse(g, 0.6, 0.3), tx, pl2, sg.Params(FREQ, N2, 1, seed=8),
                                      workers=8, want_records=True)
    r = d.records
    dep = r["depth"] == 1
    u2 = np.array([oracle_lib.uniform(8, n, 0, 1) for n in r["ray"][dep]])
    diffuse = u2 >= 0.64 + 1e-9
    ref = cf.lambertian_ground_map(tx.pos, pl2, LAM, ETA_C, "V", 100.0, n_beta=96, n_psi=192, n_cell=3)
    assert abs(r["w"][dep][diffuse].sum() / (0.36 * ref.sum()) - 1) <= 0.02


def test_diffuse_inputs_validated(oracle_lib):
    cfg = sg.tiny_config(n_rays=100)
    for S, K in ((1.5, 0.0), (0.5, -0.1), (0.5, 2.0)):
        with pytest.raises(ValueError):
            oracle_lib.radio_map(sg.with_diffuse(cfg.scene, S, K), cfg.tx, cfg.plane, cfg.params)
    with pytest.raises(ValueError):          # Gamma depends on the field: one polarisation only
        oracle_lib.radio_map(sg.with_diffuse(cfg.scene, 0.5), sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_DUAL),
                             cfg.plane, cfg.params)


@pytest.mark.parametrize("pp", [(1, 1, 1, 1.0), (1, 4, 1, 1.0), (1, 13, 1, 1.0), (2, 3, 2, 0.3), (2, 8, 5, 0.7)])
def test_scattering_pattern_normalisation(oracle_lib, pp):
    """eq. directive_model and eq. backscattering_model: the closed-form
    F_alpha(theta_i) makes the pattern integrate to 1 over the hemisphere
    (checked by quadrature at several incidence angles); the lobes peak at
    the specular direction and, for backscattering, toward the source."""
    pp = np.array(pp, dtype=np.float64)
    g, w = np.polynomial.legendre.leggauss(48)
    mu = (g + 1) / 2
    ph = (np.arange(96) + 0.5) * 2 * math.pi / 96
    n = np.array([0.0, 0.0, 1.0])
    for ci in (0.99, 0.7, 0.3, 0.05):
        si = math.sqrt(1 - ci * ci)
        ki = np.array([si, 0.0, -ci])
        tot = 0.0
        for m, wm in zip(mu, w / 2):
            st = math.sqrt(1 - m * m)
            for p_ in ph:
                ks = np.array([st * math.cos(p_), st * math.sin(p_), m])
                tot += wm * oracle_lib.scatter_pattern(pp, ki, ks, n) * 2 * math.pi / 96
        assert abs(tot - 1) < 1e-6, (pp, ci, tot)
        kr = np.array([si, 0.0, ci])
        f_r = oracle_lib.scatter_pattern(pp, ki, kr, n)
        off = np.array([-si, 0.3, ci]) / np.linalg.norm([-si, 0.3, ci])
        if pp[0] == 1:
            assert f_r > oracle_lib.scatter_pattern(pp, ki, off, n)
        else:
            back = -ki
            assert oracle_lib.scatter_pattern(pp, ki, back, n) > oracle_lib.scatter_pattern(
                pp, ki, np.array([0.0, 1.0, 0.0]), n)


@pytest.mark.parametrize("pp", [(1, 3, 1, 1.0), (2, 2, 4, 0.5)])
def test_directive_ground_matches_scattering_integral(oracle_lib, pp):
    """A fully diffuse ground with a directive (or backscattering) pattern:
    the depth-1 map equals the scattering integral with that pattern, whose
    normalisation is taken by quadrature (independent of the closed-form F
    of the oracle); the pattern evaluation itself is checked against the
    oracle's at sample directions."""
    pp = np.array(pp, dtype=np.float64)
    lobe2 = None if pp[0] == 1 else (int(pp[2]), pp[3])
    fn = lambda ki, ks, n: cf.directive_pattern(int(pp[1]), ki, ks, n, lobe2)
    rng = np.random.default_rng(1)
    for _ in range(20):
        ci = rng.uniform(0.05, 1.0)
        ki = np.array([math.sqrt(1 - ci * ci), 0.0, -ci])
        v = rng.standard_normal(3)
        v[2] = abs(v[2])
        ks = v / np.linalg.norm(v)
        n = np.array([0.0, 0.0, 1.0])
        assert fn(ki[None], ks[None], n[None])[0] == pytest.approx(oracle_lib.scatter_pattern(pp, ki, ks, n),
                                                                  rel=1e-6)
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 4.0, 4.0, 15, 15)
    g = sg.with_diffuse(sg.ground_quad(100.0), 1.0, 0.0, pp)
    res = oracle_lib.radio_map_parallel(g, tx, pl, sg.Params(FREQ, 2_000_000, 1, seed=4), workers=8,
                                        want_records=True)
    s1, s2, n = _cell_stats(res, pl, 1)
    ref = cf.lambertian_ground_map(tx.pos, pl, LAM, ETA_C, "V", 100.0, n_beta=96, n_psi=192, n_cell=3,
                                   pattern=fn)
    z = (s1 - ref) / np.sqrt(s2)
    assert n.min() >= 100 and np.abs(z).max() <= 4.5, np.abs(z).max()
    assert abs(s1.sum() / ref.sum() - 1) <= 5e-3, s1.sum() / ref.sum()


def _dlog_rperp2(eps, sig, cos_t, which, h=1e-6):
    """d ln|r_perp|^2 / d eps_r (which = 0) or d sigma (which = 1), eq. fresnel,
    central differences."""
    def r2(e, g):
        return np.abs(cf.fresnel_general(cf.eta(e, g, FREQ), cos_t)[0]) ** 2
    if which == 0:
        return (r2(eps + h, sig) - r2(eps - h, sig)) / (2 * h * r2(eps, sig))
    return (r2(eps, sig + h) - r2(eps, sig - h)) / (2 * h * r2(eps, sig))


def test_diffuse_gradient_of_a_single_scatter(oracle_lib):
    """H-pol over a fully diffuse ground (S = 1, so q(S) = 1) is pure TE:
    a depth-1 crossing weighs w = kappa 2 pi f_s Gamma^2 ||E||^2 / |k_z'| with
    Gamma^2 = |r_perp|^2 at the launch angle; the cross-polarisation matrix
    (K_x = 0.3) is unitary and the draws are fixed, so dw = w d ln|r_perp|^2."""
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_H)
    pl = sg.Plane(1.5, -30.0, -30.0, 4.0, 4.0, 15, 15)
    N = 200_000
    g = sg.with_diffuse(sg.ground_quad(100.0), 1.0, 0.3)
    r = oracle_lib.radio_map(g, tx, pl, sg.Params(FREQ, N, 1, seed=8), want_records=True,
                             grad_map=np.ones((1, pl.H, pl.W)))
    sel = r.records["depth"] == 1
    assert sel.sum() > 1000
    kz = np.abs(np.array([oracle_lib.lattice(n, N)[2] for n in r.records["ray"][sel]]))
    w = r.records["w"][sel]
    for which in (0, 1):
        expect = np.sum(w * _dlog_rperp2(*sg.CONCRETE, kz, which))
        assert r.grad[which] == pytest.approx(expect, rel=2e-5), (which, r.grad[which], expect)


def test_diffuse_gradient_matches_central_differences(oracle_lib):
    """Ground (concrete, S = 0.7, K_x = 0.25) and a box (glass, S = 0.4,
    K_x = 0.1), directional V-pol source at yaw/pitch/roll (0.3, 0.2, -0.1),
    depth 3, no refraction: q(R) = 1 - S^2 and q(S) = S^2, the draws and the
    directions do not depend on (eps_r, sigma, yaw, pitch, roll), so
    sum(G * map) is smooth in them.  The forward-mode gradient, which carries
    the field dependence of Gamma^2 through every diffuse point, must equal
    FP64 central differences of the map along two random directions."""
    import dataclasses
    mb = sg._MeshBuilder()
    mb.quad((-100.0, -100.0, 0.0), (100.0, -100.0, 0.0), (100.0, 100.0, 0.0), (-100.0, 100.0, 0.0), 0)
    mb.box((30.0, -10.0, 0.0), (50.0, 10.0, 30.0), 1, bottom=False)
    scene = sg.with_diffuse(mb.build([sg.CONCRETE, sg.GLASS], "ground+box"), [0.7, 0.4], [0.25, 0.1])
    pl = sg.Plane(1.5, -100.0, -100.0, 4.0, 4.0, 50, 50)
    prm = sg.Params(FREQ, 20_000, 3, seed=21)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((1, pl.H, pl.W))
    theta0 = np.array([*scene.eps_r, *scene.sigma, 0.3, 0.2, -0.1])

    def run(theta, grad=False):
        sc = dataclasses.replace(scene, eps_r=theta[0:2].copy(), sigma=theta[2:4].copy())
        tx = sg.Tx((0.0, 0.0, 10.0), yaw=theta[4], pitch=theta[5], roll=theta[6],
                   pattern=sg.PATTERN_DIRECTIONAL)
        return oracle_lib.radio_map(sc, tx, pl, prm, grad_map=G if grad else None)

    res = run(theta0, grad=True)
    assert res.map[0, :, :].sum() > 0
    for _ in range(2):
        v = rng.uniform(-1.0, 1.0, theta0.size) * np.maximum(np.abs(theta0), 0.1)
        h = 1e-4
        fd = (np.sum(G * run(theta0 + h * v).map) - np.sum(G * run(theta0 - h * v).map)) / (2 * h)
        assert res.grad @ v == pytest.approx(fd, rel=1e-5), (res.grad @ v, fd)
