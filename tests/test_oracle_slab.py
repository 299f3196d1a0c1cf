"""Pins of the oracle's finite-thickness walls and interaction sampling.

* Slab coefficients (Sec. "Single-Layer Slab", eq. fresnel_slab,
  eq. q_fresnel_slab) against the optical characteristic-matrix method, an
  independent route (one 2x2 matrix per layer, no Fresnel coefficients of the
  interfaces), and against their limits: a vanishing slab, a half-wave slab,
  a thick lossy slab and energy conservation without loss.
* Interaction sampling (eq. path-solver-used-dist-event with S = 0, R = 1,
  q(D) = 0) and the Pr(chi)^-1 factor of eq. radio-map-solver-ci-all-2-
  estimator: the counter layout of its random stream, the two degenerate
  walls (transparent: every ray passes; opaque: every ray reflects), and the
  exact 1/q reweighting with the reflection frequency of a glass ground.
CPU only.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import scenegen as sg

FREQ = 3.5e9
LAM = cf.wavelength(FREQ)
MATS = [(5.24, 0.12, 0.2), (6.31, 0.05, 0.01), (5.24, 0.0, 0.05), (3.0, 0.3, 0.3), (15.0, 0.02, 0.12)]
COS = (1.0, 0.97, 0.8, 0.5, 0.2, 0.05)


def test_slab_matches_characteristic_matrix(oracle_lib):
    """eq. fresnel_slab equals the Born-Wolf layer matrix, phases included
    (r_par = -r_p: the matrix method refers r_p to the tangential field)."""
    for e, s, d in MATS:
        for c in COS:
            rperp, rpar, tperp, tpar = oracle_lib.fresnel_slab(e, s, FREQ, c, d)
            rs, rp, ts, tp = cf.slab_characteristic(cf.eta(e, s, FREQ), c, d, LAM)
            for got, ref in ((rperp, rs), (rpar, -rp), (tperp, ts), (tpar, tp)):
                assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-15, (e, s, d, c, got, ref)


def test_slab_limits(oracle_lib):
    """d = 0 is transparent; a lossless half-wave slab reflects nothing and
    passes -1; a thick lossy slab reflects like the half-space and passes
    nothing; without loss |r|^2 + |t|^2 = 1 (Airy)."""
    for e, s, _ in MATS:
        for c in COS:
            rperp, rpar, tperp, tpar = oracle_lib.fresnel_slab(e, s, FREQ, c, 0.0)
            assert rperp == 0 and rpar == 0 and abs(tperp - 1) < 1e-15 and abs(tpar - 1) < 1e-15
    e, c = 5.24, 0.6
    q1 = 2 * math.pi / LAM * math.sqrt(e - (1 - c * c))      # phase thickness per metre
    rperp, rpar, tperp, tpar = oracle_lib.fresnel_slab(e, 0.0, FREQ, c, math.pi / q1)
    assert abs(rperp) < 1e-12 and abs(rpar) < 1e-12
    assert abs(tperp + 1) < 1e-12 and abs(tpar + 1) < 1e-12
    rp0, rl0 = oracle_lib.fresnel(5.24, 0.12, FREQ, c)
    rperp, rpar, tperp, tpar = oracle_lib.fresnel_slab(5.24, 0.12, FREQ, c, 50.0)
    assert abs(rperp - rp0) < 1e-12 and abs(rpar - rl0) < 1e-12
    assert abs(tperp) < 1e-12 and abs(tpar) < 1e-12
    for c in COS:
        for d in (0.013, 0.2, 0.71):
            rperp, rpar, tperp, tpar = oracle_lib.fresnel_slab(5.24, 0.0, FREQ, c, d)
            assert abs(abs(rperp) ** 2 + abs(tperp) ** 2 - 1) < 1e-12
            assert abs(abs(rpar) ** 2 + abs(tpar) ** 2 - 1) < 1e-12
            # Airy: |t|^2 = (1-R)^2 / ((1-R)^2 + 4 R sin^2(delta)), R = |r'|^2
            rs, rl = cf.fresnel_general(5.24, c)
            delta = 2 * math.pi / LAM * d * math.sqrt(5.24 - (1 - c * c))
            for r1, t in ((rs, tperp), (rl, tpar)):
                R = abs(r1) ** 2
                airy = (1 - R) ** 2 / ((1 - R) ** 2 + 4 * R * math.sin(delta) ** 2)
                assert abs(abs(t) ** 2 - airy) < 1e-12


def test_interaction_stream_counter_layout(oracle_lib):
    """The interaction draw of ray n at the end of segment l is the top 24
    bits of Philox4x32-10 word 0 at counter (n_lo, n_hi, l, 1), key (seed, 0);
    the early-termination draw uses word 3 = 0 of the same counter."""
    for seed, n, l in ((0, 0, 0), (7, 123456, 3), (0xdeadbeef, (5 << 32) + 17, 2)):
        for stream in (0, 1):
            w = oracle_lib.philox4x32([n & 0xffffffff, n >> 32, l, stream], [seed, 0])
            assert oracle_lib.uniform(seed, n, l, stream) == (int(w[0]) >> 8) / 16777216.0
        assert oracle_lib.uniform(seed, n, l, 0) != oracle_lib.uniform(seed, n, l, 1)


def test_refraction_needs_a_thickness(oracle_lib):
    cfg = sg.tiny_config(n_rays=100)
    cfg.params.refraction = 1
    with pytest.raises(ValueError):
        oracle_lib.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params)


def test_transparent_ground_is_free_space(oracle_lib):
    """A zero-thickness ground has r = 0, t = 1: every hit transmits with
    q(T) = 1 and the map is the empty scene's, while every ray that reaches
    the ground passes through it."""
    tx = sg.Tx((3.0, -2.0, 12.0))
    pl = sg.Plane(1.5, -40.0, -40.0, 2.0, 2.0, 40, 40)
    p = sg.Params(FREQ, 200_000, 3, refraction=1, seed=3)
    sc = sg.with_thickness(sg.ground_quad(100.0), [0.0])
    r = oracle_lib.radio_map(sc, tx, pl, p, want_hits=True)
    e = oracle_lib.radio_map(sg.empty_scene(), tx, pl, sg.Params(FREQ, 200_000, 3))
    assert np.array_equal(r.counts, e.counts)
    np.testing.assert_allclose(r.map, e.map, rtol=1e-12, atol=0)
    down = r.hits[:, 0] >= 0
    assert down.sum() > 50_000 and np.all(r.hits[down, 1] == -1)


def test_opaque_ground_reflects_every_ray(oracle_lib):
    """A metal sheet (sigma = 1e7 S/m, 5 mm) passes t = 0 exactly: q(R) = 1,
    so sampling reflects every ray with weight 1 and the map equals the
    half-space specular map."""
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -30.0, -30.0, 2.0, 2.0, 30, 30)
    g = sg.ground_quad(100.0, sg.METAL)
    a = oracle_lib.radio_map(g, tx, pl, sg.Params(FREQ, 100_000, 2), want_hits=True)
    b = oracle_lib.radio_map(sg.with_thickness(g), tx, pl, sg.Params(FREQ, 100_000, 2, refraction=1, seed=5),
                             want_hits=True)
    assert np.array_equal(a.hits, b.hits)
    np.testing.assert_allclose(b.map, a.map, rtol=1e-14, atol=0)


def test_sampling_reweights_exactly_and_reflects_with_q(oracle_lib):
    """Glass ground (10 mm): a reflected crossing carries the deterministic
    slab-reflection weight divided by q(R), and the rays reflect with
    frequency q(R) (binomial, 5 sigma).  q(R) comes from the
    characteristic-matrix closed form at the ray's incidence angle."""
    tx = sg.Tx((0.0, 0.0, 10.0))
    pl = sg.Plane(1.5, -60.0, -60.0, 2.0, 2.0, 60, 60)
    N = 300_000
    g = sg.with_thickness(sg.ground_quad(100.0, sg.GLASS))
    det = oracle_lib.radio_map(g, tx, pl, sg.Params(FREQ, N, 1), want_records=True)
    smp = oracle_lib.radio_map(g, tx, pl, sg.Params(FREQ, N, 1, refraction=1, seed=11), want_records=True)
    dkey = dict(zip((det.records["ray"] * 4 + det.records["depth"]).tolist(), det.records["w"].tolist()))
    sel = smp.records["depth"] == 1
    rays = smp.records["ray"][sel]
    assert rays.size > 1000
    kz = np.array([oracle_lib.lattice(n, N)[2] for n in rays])
    rs, rp, ts, tp = cf.slab_characteristic(cf.eta(*sg.GLASS, FREQ), np.abs(kz), 0.01, LAM)
    ar = np.abs(rs) ** 2 + np.abs(rp) ** 2
    qr = ar / (ar + np.abs(ts) ** 2 + np.abs(tp) ** 2)
    wd = np.array([dkey[k] for k in (rays * 4 + 1).tolist()])
    np.testing.assert_allclose(smp.records["w"][sel] * qr, wd, rtol=1e-11)
    # every ray aimed at the ground plane inside the quad and crossing z = 1.5
    # again after reflecting: its reflection is a Bernoulli(q(R)) draw
    cand = np.unique(det.records["ray"][det.records["depth"] == 1])
    kz = np.array([oracle_lib.lattice(n, N)[2] for n in cand])
    rs, rp, ts, tp = cf.slab_characteristic(cf.eta(*sg.GLASS, FREQ), np.abs(kz), 0.01, LAM)
    ar = np.abs(rs) ** 2 + np.abs(rp) ** 2
    q = ar / (ar + np.abs(ts) ** 2 + np.abs(tp) ** 2)
    got = np.unique(rays).size
    assert 0.05 < q.mean() < 0.95
    assert abs(got - q.sum()) <= 5 * math.sqrt(np.sum(q * (1 - q))), (got, q.sum())
    # each decision is the ray's own draw at counter (n, 0, 1) against q(R)
    u = np.array([oracle_lib.uniform(11, n, 0, 1) for n in cand])
    refl = np.isin(cand, rays)
    clear = np.abs(u - q) > 1e-9
    assert np.array_equal(refl[clear], (u < q)[clear])


def test_transparent_wall_keeps_the_field(oracle_lib):
    """A zero-thickness glass wall in front of a concrete ground: every ray
    that meets the wall passes with t = 1 and keeps its TE/TM basis, so the
    ground reflections behind it see the incident field unchanged and the map
    equals the ground-only map (a transmitted field put in the reflected
    basis would change the ground's TE/TM split).  The 50 m concrete slab
    reflects exactly like the half-space (its x underflows to 0)."""
    mb = sg._MeshBuilder()
    mb.quad((-100.0, -100.0, 0.0), (100.0, -100.0, 0.0), (100.0, 100.0, 0.0), (-100.0, 100.0, 0.0), 0)
    mb.quad((15.0, -50.0, 0.0), (15.0, 50.0, 0.0), (15.0, 50.0, 40.0), (15.0, -50.0, 40.0), 1)
    wall = sg.with_thickness(mb.build([sg.CONCRETE, sg.GLASS], "wall"), [50.0, 0.0])
    tx = sg.Tx((0.0, 3.0, 10.0))
    pl = sg.Plane(1.5, -20.0, -40.0, 2.0, 2.0, 40, 40)
    N = 200_000
    a = oracle_lib.radio_map(sg.ground_quad(100.0), tx, pl, sg.Params(FREQ, N, 1))
    b = oracle_lib.radio_map(wall, tx, pl, sg.Params(FREQ, N, 3, refraction=1, seed=2), want_hits=True)
    through = (b.hits[:, :2] >= 2).any(1)                 # triangles 2, 3 are the wall
    assert through.sum() > 10_000
    np.testing.assert_allclose(b.map, a.map, rtol=1e-12, atol=0)


def _dlog_gain_dsigma(coef, eps, sig, cos_t, d, h=1e-6):
    """d ln|c|^2 / d sigma of a characteristic-matrix coefficient by central
    differences (c = 0 r_s, 2 t_s)."""
    up = cf.slab_characteristic(cf.eta(eps, sig + h, FREQ), cos_t, d, LAM)[coef]
    dn = cf.slab_characteristic(cf.eta(eps, sig - h, FREQ), cos_t, d, LAM)[coef]
    c0 = cf.slab_characteristic(cf.eta(eps, sig, FREQ), cos_t, d, LAM)[coef]
    return (np.abs(up) ** 2 - np.abs(dn) ** 2) / (2 * h * np.abs(c0) ** 2)


@pytest.mark.parametrize("case", ["reflect", "transmit"])
def test_detached_slab_gradient(oracle_lib, case):
    """H-pol over a horizontal glass slab is pure TE: a crossing after one
    interaction weighs w = kappa |c_perp|^2 / (q |k_z|), so with the sampling
    probability held constant dw/d sigma = w d ln|c_perp|^2 / d sigma.  The
    oracle's forward-mode gradient of the map sum must equal the sum of
    these over the crossings, with the derivative taken from the layer
    matrix by central differences (reflect: a glass ground seen from above;
    transmit: a pane between the source and the plane)."""
    tx = sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_H)
    N = 200_000
    if case == "reflect":
        sc = sg.with_thickness(sg.ground_quad(100.0, sg.GLASS))
        pl = sg.Plane(1.5, -40.0, -40.0, 2.0, 2.0, 40, 40)
    else:
        mb = sg._MeshBuilder()
        mb.quad((-40.0, -40.0, 5.0), (40.0, -40.0, 5.0), (40.0, 40.0, 5.0), (-40.0, 40.0, 5.0), 0)
        sc = sg.with_thickness(mb.build([sg.GLASS], "pane"))
        pl = sg.Plane(1.5, -20.0, -20.0, 2.0, 2.0, 20, 20)
    G = np.ones((1, pl.H, pl.W))
    r = oracle_lib.radio_map(sc, tx, pl, sg.Params(FREQ, N, 1, refraction=1, seed=3), want_records=True,
                             grad_map=G)
    sel = r.records["depth"] == 1
    rays = r.records["ray"][sel]
    assert rays.size > 1000
    kz = np.abs(np.array([oracle_lib.lattice(n, N)[2] for n in rays]))
    dl = _dlog_gain_dsigma(0 if case == "reflect" else 2, *sg.GLASS, kz, 0.01)
    expect = np.sum(r.records["w"][sel] * dl)
    assert r.grad[1] == pytest.approx(expect, rel=2e-5), (r.grad[1], expect)
