"""Finite-thickness walls (Sec. "Single-Layer Slab", eq. fresnel_slab) and
refraction with Fresnel-importance interaction sampling (Sec. "Sampling
Interaction Types", eq. path-solver-used-dist-event) on the GPU against the
FP64 oracle, both drawing from the same Philox4x32-10 stream.  A ray whose
reflect-or-transmit draw lies within 1e-5 of q(R) is flagged by the oracle and
exempt from bit-exact hit parity (the two sides evaluate q(R) in FP32 and
FP64).  The scenes leave out the buildings' bottom faces: they coincide with
the ground, and a transmitted ray could meet both at one distance.

Per-crossing weights: |w_g - w_o| <= 5e-5 w_o.  The slab's phase thickness
q = (2 pi d / lambda) s carries the FP32 error of s (about 4 ulp, so
2.4e-7 |q| rad), and a slab reflection changes |r|^2 relative to it by up to
2 |x|^2 / |1 - x^2| times the error of the phase of x^2: for the 10 mm glass
pane (|q| <= 3.7, |x|^2 = 0.85, |1 - x^2| >= 0.15) that is 2e-5 per slab
interaction, two of them on one path 4e-5, plus the 1e-5 of the specular path.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_helpers import assert_parity, compare_maps, gpu_radio_map, gpu_scene

pytestmark = pytest.mark.gpu


def _parity(cfg):
    g = gpu_radio_map(cfg)
    o = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, want_records=True)
    d = compare_maps(cfg, g, o, 0)
    print(d)
    assert_parity(d, max_w_rel=5e-5)
    return g, o


def _tiny(thickness=0.05, refraction=1, seed=21):
    cfg = sg.tiny_config(n_rays=100_000)
    cfg.scene = sg.with_thickness(sg.tiny_scene(bottom=False), [thickness])
    cfg.params.refraction, cfg.params.seed = refraction, seed
    return cfg


def test_slab_reflection_tiny():
    """Slab coefficients without transmission (q(R) = 1)."""
    _parity(_tiny(0.2, refraction=0))


def test_refraction_tiny():
    cfg = _tiny()
    g, _ = _parity(cfg)
    refl = gpu_radio_map(_tiny(refraction=0))
    changed = (g.hits != refl.hits).any(1).mean()
    assert changed > 0.02                      # transmissions did happen


def test_refraction_manhattan():
    cfg = sg.manhattan_config(n_rays=200_000, max_depth=5)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    cfg.scene = sg.with_thickness(sg.manhattan_scene(bottoms=False))   # 20 cm concrete, 10 mm glass
    cfg.params.refraction, cfg.params.seed = 1, 77
    _parity(cfg)


def test_refraction_with_roulette():
    cfg = _tiny(seed=5)
    cfg.params.rr_p_max, cfg.params.rr_depth = 0.6, 1
    _parity(cfg)


def test_refraction_brute_force_matches_bvh():
    """The brute-force and tree kernels share the interaction code: identical
    hits and cells, weights to rounding."""
    cfg = _tiny(seed=3)
    s = gpu_scene(cfg.scene)
    a = gpu_radio_map(cfg, scene_handle=s)
    b = gpu_radio_map(cfg, scene_handle=s, accel=1)
    assert np.array_equal(a.hits, b.hits) and np.array_equal(a.cells, b.cells)
    # the two kernels contract multiply-adds independently: ulp-level
    # differences, amplified at most 20x by the slab formula
    np.testing.assert_allclose(b.weights, a.weights, rtol=5e-6, atol=0)


def test_refraction_rejections():
    import torch
    import paper_2504_21719_amd as rt
    cfg = _tiny()
    s = gpu_scene(cfg.scene)
    eps = torch.tensor(cfg.scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(cfg.scene.sigma, dtype=torch.float32, device="cuda")
    thk = torch.tensor(cfg.scene.thickness, dtype=torch.float32, device="cuda")
    out = torch.empty((1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as e:           # refraction without a thickness
        rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, out)
    assert e.value.status == rt.RT_EINVAL
    tape = rt.rt_tape_create(cfg.params)             # a tape records the sampled branches
    rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, out, tape=tape, thickness=thk)
    g = torch.ones_like(out)
    ge = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as e:             # the backward needs the same thickness
        rt.rt_radio_map_backward(s, eps, sig, cfg.tx, cfg.plane, cfg.params, tape, g, ge)
    assert e.value.status == rt.RT_EINVAL
    # several material samples share one traversal and take no extensions
    maps = torch.empty((1, 2, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as e:
        rt.rt_radio_map_batched(s, torch.stack([eps, eps]), torch.stack([sig, sig]), [cfg.tx], [10_000], cfg.plane,
                                cfg.params, maps)
    assert e.value.status == rt.RT_EUNSUPPORTED


def test_transparent_and_opaque_walls():
    """Degenerate slabs on the GPU: a zero-thickness ground passes every ray
    (the map is the empty scene's), a metal sheet reflects every ray (the map
    is the half-space specular one); one ray and depth 0 also work."""
    tx = sg.Tx((3.0, -2.0, 12.0))
    pl = sg.Plane(1.5, -40.0, -40.0, 2.0, 2.0, 40, 40)
    p = sg.Params(3.5e9, 200_000, 3, refraction=1, seed=3)
    clear = sg.Config(sg.with_thickness(sg.ground_quad(100.0), [0.0]), tx, pl, p)
    empty = sg.Config(sg.empty_scene(), tx, pl, sg.Params(3.5e9, 200_000, 3))
    a, b = gpu_radio_map(clear), gpu_radio_map(empty)
    np.testing.assert_allclose(a.map, b.map, rtol=1e-5, atol=0)
    metal = sg.ground_quad(100.0, sg.METAL)
    c = gpu_radio_map(sg.Config(sg.with_thickness(metal), tx, pl, p))
    d = gpu_radio_map(sg.Config(metal, tx, pl, sg.Params(3.5e9, 200_000, 3)))
    assert np.array_equal(c.hits, d.hits)
    np.testing.assert_allclose(c.map, d.map, rtol=1e-5, atol=0)
    one = _tiny()
    one.params.n_rays, one.params.max_depth = 1, 0
    g = gpu_radio_map(one)
    o = oracle.radio_map(one.scene, one.tx, one.plane, one.params, want_hits=True)
    assert np.array_equal(g.hits, o.hits)
