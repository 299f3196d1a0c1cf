"""Diffuse reflection (App. "Diffuse Reflection", Lambertian pattern
eq. lambertian_model, cross-polarisation eq. scattered_field; interaction
shares of eq. path-solver-used-dist-event with R = sqrt(1 - S^2)) on the GPU
against the FP64 oracle, both drawing the interaction type from Philox
counter (n, l, 1) and the diffuse direction and phases from (n, l, 2).

Per-crossing weights: |w_g - w_o| <= 5e-5 w_o, the slab-wall bound; a
diffuse bounce itself adds FP32 rounding of Gamma^2, of the frame and of
the phases (a few 1e-7), because its polar cosine is the draw itself on
both sides.
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


def _tiny(S=0.5, K=0.2, seed=13, pol=sg.POL_V):
    cfg = sg.tiny_config(n_rays=100_000)
    cfg.scene = sg.with_diffuse(cfg.scene, S, K)
    cfg.params.seed = seed
    cfg.tx = sg.Tx((0.0, 0.0, 10.0), pol=pol)
    return cfg


def test_diffuse_tiny():
    cfg = _tiny()
    g, _ = _parity(cfg)
    spec = gpu_radio_map(sg.tiny_config(n_rays=100_000))
    assert (g.cells != spec.cells).any(1).mean() > 0.05      # diffuse bounces did happen


def test_diffuse_tiny_hpol_full_cross_polarisation():
    _parity(_tiny(S=1.0, K=1.0, seed=4, pol=sg.POL_H))


def test_diffuse_manhattan():
    cfg = sg.manhattan_config(n_rays=200_000, max_depth=5)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    cfg.scene = sg.with_diffuse(cfg.scene, [0.4, 0.2], [0.1, 0.3])
    cfg.params.seed = 99
    _parity(cfg)


@pytest.mark.parametrize("pp", [(1, 3, 1, 1.0), (2, 2, 4, 0.5)])
def test_diffuse_directive_and_backscattering_patterns(pp):
    cfg = sg.manhattan_config(n_rays=200_000, max_depth=5)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    cfg.scene = sg.with_diffuse(cfg.scene, [0.5, 0.3], [0.2, 0.0], pp)
    cfg.params.seed = 5
    _parity(cfg)


def test_diffuse_with_refraction_and_roulette():
    cfg = sg.tiny_config(n_rays=100_000)
    cfg.scene = sg.with_diffuse(sg.with_thickness(sg.tiny_scene(bottom=False), [0.05]), 0.5, 0.2)
    cfg.params.refraction, cfg.params.seed = 1, 17
    cfg.params.rr_p_max, cfg.params.rr_depth = 0.7, 2
    _parity(cfg)


def test_diffuse_brute_force_matches_bvh():
    cfg = _tiny(seed=8)
    s = gpu_scene(cfg.scene)
    a = gpu_radio_map(cfg, scene_handle=s)
    b = gpu_radio_map(cfg, scene_handle=s, accel=1)
    assert np.array_equal(a.hits, b.hits) and np.array_equal(a.cells, b.cells)
    # the two kernels contract multiply-adds independently: ulp-level
    # differences, amplified at most 20x by the slab formula
    np.testing.assert_allclose(b.weights, a.weights, rtol=5e-6, atol=0)


def test_diffuse_rejections():
    import torch
    import paper_2504_21719_amd as rt
    cfg = _tiny()
    s = gpu_scene(cfg.scene)
    dev = "cuda"
    eps = torch.tensor(cfg.scene.eps_r, dtype=torch.float32, device=dev)
    sig = torch.tensor(cfg.scene.sigma, dtype=torch.float32, device=dev)
    sca = torch.tensor(cfg.scene.scattering, dtype=torch.float32, device=dev)
    xpd = torch.tensor(cfg.scene.xpd, dtype=torch.float32, device=dev)
    out = torch.empty((2, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device=dev)
    with pytest.raises(rt.RtError) as e:
        rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, out[:1], scattering=sca)
    assert e.value.status == rt.RT_EINVAL                     # xpd missing
    with pytest.raises(rt.RtError) as e:
        rt.rt_radio_map(s, eps, sig, sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_DUAL), cfg.plane, cfg.params, out,
                        scattering=sca, xpd=xpd)
    assert e.value.status == rt.RT_EUNSUPPORTED
    # a taped call records the same map (deposit order aside)
    tape = rt.rt_tape_create(cfg.params)
    ref = torch.empty_like(out[:1])
    rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, out[:1], tape=tape, scattering=sca, xpd=xpd)
    rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, ref, scattering=sca, xpd=xpd)
    torch.cuda.synchronize()
    torch.testing.assert_close(out[:1], ref, rtol=1e-4, atol=0)
