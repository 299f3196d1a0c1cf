"""Early termination (Sec. "Practical Notes", eq. radio-map-solver-rr-prob) on
the GPU against the FP64 oracle: Russian roulette and gain thresholding with
the same Philox4x32-10 stream on both sides.  A ray whose keep-or-drop
decision lies within 1e-5 of its threshold is flagged by the oracle and exempt
from bit-exact hit parity (the two sides evaluate the gain in FP32 and FP64)."""
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
    assert_parity(d)
    return g, o


def test_roulette_tiny():
    cfg = sg.tiny_config(n_rays=100_000)
    cfg.params.rr_p_max, cfg.params.rr_depth, cfg.params.seed = 0.7, 1, 9
    g, o = _parity(cfg)
    base = gpu_radio_map(sg.tiny_config(n_rays=100_000))
    dropped = (base.hits != -2).sum() - (g.hits != -2).sum()
    assert dropped > 1_000                     # the roulette did end paths


def test_roulette_and_threshold_manhattan():
    cfg = sg.manhattan_config(n_rays=200_000, max_depth=5)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    cfg.params.rr_p_max, cfg.params.rr_depth, cfg.params.seed = 0.5, 2, 1234
    cfg.params.gain_threshold = 1e-11
    _parity(cfg)


def test_termination_after_last_depth_changes_nothing():
    cfg = sg.tiny_config(n_rays=50_000)
    s = gpu_scene(cfg.scene)
    a = gpu_radio_map(cfg, scene_handle=s)
    cfg.params.rr_p_max, cfg.params.rr_depth = 0.3, cfg.params.max_depth + 1
    b = gpu_radio_map(cfg, scene_handle=s)
    assert np.array_equal(a.hits, b.hits) and np.array_equal(a.cells, b.cells)
    # the two kernel variants may contract multiply-adds differently: a few ulp
    np.testing.assert_allclose(b.weights, a.weights, rtol=4e-7, atol=0)


def test_termination_with_tape_and_rejected_batched_samples():
    """A taped call with early termination gives the untaped map; batched
    material samples have no termination and reject it."""
    import torch
    import paper_2504_21719_amd as rt
    cfg = sg.tiny_config(n_rays=10_000)
    cfg.params.rr_p_max, cfg.params.seed = 0.5, 5
    cfg.params.gain_threshold = 1e-9
    s = gpu_scene(cfg.scene)
    eps = torch.tensor(cfg.scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(cfg.scene.sigma, dtype=torch.float32, device="cuda")
    out = torch.empty((1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device="cuda")
    ref = torch.empty_like(out)
    tape = rt.rt_tape_create(cfg.params)
    rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, out, tape=tape)
    rt.rt_radio_map(s, eps, sig, cfg.tx, cfg.plane, cfg.params, ref)
    torch.cuda.synchronize()
    # same rays and weights; only the order of the atomic deposits may differ
    torch.testing.assert_close(out, ref, rtol=1e-4, atol=0)
    # several material samples share one traversal and take no extensions
    maps = torch.empty((1, 2, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as e:
        rt.rt_radio_map_batched(s, torch.stack([eps, eps]), torch.stack([sig, sig]), [cfg.tx], [10_000], cfg.plane,
                                cfg.params, maps)
    assert e.value.status == rt.RT_EUNSUPPORTED
