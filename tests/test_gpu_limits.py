"""The largest values the C ABI accepts, on the GPU.

* max_depth = 64 (the limit of rt_sbr_params): rays bouncing between two
  near-perfect metal walls over a concrete ground, every segment's hit, cell
  and weight against the oracle (per-cell protocol over every ray);
* 4096 transmitters (the limit of rt_radio_map_batched) with ragged small
  budgets in one batched call: every transmitter's map equals its own
  rt_radio_map call;
* 64 material samples (the limit) forward + backward in one batched call:
  every sample's map equals its own rt_radio_map, and the gradients of a
  spread of samples equal rt_radio_map_backward on a tape.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_helpers import assert_parity, compare_maps, gpu_radio_map

pytestmark = pytest.mark.gpu


def _mirror_corridor():
    """Two metal walls at x = +-5 m (y in [-200, 200], z in [0, 30]) over a
    concrete ground strip: horizontal rays bounce between the walls dozens of
    times before they leave along y or reach the ground."""
    V, F, M = [], [], []

    def quad(a, b, c, d, m):
        base = len(V)
        V.extend([a, b, c, d])
        F.extend([[base, base + 1, base + 2], [base, base + 2, base + 3]])
        M.extend([m, m])

    quad((-5, -200, 0), (-5, 200, 0), (-5, 200, 30), (-5, -200, 30), 1)
    quad((5, -200, 0), (5, -200, 30), (5, 200, 30), (5, 200, 0), 1)
    quad((-5, -200, 0), (5, -200, 0), (5, 200, 0), (-5, 200, 0), 0)
    return sg.Scene(np.array(V, np.float32), np.array(F, np.int32), np.array(M, np.int32),
                    np.array([5.24, 1.0]), np.array([0.12, 1e7]), name="mirror-corridor")


def test_maximum_depth_between_metal_walls():
    print("max depth: mirror corridor, 200,003 rays, L = 64", flush=True)
    scene = _mirror_corridor()
    cfg = sg.Config(scene, sg.Tx((0.3, 0.7, 10.0)), sg.Plane(1.5, -5.0, -200.0, 1.0, 1.0, 10, 400),
                    sg.Params(3.5e9, 200_003, 64))
    g = gpu_radio_map(cfg)
    assert int(g.stats[4]) == 0
    traced = (g.hits != -2).sum(1)
    assert traced.max() == 65, traced.max()          # some rays use every segment
    assert (traced >= 30).sum() > 5000 and (traced == 65).sum() > 1000
    o = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, want_records=True)
    d = compare_maps(cfg, g, o, 0, min_count=50)
    print("mirror corridor", d)
    assert d["n_cells"] >= 500
    # every reflection multiplies the FP32 field by a Fresnel and basis
    # product carrying about ten roundings (complex square root, two
    # divisions): ~1.5e-6 relative per bounce, ~1e-4 after 64 of them
    assert_parity(d, max_w_rel=1e-4)


def test_maximum_transmitter_count():
    import torch
    import paper_2504_21719_amd as rt
    print("4096 transmitters, ragged budgets", flush=True)
    cfg = sg.tiny_config()
    rng = np.random.default_rng(11)
    T = 4096
    pos = np.stack([rng.uniform(-60, 60, T), rng.uniform(-60, 60, T), rng.uniform(2, 40, T)], 1)
    txs = [sg.Tx(tuple(p)) for p in pos]
    budgets = [int(b) for b in rng.integers(1, 400, T)]
    plane = sg.Plane(1.5, -100.0, -100.0, 10.0, 10.0, 20, 20)
    params = sg.Params(3.5e9, 1, 2)
    s = rt.scene_from_mesh(cfg.scene)
    eps = torch.tensor(cfg.scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(cfg.scene.sigma, dtype=torch.float32, device="cuda")
    out = torch.full((T, 1, plane.H, plane.W), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out)
    ref = torch.empty_like(out)
    for t in range(T):
        rt.rt_radio_map(s, eps, sig, txs[t], plane, sg.Params(3.5e9, budgets[t], 2), ref[t])
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.isfinite(a).all()
    np.testing.assert_allclose(a, b, rtol=2e-5, atol=1e-7 * float(b.max()))


def test_maximum_sample_count_with_gradients():
    import torch
    import paper_2504_21719_amd as rt
    print("64 material samples forward + backward", flush=True)
    scene = sg.manhattan_scene()
    S = 64
    E, Sg = sg.random_materials(scene, S, seed=12)
    tx = sg.Tx((10.0, -20.0, 30.0), yaw=0.5, pitch=-0.2, pattern=sg.PATTERN_DIRECTIONAL)
    plane = sg.Plane(1.5, -500.0, -500.0, 5.0, 5.0, 200, 200)
    n_rays = 60_001
    s = rt.scene_from_mesh(scene)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    g = torch.randn((1, S, plane.H, plane.W), generator=torch.Generator().manual_seed(13)).to("cuda")
    g = torch.nn.functional.avg_pool2d(g.view(S, 1, plane.H, plane.W), 9, 1, 4).view_as(g).contiguous()
    out = torch.empty((1, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    nm = scene.n_materials
    grads = torch.empty((1, S, 2 * nm + 3), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps, sig, [tx], [n_rays], plane, sg.Params(3.5e9, 1, 4), out, grad_maps=g,
                            grads=grads)
    torch.cuda.synchronize()
    p = sg.Params(3.5e9, n_rays, 4)
    tape = rt.rt_tape_create(p)
    for k in range(S):
        m = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
        e_k, s_k = eps[k].contiguous(), sig[k].contiguous()
        rt.rt_radio_map(s, e_k, s_k, tx, plane, p, m, tape=tape)
        a, b = out[0, k].cpu().numpy(), m[0].cpu().numpy()
        big = b > 1e-9 * b.max()
        np.testing.assert_allclose(a[big], b[big], rtol=2e-5)
        if k % 9 == 0 or k == S - 1:
            ge, gs, go = (torch.empty(n, device="cuda") for n in (nm, nm, 3))
            rt.rt_radio_map_backward(s, e_k, s_k, tx, plane, p, tape, g[0, k].contiguous()[None], ge, gs, go)
            torch.cuda.synchronize()
            ref = torch.cat([ge, gs, go]).cpu().numpy().astype(np.float64)
            got = grads[0, k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).max()), (k, got, ref)
