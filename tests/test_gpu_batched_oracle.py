"""Batched radio maps (rt_radio_map_batched) against the FP64 oracle.

"Radio maps for multiple sources in parallel" (Sec. "Radio Map Solver"):
* several transmitters with uneven ray budgets in one persistent
  launch: each transmitter's batched map against the oracle's map for that
  transmitter alone, under the per-cell protocol (cells with >= 100
  crossings within 1e-3 plus the border allowance).  The batched call has no
  per-ray records, so the rays whose hits differ from the oracle's are found
  from a single-transmitter call with records, and the oracle is replayed
  along those hits (replay-corrected map);
* several material samples with gradients in one launch: each (transmitter,
  sample) map against the oracle at that sample's materials, and each
  vector-Jacobian product against the oracle's forward-mode gradient of
  sum(G * map) (within 1e-3 per component, plus 1e-5 of the largest).
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_helpers import GpuResult, assert_parity, compare_maps, gpu_radio_map

pytestmark = pytest.mark.gpu


def _smooth_field(H, W, seed, n_modes=6, min_wavelength=20.0):
    rng = np.random.default_rng(seed)
    j, i = np.mgrid[0:H, 0:W].astype(np.float64)
    G = np.zeros((H, W))
    for _ in range(n_modes):
        kx, ky = rng.uniform(-1, 1, 2) * 2 * np.pi / min_wavelength
        G += rng.standard_normal() * np.cos(kx * i + ky * j + rng.uniform(0, 2 * np.pi))
    return G


# Street-intersection transmitters at several heights.  A rooftop source
# sends few rays to the ground near it (its own roof shadows the steep ones),
# so at test-sized budgets no 5 m cell would reach 100 crossings; from a
# street the smallest budget below still gives a few dozen such cells.
STREET_TX = ((-100.0, 200.0, 25.0), (0.0, 0.0, 30.0), (300.0, -100.0, 18.0))


def _setup(n_tx, budgets, directional=False):
    scene = sg.manhattan_scene()
    txs = [sg.Tx(p) for p in STREET_TX[:n_tx]]
    if directional:
        txs = [sg.Tx(t.pos, yaw=0.4 * (i + 1), pitch=-0.15 * (i + 1), roll=0.05, pattern=sg.PATTERN_DIRECTIONAL)
               for i, t in enumerate(txs)]
    plane = sg.Plane(1.5, -500.0, -500.0, 5.0, 5.0, 200, 200)
    return scene, txs, np.asarray(budgets, np.int64), plane


def test_batched_transmitters_match_oracle():
    """Three street-level transmitters with budgets 23,457 / 150,001 / 400,000
    (a ragged small one first in the caller's order; the library orders them
    largest first), L = 5, 5 m cells."""
    import torch
    import paper_2504_21719_amd as rt
    scene, txs, budgets, plane = _setup(3, [23_457, 150_001, 400_000])
    s = rt.scene_from_mesh(scene)
    eps = torch.tensor(scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(scene.sigma, dtype=torch.float32, device="cuda")
    T = len(txs)
    out = torch.full((T, 1, plane.H, plane.W), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, sg.Params(3.5e9, 1, 5), out)
    torch.cuda.synchronize()
    maps = out.cpu().numpy()
    assert np.isfinite(maps).all()
    for t in range(T):
        cfg = sg.Config(scene, txs[t], plane, sg.Params(3.5e9, int(budgets[t]), 5))
        single = gpu_radio_map(cfg, scene_handle=s, records=True)
        o = oracle.radio_map(scene, txs[t], plane, cfg.params, want_records=True)
        g = GpuResult(maps[t], single.hits, single.cells, single.weights, None)
        d = compare_maps(cfg, g, o, 0)
        print("tx", t, int(budgets[t]), d)
        assert d["n_cells"] >= 20, d
        assert_parity(d)


def test_batched_material_samples_and_gradients_match_oracle():
    """Two directional street-level transmitters (budgets 60,001 and 200,000,
    L = 4) and three material samples in one forward + backward launch: every
    (transmitter, sample) map and VJP against the oracle at that sample."""
    import torch
    import paper_2504_21719_amd as rt
    scene, txs, budgets, plane = _setup(2, [60_001, 200_000], directional=True)
    S = 3
    E, Sg = sg.random_materials(scene, S, seed=9)
    s = rt.scene_from_mesh(scene)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    T = len(txs)
    P = 2 * scene.n_materials + 3
    G = np.stack([np.stack([_smooth_field(plane.H, plane.W, seed=100 + 10 * t + k) for k in range(S)])
                  for t in range(T)])
    gm = torch.tensor(G, dtype=torch.float32, device="cuda")
    out = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    grads = torch.full((T, S, P), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, sg.Params(3.5e9, 1, 4), out, grad_maps=gm,
                            grads=grads)
    torch.cuda.synchronize()
    maps, gr = out.cpu().numpy(), grads.cpu().numpy().astype(np.float64)
    for t in range(T):
        cfg = sg.Config(scene, txs[t], plane, sg.Params(3.5e9, int(budgets[t]), 4))
        single = None
        for k in range(S):
            single = gpu_radio_map(cfg, scene_handle=s, records=True, eps_r=E[k], sigma=Sg[k])
            o = oracle.radio_map(scene, txs[t], plane, cfg.params, eps_r=E[k], sigma=Sg[k], want_records=True,
                                 grad_map=G[t, k][None])
            d = compare_maps(cfg, GpuResult(maps[t, k][None], single.hits, single.cells, single.weights, None),
                             o, 0, min_count=50)
            print("tx", t, "sample", k, d)
            assert d["n_cells"] >= 20, d
            assert_parity(d)
            scale = np.max(np.abs(o.grad))
            err = np.abs(gr[t, k] - o.grad)
            print("grad", gr[t, k], o.grad)
            assert np.all(err <= 1e-3 * np.abs(o.grad) + 1e-5 * scale), (t, k, gr[t, k], o.grad)
            # the orientation derivatives of a directional source are not small
            assert np.abs(o.grad[2 * scene.n_materials:2 * scene.n_materials + 2]).max() > 1e-3 * scale
