"""Batched radio maps (rt_radio_map_batched) against per-call results.

* several transmitters with uneven ray budgets in one persistent launch equal
  the per-transmitter rt_radio_map maps (FP32 atomic order aside), so every
  ray of every transmitter was traced exactly once;
* several material samples (one traversal) equal per-sample rt_radio_map;
* forward + backward for material samples equals per-sample rt_radio_map +
  rt_radio_map_backward, for sample counts that split unevenly over the
  wavefronts of a 64-ray group, and repeats bit for bit;
* the captured HIP graph replays: every replay, with eager work in between,
  equals the first (eager) result.
"""
import math

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _setup(n_tx=6, seed=5, lo=2e4, hi=3e5, S=1):
    import torch
    import paper_2504_21719_amd as rt
    scene = sg.manhattan_scene()
    txs, budgets = sg.rooftop_transmitters(n_tx, seed=seed, buildings=sg.manhattan_buildings(scene),
                                           budget_lo=lo, budget_hi=hi)
    budgets[0] = 12_347          # a ragged small budget
    plane = sg.Plane(1.5, -500.0, -500.0, 4.0, 4.0, 250, 250)
    params = sg.Params(3.5e9, 1, 5)
    s = rt.scene_from_mesh(scene)
    return rt, torch, scene, s, txs, budgets, plane, params


def _plain(rt, torch, s, eps, sig, tx, budget, plane, params):
    out = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
    p = sg.Params(params.freq_hz, int(budget), params.max_depth)
    rt.rt_radio_map(s, eps, sig, tx, plane, p, out)
    return out


def test_multi_transmitter_matches_plain_loop():
    rt, torch, scene, s, txs, budgets, plane, params = _setup()
    eps = torch.tensor(scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(scene.sigma, dtype=torch.float32, device="cuda")
    T = len(txs)
    out = torch.full((T, 1, plane.H, plane.W), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out)
    torch.cuda.synchronize()
    first = out.clone()
    for t in range(T):
        ref = _plain(rt, torch, s, eps, sig, txs[t], budgets[t], plane, params)
        torch.cuda.synchronize()
        a, b = out[t, 0].cpu().numpy(), ref[0].cpu().numpy()
        assert np.isfinite(a).all()
        big = b > 1e-9 * b.max()
        np.testing.assert_allclose(a[big], b[big], rtol=2e-5)
        assert np.all(a[~big] <= 2e-9 * b.max())
    # graph replays, with eager work between them
    for rep in range(3):
        _plain(rt, torch, s, eps, sig, txs[0], 5000, plane, params)
        out.fill_(float("nan"))
        rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.cpu().numpy(), first.cpu().numpy(), rtol=2e-5, atol=1e-30)


def test_tiny_budgets_at_wavefront_boundaries():
    """Budgets of 1 (the one-ray lattice), 2, 63, 64, 65 and 129 rays, so that
    transmitters start and end inside and on the edges of 64-ray groups: every
    transmitter's batched map equals its own call, forward only and with
    gradients of two material samples."""
    rt, torch, scene, s, txs, _, plane, params = _setup(n_tx=6)
    budgets = [1, 2, 63, 64, 65, 129]
    eps = torch.tensor(scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(scene.sigma, dtype=torch.float32, device="cuda")
    T = len(txs)
    out = torch.full((T, 1, plane.H, plane.W), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out)
    torch.cuda.synchronize()
    for t in range(T):
        ref = _plain(rt, torch, s, eps, sig, txs[t], budgets[t], plane, params)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out[t, 0].cpu().numpy(), ref[0].cpu().numpy(), rtol=2e-5, atol=1e-30)
    S = 2
    E, Sg = sg.random_materials(scene, S, seed=10)
    eS = torch.tensor(E, dtype=torch.float32, device="cuda")
    sS = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    g = torch.ones((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    outs = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    nm = scene.n_materials
    grads = torch.empty((T, S, 2 * nm + 3), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eS, sS, txs, budgets, plane, params, outs, grad_maps=g, grads=grads)
    torch.cuda.synchronize()
    for t in range(T):
        p = sg.Params(params.freq_hz, budgets[t], params.max_depth)
        for k in range(S):
            m = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
            tape = rt.rt_tape_create(p)
            e_k, s_k = eS[k].contiguous(), sS[k].contiguous()
            rt.rt_radio_map(s, e_k, s_k, txs[t], plane, p, m, tape=tape)
            ge, gs, go = (torch.empty(n, device="cuda") for n in (nm, nm, 3))
            rt.rt_radio_map_backward(s, e_k, s_k, txs[t], plane, p, tape, g[t, k].contiguous()[None], ge, gs, go)
            torch.cuda.synchronize()
            np.testing.assert_allclose(outs[t, k].cpu().numpy(), m[0].cpu().numpy(), rtol=2e-5, atol=1e-30)
            ref = torch.cat([ge, gs, go]).cpu().numpy().astype(np.float64)
            got = grads[t, k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).max() + 1e-30), (t, k)


def test_material_samples_match_plain_calls():
    rt, torch, scene, s, txs, budgets, plane, params = _setup(n_tx=3)
    S = 4
    E, Sg = sg.random_materials(scene, S, seed=5)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    T = len(txs)
    out = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, out)
    torch.cuda.synchronize()
    for t in range(T):
        for k in range(S):
            ref = _plain(rt, torch, s, eps[k].contiguous(), sig[k].contiguous(), txs[t], budgets[t], plane, params)
            torch.cuda.synchronize()
            a, b = out[t, k].cpu().numpy(), ref[0].cpu().numpy()
            big = b > 1e-9 * b.max()
            np.testing.assert_allclose(a[big], b[big], rtol=2e-5)


def test_material_samples_fwd_bwd_match_plain_adjoint():
    rt, torch, scene, s, txs, budgets, plane, params = _setup(n_tx=2)
    txs = [sg.Tx(t.pos, yaw=0.4 + 0.3 * i, pitch=-0.15, pattern=sg.PATTERN_DIRECTIONAL) for i, t in enumerate(txs)]
    S = 3
    E, Sg = sg.random_materials(scene, S, seed=6)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    T = len(txs)
    g = torch.randn((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    # smooth upstream gradient (a blurred random field)
    g = torch.nn.functional.avg_pool2d(g.view(T * S, 1, plane.H, plane.W), 9, 1, 4).view_as(g).contiguous()
    out = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    nm = scene.n_materials
    grads = torch.empty((T, S, 2 * nm + 3), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, out, grad_maps=g, grads=grads)
    torch.cuda.synchronize()
    for t in range(T):
        p = sg.Params(params.freq_hz, int(budgets[t]), params.max_depth)
        for k in range(S):
            m = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
            tape = rt.rt_tape_create(p)
            e_k, s_k = eps[k].contiguous(), sig[k].contiguous()
            rt.rt_radio_map(s, e_k, s_k, txs[t], plane, p, m, tape=tape)
            ge = torch.empty(nm, device="cuda")
            gs = torch.empty(nm, device="cuda")
            go = torch.empty(3, device="cuda")
            rt.rt_radio_map_backward(s, e_k, s_k, txs[t], plane, p, tape, g[t, k].contiguous()[None], ge, gs, go)
            torch.cuda.synchronize()
            ref = torch.cat([ge, gs, go]).cpu().numpy().astype(np.float64)
            got = grads[t, k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).max()), (t, k, got, ref)
            a, b = out[t, k].cpu().numpy(), m[0].cpu().numpy()
            big = b > 1e-9 * b.max()
            np.testing.assert_allclose(a[big], b[big], rtol=2e-5)


@pytest.mark.parametrize("S,L", [(1, 5), (6, 5), (2, 7)])
def test_material_samples_uneven_wavefront_share_and_determinism(S, L):
    """The sample kernel gives each group of 64 rays to min(4, S) wavefronts
    that take every fourth sample: S = 1 runs one wavefront per group, S = 6
    two wavefronts with two samples and two with one.  Maps and gradients of
    the first and last sample equal per-sample forward + adjoint calls, and a
    second call reproduces every gradient bit for bit (partial sums in a
    fixed order).  Paths of up to six segments take the variant that keeps
    the forward fields in LDS, longer ones (L = 7) the one that keeps them in
    registers."""
    rt, torch, scene, s, txs, budgets, plane, params = _setup(n_tx=2)
    params = sg.Params(params.freq_hz, 1, L)
    txs = [sg.Tx(t.pos, yaw=0.2 + 0.5 * i, pitch=-0.1, pattern=sg.PATTERN_DIRECTIONAL) for i, t in enumerate(txs)]
    E, Sg = sg.random_materials(scene, S, seed=8)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    T = len(txs)
    g = torch.randn((T, S, plane.H, plane.W), generator=torch.Generator().manual_seed(9)).to("cuda")
    g = torch.nn.functional.avg_pool2d(g.view(T * S, 1, plane.H, plane.W), 9, 1, 4).view_as(g).contiguous()
    out = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    nm = scene.n_materials
    grads = torch.empty((T, S, 2 * nm + 3), dtype=torch.float32, device="cuda")
    grads2 = torch.empty_like(grads)
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, out, grad_maps=g, grads=grads)
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, torch.empty_like(out), grad_maps=g,
                            grads=grads2)
    torch.cuda.synchronize()
    assert torch.equal(grads, grads2)
    for t in range(T):
        p = sg.Params(params.freq_hz, int(budgets[t]), params.max_depth)
        for k in sorted({0, S - 1}):
            m = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
            tape = rt.rt_tape_create(p)
            e_k, s_k = eps[k].contiguous(), sig[k].contiguous()
            rt.rt_radio_map(s, e_k, s_k, txs[t], plane, p, m, tape=tape)
            ge, gs, go = (torch.empty(n, device="cuda") for n in (nm, nm, 3))
            rt.rt_radio_map_backward(s, e_k, s_k, txs[t], plane, p, tape, g[t, k].contiguous()[None], ge, gs, go)
            torch.cuda.synchronize()
            ref = torch.cat([ge, gs, go]).cpu().numpy().astype(np.float64)
            got = grads[t, k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).max()), (t, k, got, ref)
            a, b = out[t, k].cpu().numpy(), m[0].cpu().numpy()
            big = b > 1e-9 * b.max()
            np.testing.assert_allclose(a[big], b[big], rtol=2e-5)


def test_material_samples_with_slab_walls_and_arrays():
    """Slab walls without refraction and transmit arrays leave every path
    unchanged, so material samples share one traversal with them too: maps
    and gradients of three samples for two transmitters (one with an array)
    equal per-sample rt_radio_map + rt_radio_map_backward with the same
    thickness."""
    import dataclasses
    rt, torch, scene, s, txs, budgets, plane, params = _setup(n_tx=2)
    scene = sg.with_thickness(sg.manhattan_scene(bottoms=False))
    s = rt.scene_from_mesh(scene)
    txs = [sg.Tx(t.pos, yaw=0.4 + 0.3 * i, pitch=-0.15, pattern=sg.PATTERN_DIRECTIONAL,
                 array=sg.random_array(5, 0.12, seed=31) if i == 1 else None) for i, t in enumerate(txs)]
    thk = torch.tensor(scene.thickness, dtype=torch.float32, device="cuda")
    S = 3
    E, Sg = sg.random_materials(scene, S, seed=7)
    eps = torch.tensor(E, dtype=torch.float32, device="cuda")
    sig = torch.tensor(Sg, dtype=torch.float32, device="cuda")
    T = len(txs)
    g = torch.randn((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    g = torch.nn.functional.avg_pool2d(g.view(T * S, 1, plane.H, plane.W), 9, 1, 4).view_as(g).contiguous()
    out = torch.empty((T, S, plane.H, plane.W), dtype=torch.float32, device="cuda")
    fwd_only = torch.empty_like(out)
    nm = scene.n_materials
    grads = torch.empty((T, S, 2 * nm + 3), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, out, grad_maps=g, grads=grads, thickness=thk)
    rt.rt_radio_map_batched(s, eps, sig, txs, budgets, plane, params, fwd_only, thickness=thk)
    torch.cuda.synchronize()
    for t in range(T):
        p = dataclasses.replace(params, n_rays=int(budgets[t]))
        for k in range(S):
            m = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
            tape = rt.rt_tape_create(p)
            e_k, s_k = eps[k].contiguous(), sig[k].contiguous()
            rt.rt_radio_map(s, e_k, s_k, txs[t], plane, p, m, tape=tape, thickness=thk)
            ge = torch.empty(nm, device="cuda")
            gs = torch.empty(nm, device="cuda")
            go = torch.empty(3, device="cuda")
            rt.rt_radio_map_backward(s, e_k, s_k, txs[t], plane, p, tape, g[t, k].contiguous()[None], ge, gs, go,
                                     thickness=thk)
            torch.cuda.synchronize()
            ref = torch.cat([ge, gs, go]).cpu().numpy().astype(np.float64)
            got = grads[t, k].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-6 * np.abs(ref).max()), (t, k, got, ref)
            b = m[0].cpu().numpy()
            big = b > 1e-9 * b.max()
            for a in (out[t, k].cpu().numpy(), fwd_only[t, k].cpu().numpy()):
                np.testing.assert_allclose(a[big], b[big], rtol=2e-5)


@pytest.mark.parametrize("case", ["arrays", "slab_refraction_roulette", "diffuse_threshold"])
def test_multi_transmitter_extensions_match_single_calls(case):
    """One material set, no gradients: transmit arrays (two of six
    transmitters), slab walls with refraction and Russian roulette, or
    diffuse reflection (directive pattern) with gain thresholding, batched
    over uneven budgets.  Every transmitter's map equals its rt_radio_map map:
    each ray draws from the streams of its own lattice index, as in a single
    call.  The two kernels may round a multiply-add differently, so a
    decision that falls exactly on its threshold may go the other way: a few
    cells may differ; the totals agree within 1e-4."""
    import dataclasses
    rt, torch, scene, s, txs, budgets, plane, params = _setup()
    kw = {}
    if case == "arrays":
        txs = [dataclasses.replace(t, array=sg.random_array(6, 0.15, seed=20 + i)) if i in (1, 3) else t
               for i, t in enumerate(txs)]
    elif case == "slab_refraction_roulette":
        scene = sg.with_thickness(sg.manhattan_scene(bottoms=False))
        s = rt.scene_from_mesh(scene)
        params = sg.Params(3.5e9, 1, 5, refraction=1, rr_p_max=0.5, rr_depth=2, seed=7)
        kw["thickness"] = torch.tensor(scene.thickness, dtype=torch.float32, device="cuda")
    else:
        scene = sg.with_diffuse(scene, [0.4, 0.2], [0.1, 0.3], (1, 3, 1, 1.0))
        params = sg.Params(3.5e9, 1, 5, gain_threshold=1e-13, seed=11)
        for name, v in (("scattering", scene.scattering), ("xpd", scene.xpd),
                        ("scatter_pattern", scene.scatter_pattern)):
            kw[name] = torch.tensor(v, dtype=torch.float32, device="cuda")
    eps = torch.tensor(scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(scene.sigma, dtype=torch.float32, device="cuda")
    T = len(txs)
    out = torch.full((T, 1, plane.H, plane.W), float("nan"), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out, **kw)
    torch.cuda.synchronize()
    for t in range(T):
        ref = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
        p = dataclasses.replace(params, n_rays=int(budgets[t]))
        rt.rt_radio_map(s, eps, sig, txs[t], plane, p, ref, **kw)
        torch.cuda.synchronize()
        a, b = out[t, 0].cpu().numpy().astype(np.float64), ref[0].cpu().numpy().astype(np.float64)
        assert np.isfinite(a).all() and b.max() > 0
        off = ~np.isclose(a, b, rtol=1e-4, atol=1e-7 * b.max())
        assert off.sum() <= 20, (t, int(off.sum()))
        assert a.sum() == pytest.approx(b.sum(), rel=1e-4)


@pytest.mark.parametrize("deposit", [1, 2])
def test_multi_transmitter_deposits_stay_in_their_maps(deposit):
    """A wavefront can hold rays of several transmitters, so its same-cell
    sums must group lanes by transmitter as well as by cell.  256 iso
    transmitters at the street intersection (0, 0, 30) with lattices of 2 or 4 rays
    (per-ray weights differ twofold): one claim of work spans about twenty
    transmitters, whose downward rays cross the 250 m cell below them in the
    same iteration.  Every transmitter's batched map equals its single-call
    map, with per-lane atomics and with wavefront sums."""
    rt, torch, scene, s, txs, budgets, plane, params = _setup(n_tx=1)
    pos = (0.0, 0.0, 30.0)
    T = 256
    txs = [sg.Tx(pos) for _ in range(T)]
    budgets = [2 if i % 2 == 0 else 4 for i in range(T)]
    plane = sg.Plane(1.5, pos[0] - 500.0, pos[1] - 500.0, 250.0, 250.0, 4, 4)
    eps = torch.tensor(scene.eps_r, dtype=torch.float32, device="cuda")
    sig = torch.tensor(scene.sigma, dtype=torch.float32, device="cuda")
    out = torch.empty((T, 1, plane.H, plane.W), dtype=torch.float32, device="cuda")
    rt.rt_radio_map_batched(s, eps[None], sig[None], txs, budgets, plane, params, out, deposit=deposit)
    torch.cuda.synchronize()
    got = out[:, 0].cpu().numpy()
    assert (got > 0).any()
    for t in range(T):
        ref = torch.empty((1, plane.H, plane.W), dtype=torch.float32, device="cuda")
        p = sg.Params(params.freq_hz, int(budgets[t]), params.max_depth)
        rt.rt_radio_map(s, eps, sig, txs[t], plane, p, ref, deposit=deposit)
        torch.cuda.synchronize()
        b = ref[0].cpu().numpy()
        np.testing.assert_allclose(got[t], b, rtol=2e-5, atol=1e-7 * max(b.max(), 1e-30),
                                   err_msg="transmitter %d" % t)
