"""Synthetic transmit arrays with precoding (Sec. "Handling Multiple Transmit
Antennas") on the GPU against the FP64 oracle.

Tolerance.  The kernel forms alpha = sum_i u_i exp(j phi_i) with the phase
reduced exactly in FP64 and the exponential and the sum in FP32, so its
absolute error is a few 1e-7 times sum_i |u_i|; a crossing's weight w =
|alpha|^2 w1 (w1 the single-element weight) therefore carries an error of
order 1e-6 (sum |u_i|)^2 w1 on top of the 1e-5 relative budget of the
single-element path.  Per crossing:
    |w_gpu - w_oracle| <= 1e-5 w_oracle + 1e-5 (sum |u_i|)^2 w1,
and per cell (>= 100 crossings) the same with the cell sums, plus the border
allowance of the map protocol.  Near a null of the array the relative error
of a weight is unbounded, which is why the second term is absolute in w1.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_helpers import compare_hits, compare_sampled, gpu_radio_map, gpu_scene, scene_diag

pytestmark = pytest.mark.gpu
LAM = 299792458.0 / 3.5e9


def _steered_ula(n, c0):
    base = sg.linear_array(n, 0.5 * LAM)
    u = np.exp(-2j * math.pi * base.positions[:, 0] / LAM * c0) / math.sqrt(n)
    return sg.TxArray(base.positions, u.astype(np.complex64))


def _check(cfg, tx):
    g = gpu_radio_map(cfg, tx=tx)
    o = oracle.radio_map(cfg.scene, tx, cfg.plane, cfg.params, want_records=True)
    tx1 = sg.Tx(tx.pos, tx.yaw, tx.pitch, tx.roll, tx.pattern, tx.pattern_q, tx.pol)
    o1 = oracle.radio_map(cfg.scene, tx1, cfg.plane, cfg.params, want_records=True)
    rec, rec1 = o.records, o1.records
    assert np.array_equal(rec["ray"], rec1["ray"]) and np.array_equal(rec["depth"], rec1["depth"])
    S2 = float(np.sum(np.abs(tx.array.precoding.astype(np.complex128)))) ** 2
    hr, bad, _ = compare_hits(g.hits, o.hits, o.flags)
    assert hr["ok"], hr
    keep = ~np.isin(rec["ray"], bad)
    r, l = rec["ray"][keep], rec["depth"][keep]
    border = rec["border"][keep] <= 1e-6 * (rec["length"][keep] + scene_diag(cfg.scene))
    gc = g.cells[r, l]
    assert np.all((gc == rec["cell"][keep]) | border)
    gw = g.weights[r, l].astype(np.float64)
    ow, w1 = rec["w"][keep], rec1["w"][keep]
    err = np.abs(gw - ow)
    tol = 1e-5 * ow + 1e-5 * S2 * w1
    assert np.all((err <= tol) | border), float(np.max((err - tol)[~border]))
    # maps: cells with >= 100 crossings, without the mismatched rays
    W, H = cfg.plane.W, cfg.plane.H
    G = g.map[0].astype(np.float64).ravel().copy()
    if bad.size:
        bc, bw = g.cells[bad].ravel(), g.weights[bad].ravel().astype(np.float64)
        G -= np.bincount(bc[bc >= 0], weights=bw[bc >= 0], minlength=W * H)
    O = np.bincount(rec["cell"][keep], weights=ow, minlength=W * H)
    O1 = np.bincount(rec["cell"][keep], weights=w1, minlength=W * H)
    cnt = np.bincount(rec["cell"][keep], minlength=W * H)
    Bm = np.bincount(rec["cell"][keep][border], weights=ow[border], minlength=W * H).reshape(H, W)
    Bp = np.pad(Bm, 1)
    B = sum(Bp[1 + dj: 1 + dj + H, 1 + di: 1 + di + W] for dj in (-1, 0, 1) for di in (-1, 0, 1)).ravel()
    q = cnt >= 100
    assert q.sum() >= 50
    fail = q & (np.abs(G - O) > 1e-3 * O + 1e-5 * S2 * O1 + B)
    assert not fail.any(), int(fail.sum())
    return g, o


def test_single_element_array_is_bit_identical():
    """One element at the centre with weight 1: alpha = 1 exactly."""
    cfg = sg.tiny_config(n_rays=50_000)
    s = gpu_scene(cfg.scene)
    a = gpu_radio_map(cfg, scene_handle=s)
    one = sg.TxArray(np.zeros((1, 3)), np.ones(1, np.complex64))
    b = gpu_radio_map(cfg, scene_handle=s, tx=sg.Tx(cfg.tx.pos, array=one))
    # per-segment weights are deterministic; the maps differ only in the
    # order of their FP32 atomic sums
    assert np.array_equal(a.hits, b.hits) and np.array_equal(a.cells, b.cells)
    assert np.array_equal(a.weights, b.weights)
    np.testing.assert_allclose(b.map, a.map, rtol=2e-5, atol=1e-30)


def test_steered_ula_tiny():
    cfg = sg.tiny_config(n_rays=100_000)
    _check(cfg, sg.Tx(cfg.tx.pos, array=_steered_ula(16, 0.3)))


def test_random_array_rotated_pattern_manhattan():
    cfg = sg.manhattan_config(n_rays=200_000, max_depth=5)
    cfg.plane = sg.Plane(1.5, -500.0, -500.0, 10.0, 10.0, 100, 100)
    tx = sg.Tx((0.0, 0.0, 30.0), yaw=0.5, pitch=-0.2, roll=0.1, pattern=sg.PATTERN_DIRECTIONAL,
               array=sg.random_array(24, 0.3, seed=13))
    _check(cfg, tx)


def test_large_ula_full_lattice_sampled():
    """256-element steered ULA on the Manhattan lattice (1e7 rays): the map
    equals the sum of the per-segment weights, and strided rays match the
    oracle's crossing weights."""
    cfg = sg.manhattan_config()
    tx = sg.Tx(cfg.tx.pos, array=_steered_ula(256, 0.5))
    g = gpu_radio_map(cfg, tx=tx)
    c, w = g.cells.ravel(), g.weights.ravel().astype(np.float64)
    acc = np.bincount(c[c >= 0], weights=w[c >= 0], minlength=cfg.plane.W * cfg.plane.H)
    acc = acc.reshape(cfg.plane.H, cfg.plane.W)
    big = acc > 1e-9 * acc.max()
    np.testing.assert_allclose(g.map[0][big], acc[big], rtol=1e-4)
    N = cfg.params.n_rays
    ids = np.arange(11, N, N // 100_000, dtype=np.int64)[:100_000]
    o = oracle.radio_map(cfg.scene, tx, cfg.plane, cfg.params, ray_ids=ids, want_records=True)
    S2 = float(np.sum(np.abs(tx.array.precoding.astype(np.complex128)))) ** 2
    tx1 = sg.Tx(cfg.tx.pos)

    def tol(recs, rids, rhits):
        # 1e-5 (sum |u_i|)^2 w1 (times 4 at this array size), with w1 the
        # single-element weight of the same crossing (same path: alpha
        # changes no direction)
        o1 = oracle.radio_map(cfg.scene, tx1, cfg.plane, cfg.params, ray_ids=rids, replay_hits=rhits,
                              want_records=True)
        k1 = o1.records["ray"].astype(np.int64) * 128 + o1.records["depth"]
        k = recs["ray"].astype(np.int64) * 128 + recs["depth"]
        i = np.searchsorted(k1, k)
        assert np.array_equal(k1[i], k)
        return 4e-5 * S2 * o1.records["w"][i]

    d = compare_sampled(cfg, g.hits[ids], g.cells[ids], g.weights[ids], ids, o, 1e-5, tol_fn=tol)
    print("ula 256", d)
    assert d["ok"], d
    assert d["n_checked"] > 50_000
