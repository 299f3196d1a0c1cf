"""The parity protocol's own checks, on the CPU.

The GPU parity tests compare the HIP path's records with the oracle's through
gpu_helpers.compare_maps and compare_sampled.  Here both sides come from the
oracle (the "GPU" side is the oracle's output rounded to FP32), so the
protocol must pass; planted differences must then fail it, and a mismatch on
an oracle-flagged ray must be scored against the oracle replayed along the
other side's hit sequence rather than dropped.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_helpers import GpuResult, compare_hits, compare_maps, compare_sampled, replay_oracle


def _as_gpu(cfg, o):
    n, L1 = o.hits.shape
    cells = np.full((n, L1), -1, np.int32)
    w = np.zeros((n, L1), np.float32)
    r = o.records
    cells[r["ray"], r["depth"]] = r["cell"]
    w[r["ray"], r["depth"]] = r["w"].astype(np.float32)
    return GpuResult(o.map.astype(np.float32), o.hits.copy(), cells, w, None)


@pytest.fixture(scope="module")
def tiny():
    cfg = sg.tiny_config(n_rays=20_000)
    o = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, want_records=True)
    return cfg, o


def test_identical_sides_pass(tiny):
    cfg, o = tiny
    d = compare_maps(cfg, _as_gpu(cfg, o), o, 0, min_count=20)
    assert d["hits"]["ok"] and d["hits"]["mismatched"] == 0
    assert d["n_fail"] == 0 and d["cell_mismatch"] == 0 and d["n_cells"] > 50
    assert d["max_w_rel"] < 1e-7


def test_fraction_is_taken_over_the_rays_compared(tiny):
    cfg, o = tiny
    h = o.hits.copy()
    f = o.flags.copy()
    f[:, 0] |= oracle.FLAG_EDGE            # every ray exempt
    h[:3, 0] = -7                          # three mismatched rays
    rep, bad, rng = compare_hits(h, o.hits, f)
    assert rep["mismatched"] == 3 and rep["exempt"] == 3
    assert not rep["ok"]                   # 3 > 1e-4 x 20,000
    rep, _, _ = compare_hits(h[:30_000], o.hits, f, max_frac=2e-4)
    assert rep["ok"]                       # 3 <= 2e-4 x 20,000
    rep, _, _ = compare_hits(h[:5000], o.hits[:5000], f[:5000])
    assert not rep["ok"] and rep["cap"] == 0.5   # a 5,000-ray sample must match exactly


def test_unflagged_mismatch_fails(tiny):
    cfg, o = tiny
    g = _as_gpu(cfg, o)
    r = int(np.nonzero((o.hits[:, 1] >= 0) & ((o.flags[:, :2] != 0).sum(1) == 0))[0][0])
    g.hits[r, 1] = (g.hits[r, 1] + 1) % cfg.scene.n_triangles
    d = compare_maps(cfg, g, o, 0, min_count=20)
    assert not d["hits"]["ok"] and d["hits"]["n_unexplained"] == 1


def test_wrong_weight_and_cell_fail(tiny):
    cfg, o = tiny
    g = _as_gpu(cfg, o)
    r = o.records
    far = np.nonzero(r["border"] > 1e-3)[0][0]
    g.weights[r["ray"][far], r["depth"][far]] *= 1.0 + 3e-5
    d = compare_maps(cfg, g, o, 0, min_count=20)
    assert d["max_w_rel"] > 2e-5
    g = _as_gpu(cfg, o)
    g.cells[r["ray"][far], r["depth"][far]] += 1
    d = compare_maps(cfg, g, o, 0, min_count=20)
    assert d["cell_mismatch"] == 1


def test_flagged_mismatch_is_replayed_not_dropped():
    """The straight-down ray of the tiny scene lands on the diagonal shared by
    the two ground triangles (edge- and polar-flagged).  A side that picks the
    other triangle is scored against the oracle forced along that choice:
    with the replayed records it passes; a wrong weight on that ray fails."""
    cfg = sg.tiny_config(n_rays=20_000)
    o = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, want_records=True)
    N = cfg.params.n_rays
    r = N - 1
    assert o.hits[r, 0] in (0, 1) and (o.flags[r, 0] & (oracle.FLAG_EDGE | oracle.FLAG_POLAR))
    alt = o.hits[r].copy()
    alt[0] = 1 - alt[0]
    res = replay_oracle(cfg, np.array([r], np.int64), alt[None])
    recs, rh = res[0]
    assert np.array_equal(rh[0], alt)
    g = _as_gpu(cfg, o)
    g.hits[r] = alt
    g.cells[r] = -1
    g.weights[r] = 0
    g.cells[r, recs["depth"]] = recs["cell"]
    g.weights[r, recs["depth"]] = recs["w"].astype(np.float32)
    d = compare_maps(cfg, g, o, 0, min_count=20)
    assert d["hits"]["mismatched"] == 1 and d["hits"]["exempt"] == 1
    assert d["n_replayed"] == 1 and d["n_dropped"] == 0
    assert d["cell_mismatch"] == 0 and d["cross_only_gpu"] == 0 and d["cross_only_oracle"] == 0
    assert d["max_w_rel_replayed"] < 1e-7
    g.weights[r, recs["depth"][-1]] *= 1.0 + 1e-4
    d = compare_maps(cfg, g, o, 0, min_count=20)
    assert d["max_w_rel_replayed"] > 5e-5
    # the same ray through the sampled protocol
    ids = np.array([0, 5, r], np.int64)
    os_ = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_ids=ids, want_records=True)
    ds = compare_sampled(cfg, g.hits[ids], g.cells[ids], g.weights[ids], ids, os_, 1e-5, max_frac=0.5)
    assert ds["n_replayed"] == 1 and ds["weight_fail"] == 1 and not ds["ok"]
    g.weights[r, recs["depth"][-1]] = np.float32(recs["w"][-1])
    ds = compare_sampled(cfg, g.hits[ids], g.cells[ids], g.weights[ids], ids, os_, 1e-5, max_frac=0.5)
    assert ds["ok"], ds
