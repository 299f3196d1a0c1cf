"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI,
run the oracle on the same seeded inputs, and compare them.

The comparison protocol (integer hit sequences, per-crossing cells and
weights, per-cell maps) only ever feeds oracle inputs from the seeded input
generators; GPU outputs are compared against oracle outputs, never fed back.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

import oracle
import scenegen as sg

EXEMPT_FLAGS = (oracle.FLAG_EDGE | oracle.FLAG_TIE | oracle.FLAG_GRAZING | oracle.FLAG_NEAR | oracle.FLAG_POLAR
                | oracle.FLAG_TERM | oracle.FLAG_CHOICE)


@dataclasses.dataclass
class GpuResult:
    map: np.ndarray            # [npol][H][W] float32
    hits: Optional[np.ndarray]
    cells: Optional[np.ndarray]
    weights: Optional[np.ndarray]
    stats: Optional[np.ndarray]


def gpu_scene(scene):
    import paper_2504_21719_amd as rt
    return rt.scene_from_mesh(scene)


def gpu_radio_map(cfg, *, scene_handle=None, ray_begin=None, ray_end=None, records=True, accel=0, deposit=0,
                  block_size=0, eps_r=None, sigma=None, tx=None, stream=None, thickness=None, scattering=None,
                  xpd=None, pattern=None):
    import torch
    import paper_2504_21719_amd as rt
    s = scene_handle if scene_handle is not None else gpu_scene(cfg.scene)
    tx = tx if tx is not None else cfg.tx
    npol = 2 if tx.pol == sg.POL_DUAL else 1
    b = cfg.params.ray_begin if ray_begin is None else ray_begin
    e = cfg.params.end() if ray_end is None else ray_end
    n = e - b
    L = cfg.params.max_depth
    dev = "cuda"
    eps = torch.tensor(cfg.scene.eps_r if eps_r is None else eps_r, dtype=torch.float32, device=dev)
    sig = torch.tensor(cfg.scene.sigma if sigma is None else sigma, dtype=torch.float32, device=dev)
    if thickness is None:
        thickness = cfg.scene.thickness
    thk = None if thickness is None else torch.tensor(thickness, dtype=torch.float32, device=dev)
    if scattering is None:
        scattering, xpd = cfg.scene.scattering, cfg.scene.xpd
    sca = None if scattering is None else torch.tensor(scattering, dtype=torch.float32, device=dev)
    xp = None if xpd is None else torch.tensor(xpd, dtype=torch.float32, device=dev)
    if pattern is None:
        pattern = cfg.scene.scatter_pattern
    pat = None if pattern is None else torch.tensor(pattern, dtype=torch.float32, device=dev)
    out = torch.full((npol, cfg.plane.H, cfg.plane.W), float("nan"), dtype=torch.float32, device=dev)
    hits = cells = weights = stats = None
    if records:
        hits = torch.empty((max(n, 1), L + 1), dtype=torch.int32, device=dev)
        cells = torch.empty((max(n, 1), L + 1), dtype=torch.int32, device=dev)
        weights = torch.empty((max(n, 1), L + 1), dtype=torch.float32, device=dev)
        stats = torch.zeros(8, dtype=torch.int64, device=dev)
    rt.rt_radio_map(s, eps, sig, tx, cfg.plane, cfg.params, out, hits=hits, cells=cells, weights=weights,
                    stats=stats, ray_begin=b, ray_end=e, accel=accel, deposit=deposit, block_size=block_size,
                    stream=stream, thickness=thk, scattering=sca, xpd=xp, scatter_pattern=pat)
    torch.cuda.synchronize()
    c = lambda t: None if t is None else t.cpu().numpy()[:n] if t.dim() == 2 else t.cpu().numpy()
    return GpuResult(out.cpu().numpy(), c(hits), c(cells), c(weights), None if stats is None else stats.cpu().numpy())


def scene_diag(scene) -> float:
    V = scene.vertices.astype(np.float64)
    if V.shape[0] == 0:
        return 0.0
    return float(np.linalg.norm(V.max(0) - V.min(0)))


RNG_FLAGS = oracle.FLAG_TERM | oracle.FLAG_CHOICE


def compare_hits(g_hits, o_hits, o_flags, max_frac=1e-4):
    """Integer protocol over the rays compared: hit sequences bit-exact except
    rays the oracle flagged (edge, tie, grazing, near-origin, polar ray,
    random-decision near-tie) at or before their first mismatch, and such rays
    at most ``max_frac`` of the rays compared (no floor of one ray: a sample
    too small to resolve the fraction must match exactly).

    Returns (report, bad, rng): the mismatched run indices, and for each of
    them whether its exemption is a random-decision near-tie (early
    termination or interaction type), which a forced hit sequence cannot
    replay."""
    n = int(g_hits.shape[0])
    diff = g_hits != o_hits
    bad = np.nonzero(diff.any(1))[0]
    if bad.size:
        first = np.argmax(diff[bad], axis=1)
        fl = o_flags[bad]
        ex = np.cumsum((fl & EXEMPT_FLAGS) != 0, axis=1)[np.arange(bad.size), first] > 0
        rng = np.cumsum((fl & RNG_FLAGS) != 0, axis=1)[np.arange(bad.size), first] > 0
    else:
        ex = rng = np.zeros(0, bool)
    unexplained = bad[~ex].tolist()
    report = dict(rays=n, mismatched=int(bad.size), exempt=int(ex.sum()), frac=bad.size / max(n, 1),
                  cap=max_frac * n, unexplained=unexplained[:20], n_unexplained=len(unexplained))
    report["ok"] = (not unexplained) and bad.size <= max_frac * n
    return report, bad, rng


def _keys(ray, depth):
    return ray.astype(np.int64) * 128 + depth.astype(np.int64)


def replay_oracle(cfg, ray_ids, hits, **kw):
    """Oracle records of rays forced along given hit sequences (the GPU's),
    with the oracle's own FP64 arithmetic on that path.  Returns (records,
    replayed hits) or None where the oracle cannot follow the sequence."""
    def run(ids, h):
        return oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_ids=ids, replay_hits=h,
                                want_records=True, **kw)
    try:
        r = run(ray_ids, hits)
        return [(r.records, r.hits)]
    except ValueError:
        out = []
        for i in range(ray_ids.size):
            try:
                r = run(ray_ids[i:i + 1], hits[i:i + 1])
                out.append((r.records, r.hits))
            except ValueError:
                out.append(None)
        return out


def compare_maps(cfg, g: GpuResult, o, ray_begin, min_count=100, rel=1e-3, max_frac=1e-4):
    """Per-cell protocol over a ray range [ray_begin, ray_begin + n).

    * hit sequences: compare_hits over the rays compared;
    * mismatched rays are scored against a replay-corrected oracle: their
      oracle crossings are replaced by the oracle's FP64 crossings along the
      GPU's hit sequence (forced hits), so the GPU's own deposits on those
      rays are checked too.  Only rays whose exemption is a random-decision
      near-tie (which a forced hit sequence cannot follow) are removed from
      both sides;
    * every GPU crossing must match a crossing of the corrected oracle and
      land in its cell, unless the oracle marked it within delta_b of a cell
      border; weights are compared crossing by crossing;
    * every cell with >= min_count corrected-oracle crossings must satisfy
      |G - O'| <= rel * O' + B, with B the oracle weight of border-flagged
      crossings in the cell and its 8 neighbours.
    Returns a dict of diagnostics.  Polarisation 0 only.
    """
    W, H = cfg.plane.W, cfg.plane.H
    n = g.hits.shape[0]
    hr, bad, rng = compare_hits(g.hits, o.hits, o.flags, max_frac)
    rec = o.records
    rrel = rec["ray"] - ray_begin
    badset = np.zeros(n, bool)
    badset[bad] = True
    drop = np.zeros(n, bool)
    drop[bad[rng]] = True
    # replay the GPU's hit sequence through the oracle for the other mismatched rays
    rep_ids = bad[~rng]
    parts = []
    n_replayed = 0
    if rep_ids.size:
        res = replay_oracle(cfg, ray_begin + rep_ids.astype(np.int64), g.hits[rep_ids])
        groups = [rep_ids] if len(res) == 1 else [rep_ids[i:i + 1] for i in range(rep_ids.size)]
        for ids, r in zip(groups, res):
            if r is None:
                drop[ids] = True
                continue
            recs, rh = r
            same = (rh == g.hits[ids]).all(1)
            drop[ids[~same]] = True
            keep_r = np.isin(recs["ray"] - ray_begin, ids[same])
            parts.append({k: v[keep_r] for k, v in recs.items()})
            n_replayed += int(same.sum())
    # corrected oracle records: unchanged rays + replayed rays, sorted by (ray, depth)
    base = ~badset[rrel]
    R = {k: np.concatenate([v[base]] + [p[k] for p in parts]) for k, v in rec.items()}
    order = np.argsort(_keys(R["ray"], R["depth"]), kind="stable")
    R = {k: v[order] for k, v in R.items()}
    r_rel = R["ray"] - ray_begin
    keep = ~drop[r_rel]
    R = {k: v[keep] for k, v in R.items()}
    r_rel = r_rel[keep]
    o_key = _keys(r_rel, R["depth"])
    # GPU crossings of rays not dropped, in (ray, depth) order
    gsel = (g.cells >= 0) & (~drop[:, None])
    g_r, g_l = np.nonzero(gsel)
    g_key = _keys(g_r, g_l)
    E = scene_diag(cfg.scene)
    border = R["border"] <= 1e-6 * (R["length"] + E)
    common, oi, gi = np.intersect1d(o_key, g_key, assume_unique=True, return_indices=True)
    only_o_mask = np.ones(o_key.size, bool)
    only_o_mask[oi] = False
    only_o = int((only_o_mask & ~border).sum())
    only_g = int(g_key.size - common.size)
    gc = g.cells[g_r[gi], g_l[gi]]
    oc = R["cell"][oi]
    cell_mismatch = (gc != oc) & ~border[oi]
    gw = g.weights[g_r[gi], g_l[gi]].astype(np.float64)
    ow = R["w"][oi]
    wrel = np.abs(gw - ow) / np.maximum(ow, 1e-300)
    rep_rows = np.isin(g_r[gi], rep_ids[~drop[rep_ids]]) if rep_ids.size else np.zeros(gi.size, bool)
    # maps: GPU without the dropped rays, corrected oracle map
    G = g.map[0].astype(np.float64).ravel().copy()
    dr = np.nonzero(drop)[0]
    if dr.size:
        bc = g.cells[dr].ravel()
        bw = g.weights[dr].ravel().astype(np.float64)
        m = bc >= 0
        G -= np.bincount(bc[m], weights=bw[m], minlength=W * H)
    O = np.bincount(R["cell"], weights=R["w"], minlength=W * H).astype(np.float64)
    cnt = np.bincount(R["cell"], minlength=W * H)
    # border allowance: oracle mass of flagged crossings in the 3x3 neighbourhood
    Bm = np.bincount(R["cell"][border], weights=R["w"][border], minlength=W * H).reshape(H, W)
    Bp = np.pad(Bm, 1)
    B = sum(Bp[1 + dj: 1 + dj + H, 1 + di: 1 + di + W] for dj in (-1, 0, 1) for di in (-1, 0, 1)).ravel()
    q = cnt >= min_count
    err = np.abs(G - O)
    fail = q & (err > rel * O + B)
    clean = q & (B == 0)
    return dict(hits=hr, n_cells=int(q.sum()), n_fail=int(fail.sum()),
                max_rel_clean=float((err[clean] / O[clean]).max()) if clean.any() else 0.0,
                max_rel_all=float((err[q] / O[q]).max()) if q.any() else 0.0,
                cross_only_oracle=only_o, cross_only_gpu=only_g,
                cell_mismatch=int(cell_mismatch.sum()), n_border=int(border.sum()),
                max_w_rel=float(wrel.max()) if wrel.size else 0.0, n_common=int(common.size),
                n_replayed=n_replayed, n_dropped=int(drop.sum()),
                max_w_rel_replayed=float(wrel[rep_rows].max()) if rep_rows.any() else 0.0)


def compare_sampled(cfg, hits, cells, weights, ids, o, w_rel, diag=None, max_frac=1e-4, tol_fn=None, oracle_kw=None):
    """Integer and per-crossing protocol on a sample of lattice rays.

    hits / cells / weights: GPU records of the sampled rays, row i for lattice
    ray ids[i]; o: the oracle run over the same ids with records.  Checks:
    * compare_hits over the rays compared (at most max_frac of them mismatched,
      all oracle-flagged);
    * for every ray, matched or replayed (a mismatched ray is rerun through the
      oracle along the GPU's hit sequence), the same crossing set, the same
      cell unless the oracle marks the crossing within delta_b of a border, and
      weights of every common crossing within w_rel (plus tol_fn(records, ids,
      replay_hits), an absolute allowance per record, if given).
    Only rays whose exemption is a random-decision near-tie are left out.
    Returns a dict of diagnostics; `ok` is the verdict."""
    kw = dict(oracle_kw or {})
    rep, bad, rng = compare_hits(hits, o.hits, o.flags, max_frac)
    E = scene_diag(cfg.scene) if diag is None else diag
    pos = np.full(int(ids.max()) + 1 if ids.size else 1, -1, np.int64)
    pos[ids] = np.arange(ids.size)
    dropped = set(bad[rng].tolist())
    recs_all = []
    rec = o.records
    keep = ~np.isin(pos[rec["ray"]], bad)
    base = {k: v[keep] for k, v in rec.items()}
    base["_tol"] = tol_fn(base, ids, None) if tol_fn else np.zeros(base["w"].size)
    recs_all.append(base)
    n_replayed = 0
    rb = bad[~rng]
    if rb.size:
        res = replay_oracle(cfg, ids[rb], hits[rb], **kw)
        groups = [rb] if len(res) == 1 else [rb[i:i + 1] for i in range(rb.size)]
        for grp, r in zip(groups, res):
            if r is None:
                dropped.update(grp.tolist())
                continue
            rr, rh = r
            same = (rh == hits[grp]).all(1)
            dropped.update(grp[~same].tolist())
            kr = np.isin(pos[rr["ray"]], grp[same])
            sub = {k: v[kr] for k, v in rr.items()}
            sub["_tol"] = tol_fn(sub, ids[grp[same]], hits[grp[same]]) if tol_fn else np.zeros(sub["w"].size)
            recs_all.append(sub)
            n_replayed += int(same.sum())
    R = {k: np.concatenate([q[k] for q in recs_all]) for k in recs_all[0]}
    row = pos[R["ray"]]
    border = R["border"] <= 1e-6 * (R["length"] + E)
    okrow = np.ones(ids.size, bool)
    okrow[list(dropped)] = False
    o_key = _keys(row, R["depth"])
    gsel = (cells >= 0) & okrow[:, None]
    g_r, g_l = np.nonzero(gsel)
    g_key = _keys(g_r, g_l)
    common, oi, gi = np.intersect1d(o_key, g_key, assume_unique=True, return_indices=True)
    only_o = np.ones(o_key.size, bool)
    only_o[oi] = False
    gc = cells[g_r[gi], g_l[gi]]
    cm = (gc != R["cell"][oi]) & ~border[oi]
    gw = weights[g_r[gi], g_l[gi]].astype(np.float64)
    ow = R["w"][oi]
    err = np.abs(gw - ow)
    tol = w_rel * ow + R["_tol"][oi]
    wbad = err > tol                 # a border flag excuses the cell, never the weight
    d = dict(hits=rep, n_replayed=n_replayed, n_dropped=len(dropped), n_crossings=int(o_key.size),
             cross_only_oracle=int((only_o & ~border).sum()), cross_only_gpu=int(g_key.size - common.size),
             cell_mismatch=int(cm.sum()), weight_fail=int(wbad.sum()), n_checked=int(common.size),
             n_border=int(border.sum()),
             max_w_rel=float((err / np.maximum(ow, 1e-300)).max()) if common.size else 0.0)
    d["ok"] = (rep["ok"] and d["cross_only_oracle"] == 0 and d["cross_only_gpu"] == 0 and d["cell_mismatch"] == 0
               and d["weight_fail"] == 0)
    return d


def assert_parity(d, max_w_rel=1e-5):
    assert d["hits"]["ok"], d["hits"]
    assert d["cross_only_oracle"] == 0 and d["cross_only_gpu"] == 0, d
    assert d["cell_mismatch"] == 0, d
    assert d["n_fail"] == 0, d
    assert d["max_w_rel"] <= max_w_rel, d
