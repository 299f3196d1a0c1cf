"""FP64 CPU oracle of the SBR radio map (test infrastructure): specular
reflection by default; slab walls, refraction, diffuse reflection, transmit
arrays and early termination on request.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it.

The arithmetic lives in ``sbr_oracle.c`` (plain C99, double precision, one
thread, brute-force intersection).  This module only builds that file with
gcc (no fast-math), marshals arguments with ctypes, and offers a process-pool
helper that splits a ray range across worker processes and sums their maps
(the map is a sum over rays, so the split changes nothing but the summation
order).
"""
from __future__ import annotations

import ctypes as C
import gc
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

FLAG_EDGE, FLAG_TIE, FLAG_GRAZING, FLAG_NEAR, FLAG_POLAR, FLAG_TERM, FLAG_CHOICE = 1, 2, 4, 8, 16, 32, 64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Tx(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("yaw", C.c_double), ("pitch", C.c_double),
                ("roll", C.c_double), ("pattern", C.c_int32), ("q", C.c_double),
                ("pol", C.c_int32), ("n_ant", C.c_int32), ("ant_pos", C.c_void_p),
                ("precoding", C.c_void_p)]


class _Plane(C.Structure):
    _fields_ = [("z", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("W", C.c_int32), ("H", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("freq", C.c_double), ("n_rays", C.c_int64), ("max_depth", C.c_int32),
                ("t_min", C.c_double), ("rr_depth", C.c_int32), ("rr_p_max", C.c_double),
                ("gain_threshold", C.c_double), ("seed", C.c_uint32), ("refraction", C.c_int32)]


class _Out(C.Structure):
    _fields_ = [("map", C.c_void_p), ("counts", C.c_void_p), ("hits", C.c_void_p),
                ("flags", C.c_void_p), ("rec_cap", C.c_int64), ("rec_n", C.c_int64),
                ("rec_ray", C.c_void_p), ("rec_depth", C.c_void_p), ("rec_cell", C.c_void_p),
                ("rec_w", C.c_void_p), ("rec_border", C.c_void_p), ("rec_len", C.c_void_p),
                ("grad_map", C.c_void_p), ("grad", C.c_void_p), ("replay_hits", C.c_void_p),
                ("tri_tests", C.c_int64), ("segments", C.c_int64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            L.or_radio_map.restype = C.c_int
            L.or_radio_map.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.POINTER(_Tx),
                                       C.POINTER(_Plane), C.POINTER(_Params), C.c_void_p, C.c_int64,
                                       C.c_int64, C.c_int64, C.POINTER(_Out)]
            L.or_fresnel.restype = None
            L.or_fresnel.argtypes = [C.c_double] * 4 + [C.POINTER(C.c_double)] * 4
            L.or_fresnel_slab.restype = None
            L.or_fresnel_slab.argtypes = [C.c_double] * 5 + [C.c_void_p]
            L.or_path_field.restype = C.c_int
            L.or_path_field.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_void_p, C.c_void_p]
            L.or_scatter_pattern.restype = C.c_double
            L.or_scatter_pattern.argtypes = [C.c_void_p] * 4
            L.or_uniform.restype = C.c_double
            L.or_uniform.argtypes = [C.c_uint32, C.c_int64, C.c_int, C.c_uint32]
            L.or_launch_field.restype = None
            L.or_launch_field.argtypes = [C.c_double] * 3 + [C.POINTER(_Tx), C.c_int, C.c_void_p, C.c_void_p]
            L.or_lattice_dir.restype = None
            L.or_lattice_dir.argtypes = [C.c_int64, C.c_int64, C.c_void_p]
            L.or_philox4x32.restype = None
            L.or_philox4x32.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
            L.or_fibonacci.restype = None
            L.or_fibonacci.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
            _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _tx(tx) -> _Tx:
    t = _Tx()
    t.pos[:] = [float(v) for v in tx.pos]
    t.yaw, t.pitch, t.roll = float(tx.yaw), float(tx.pitch), float(tx.roll)
    t.pattern, t.q, t.pol = int(tx.pattern), float(tx.pattern_q), int(tx.pol)
    ant = getattr(tx, "array", None)
    if ant is not None:
        pos = np.ascontiguousarray(ant.positions, dtype=np.float64).reshape(-1, 3)
        u = np.asarray(ant.precoding).astype(np.complex128).reshape(-1)
        if u.shape[0] != pos.shape[0]:
            raise ValueError("one precoding weight per array element")
        prec = np.ascontiguousarray(np.stack([u.real, u.imag], axis=1))
        t.n_ant = pos.shape[0]
        t.ant_pos, t.precoding = pos.ctypes.data, prec.ctypes.data
        t._keep = (pos, prec)          # the arrays live as long as the struct
    return t


def philox4x32(ctr, key):
    """Philox4x32-10 block (four 32-bit counter words, two key words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().or_philox4x32(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def _plane(p) -> _Plane:
    return _Plane(float(p.z), float(p.x0), float(p.y0), float(p.dx), float(p.dy), int(p.W), int(p.H))


@dataclass
class OracleResult:
    map: np.ndarray                 # float64 [npol][H][W]
    counts: np.ndarray              # int64 [H][W]
    hits: Optional[np.ndarray]      # int32 [n_run][L+1]
    flags: Optional[np.ndarray]     # uint8 [n_run][L+1]
    records: Optional[dict]         # crossing records
    grad: Optional[np.ndarray]      # float64 [2 n_mat + 3]
    segments: int
    tri_tests: int


def radio_map(scene, tx, plane, params, *, ray_ids=None, ray_begin=None, ray_end=None,
              eps_r=None, sigma=None, thickness=None, scattering=None, xpd=None, pattern=None, want_hits=False,
              want_records=False, rec_cap=None,
              grad_map=None, replay_hits=None) -> OracleResult:
    """Run the oracle over a ray range (default: the params' range) or an explicit list.

    ``thickness`` (metres per material; default ``scene.thickness``, None =
    half-space walls) switches to the slab coefficients; ``params.refraction``
    samples reflection or transmission at every hit and needs a thickness.
    ``scattering`` / ``xpd`` (S and K_x per material; default ``scene.scattering``
    and ``scene.xpd``) enable Lambertian diffuse reflection."""
    L = lib()
    V = np.ascontiguousarray(scene.vertices, dtype=np.float32)
    F = np.ascontiguousarray(scene.triangles, dtype=np.int32)
    M = np.ascontiguousarray(scene.tri_material, dtype=np.int32)
    eps = np.ascontiguousarray(scene.eps_r if eps_r is None else eps_r, dtype=np.float64)
    sig = np.ascontiguousarray(scene.sigma if sigma is None else sigma, dtype=np.float64)
    if thickness is None:
        thickness = getattr(scene, "thickness", None)
    thk = None if thickness is None else np.ascontiguousarray(thickness, dtype=np.float64)
    if scattering is None:
        scattering = getattr(scene, "scattering", None)
    if xpd is None:
        xpd = getattr(scene, "xpd", None)
    sca = None if scattering is None else np.ascontiguousarray(scattering, dtype=np.float64)
    xp = None if xpd is None else np.ascontiguousarray(xpd, dtype=np.float64)
    if pattern is None:
        pattern = getattr(scene, "scatter_pattern", None)
    pat = None if pattern is None else np.ascontiguousarray(pattern, dtype=np.float64).reshape(-1, 4)
    n_mat = int(eps.shape[0])
    npol = 2 if int(tx.pol) == 2 else 1
    Lmax = int(params.max_depth)
    if ray_ids is not None:
        ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        n_run = int(ids.shape[0])
        b = e = 0
    else:
        ids = None
        b = int(params.ray_begin if ray_begin is None else ray_begin)
        e = int(params.end() if ray_end is None else ray_end)
        n_run = e - b
    out = _Out()
    mp = np.zeros((npol, plane.H, plane.W), np.float64)
    cnt = np.zeros((plane.H, plane.W), np.int64)
    out.map, out.counts = mp.ctypes.data, cnt.ctypes.data
    hits = flags = None
    if want_hits or want_records:
        hits = np.zeros((n_run, Lmax + 1), np.int32)
        flags = np.zeros((n_run, Lmax + 1), np.uint8)
        out.hits, out.flags = hits.ctypes.data, flags.ctypes.data
    recs = None
    if want_records:
        cap = int(rec_cap if rec_cap is not None else n_run * (Lmax + 1))
        recs = dict(ray=np.zeros(cap, np.int64), depth=np.zeros(cap, np.int32),
                    cell=np.zeros(cap, np.int32), w=np.zeros(cap, np.float64),
                    border=np.zeros(cap, np.float64), length=np.zeros(cap, np.float64))
        out.rec_cap = cap
        out.rec_ray, out.rec_depth, out.rec_cell = (recs["ray"].ctypes.data, recs["depth"].ctypes.data,
                                                    recs["cell"].ctypes.data)
        out.rec_w, out.rec_border, out.rec_len = (recs["w"].ctypes.data, recs["border"].ctypes.data,
                                                  recs["length"].ctypes.data)
    grad = None
    gm = None
    if grad_map is not None:
        gm = np.ascontiguousarray(np.broadcast_to(grad_map, (npol, plane.H, plane.W)), dtype=np.float64)
        grad = np.zeros(2 * n_mat + 3, np.float64)
        out.grad_map, out.grad = gm.ctypes.data, grad.ctypes.data
    rh = None
    if replay_hits is not None:
        rh = np.ascontiguousarray(replay_hits, dtype=np.int32)
        assert rh.shape == (n_run, Lmax + 1)
        out.replay_hits = rh.ctypes.data
    prm = _Params(float(params.freq_hz), int(params.n_rays), Lmax, float(params.t_min),
                  int(getattr(params, "rr_depth", 1)), float(getattr(params, "rr_p_max", 0.0)),
                  float(getattr(params, "gain_threshold", 0.0)), int(getattr(params, "seed", 0)) & 0xffffffff,
                  int(getattr(params, "refraction", 0)))
    txs, pls = _tx(tx), _plane(plane)
    rc = L.or_radio_map(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], M.ctypes.data, n_mat,
                        eps.ctypes.data, sig.ctypes.data, _ptr(thk), _ptr(sca), _ptr(xp), _ptr(pat), C.byref(txs), C.byref(pls), C.byref(prm),
                        _ptr(ids), n_run if ids is not None else 0, b, e, C.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (code %d)" % rc)
    if recs is not None:
        n = min(int(out.rec_n), int(out.rec_cap))
        if int(out.rec_n) > int(out.rec_cap):
            raise RuntimeError("crossing-record capacity exceeded")
        recs = {k: v[:n] for k, v in recs.items()}
    return OracleResult(mp, cnt, hits, flags, recs, grad, int(out.segments), int(out.tri_tests))


def fresnel(eps_r, sigma, freq, cos_theta):
    """(r_perp, r_par) of eq. fresnel_vac, as complex numbers (oracle arithmetic)."""
    L = lib()
    a, b, c, d = (C.c_double(), C.c_double(), C.c_double(), C.c_double())
    L.or_fresnel(eps_r, sigma, freq, cos_theta, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
    return complex(a.value, b.value), complex(c.value, d.value)


def path_field(points, normals, eps_r, sigma, freq, E0):
    """Field at the end of a specular chain (source, reflection points, end
    point) carried with the radio map's interaction step; returns (E, k) with
    E complex [3] and k the direction of the last segment."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    nr = np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3)
    er = np.ascontiguousarray(eps_r, dtype=np.float64).ravel()
    sg_ = np.ascontiguousarray(sigma, dtype=np.float64).ravel()
    if nr.shape[0] != pts.shape[0] - 2 or er.size != nr.shape[0] or sg_.size != nr.shape[0]:
        raise ValueError("path_field: one normal and one material per reflection point")
    e0 = np.ascontiguousarray(np.stack([np.real(E0), np.imag(E0)], axis=1).ravel(), dtype=np.float64)
    out = np.zeros(9)
    if lib().or_path_field(pts.ctypes.data, pts.shape[0], nr.ctypes.data, er.ctypes.data, sg_.ctypes.data,
                           float(freq), e0.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("path_field: bad sizes")
    return out[0:6:2] + 1j * out[1:6:2], out[6:9]


def fresnel_slab(eps_r, sigma, freq, cos_theta, d):
    """(r_perp, r_par, t_perp, t_par) of a slab of thickness d, eq. fresnel_slab."""
    o = np.zeros(8)
    lib().or_fresnel_slab(eps_r, sigma, freq, cos_theta, d, o.ctypes.data)
    return complex(o[0], o[1]), complex(o[2], o[3]), complex(o[4], o[5]), complex(o[6], o[7])


def scatter_pattern(pp, ki, ks, n):
    """f_s of the oracle: pp = (kind, alpha_R, alpha_I, Lambda); unit vectors."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (pp, ki, ks, n)]
    return float(lib().or_scatter_pattern(*[x.ctypes.data for x in a]))


def uniform(seed, n, l, stream):
    """The oracle's uniform draw for ray n, index l and stream (0 termination, 1 interaction type)."""
    return float(lib().or_uniform(int(seed) & 0xffffffff, int(n), int(l), int(stream)))


def launch_field(k, tx, pol_index=0):
    """Global-frame transmitted field vector and its d/d(yaw,pitch,roll) [3][3]."""
    L = lib()
    E = np.zeros(3)
    dE = np.zeros((3, 3))
    t = _tx(tx)
    L.or_launch_field(float(k[0]), float(k[1]), float(k[2]), C.byref(t), pol_index, E.ctypes.data, dE.ctypes.data)
    return E, dE


def lattice(n, N):
    L = lib()
    k = np.zeros(3)
    L.or_lattice_dir(int(n), int(N), k.ctypes.data)
    return k


def fibonacci_angles(n, N):
    L = lib()
    th, ph = C.c_double(), C.c_double()
    L.or_fibonacci(int(n), int(N), C.byref(th), C.byref(ph))
    return th.value, ph.value


# ---------------------------------------------------------------- parallel
def _worker(args):
    scene, tx, plane, params, b, e, kw = args
    return radio_map(scene, tx, plane, params, ray_begin=b, ray_end=e, **kw)


def radio_map_parallel(scene, tx, plane, params, workers=None, chunks_per_worker=1, replay_hits=None, **kw):
    """Split [ray_begin, ray_end) over a process pool and combine the chunks.

    Maps, counts and gradients are summed; hits, flags and crossing records
    are concatenated in ray order.  ``replay_hits`` ([n_rays_run][L+1]) is
    split along with the rays.
    """
    import multiprocessing as mp
    workers = int(workers or min(16, os.cpu_count() or 1))
    b0, e0 = int(params.ray_begin), int(params.end())
    n = e0 - b0
    nchunk = max(1, min(n, workers * chunks_per_worker))
    edges = [b0 + (n * i) // nchunk for i in range(nchunk + 1)]
    jobs = []
    for i in range(nchunk):
        if edges[i + 1] <= edges[i]:
            continue
        kwi = dict(kw)
        if replay_hits is not None:
            kwi["replay_hits"] = replay_hits[edges[i] - b0: edges[i + 1] - b0]
        jobs.append((scene, tx, plane, params, edges[i], edges[i + 1], kwi))
    lib()  # build before forking
    gc.collect()  # collect before forking, so that no finalizer runs in a worker
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = pool.map(_worker, jobs)
    mp_ = sum(p.map for p in parts)
    cnt = sum(p.counts for p in parts)
    grad = sum(p.grad for p in parts) if parts[0].grad is not None else None
    hits = np.concatenate([p.hits for p in parts]) if parts[0].hits is not None else None
    flags = np.concatenate([p.flags for p in parts]) if parts[0].flags is not None else None
    recs = None
    if parts[0].records is not None:
        recs = {k: np.concatenate([p.records[k] for p in parts]) for k in parts[0].records}
    return OracleResult(mp_, cnt, hits, flags, recs, grad, sum(p.segments for p in parts),
                        sum(p.tri_tests for p in parts))
