"""Python binding of librtmap.so, the MI355X SBR radio-map library.

Argument marshalling only: every step of the SBR path runs in the HIP
kernels behind the C ABI declared in ``include/rt.h``.  PyTorch supplies
device memory and the current HIP stream.  The functions keep the C names
(``rt_build_scene``, ``rt_radio_map``, ``rt_radio_map_backward``,
``rt_radio_map_batched``, ...).

There is no fallback: importing this package without the built library, or
calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmap.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EOVERFLOW, RT_EUNSUPPORTED = range(6)
RT_ACCEL_BVH, RT_ACCEL_BRUTE, RT_ACCEL_BVH2, RT_ACCEL_BVH4 = 0, 1, 2, 3
RT_DEPOSIT_AUTO, RT_DEPOSIT_ATOMIC, RT_DEPOSIT_WAVE = 0, 1, 2
RT_POL_V, RT_POL_H, RT_POL_DUAL = 0, 1, 2

EXPORTED = ["rt_last_error", "rt_build_scene", "rt_scene_destroy", "rt_scene_info_get", "rt_radio_map",
            "rt_tape_bytes", "rt_tape_create", "rt_tape_destroy", "rt_radio_map_backward",
            "rt_radio_map_backward_noalloc",
            "rt_radio_map_batched", "rt_tune", "rt_set_launch_config", "rt_scene_export"]


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("rt status %d: %s" % (status, msg))
        self.status = status


class rt_scene_info(C.Structure):
    _fields_ = [("n_triangles", C.c_int64), ("n_materials", C.c_int32), ("bvh_depth", C.c_int32),
                ("n_nodes", C.c_int64), ("device_bytes", C.c_int64), ("build_ms", C.c_double),
                ("tuned_block", C.c_int32), ("tuned_deposit", C.c_int32), ("tuned_refill", C.c_int32),
                ("tuned_order", C.c_int32), ("tuned_width", C.c_int32), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3)]


class rt_materials(C.Structure):
    _fields_ = [("eps_r", C.c_void_p), ("sigma", C.c_void_p), ("thickness", C.c_void_p),
                ("scattering", C.c_void_p), ("xpd", C.c_void_p), ("scatter_pattern", C.c_void_p)]


class rt_tx(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("yaw", C.c_double), ("pitch", C.c_double), ("roll", C.c_double),
                ("pattern", C.c_int32), ("pattern_q", C.c_float), ("pol", C.c_int32),
                ("n_ant", C.c_int32), ("ant_pos", C.c_void_p), ("precoding", C.c_void_p)]


class rt_plane(C.Structure):
    _fields_ = [("z", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double),
                ("dy", C.c_double), ("W", C.c_int32), ("H", C.c_int32)]


class rt_sbr_params(C.Structure):
    _fields_ = [("freq_hz", C.c_double), ("n_rays", C.c_int64), ("ray_begin", C.c_int64),
                ("ray_end", C.c_int64), ("max_depth", C.c_int32), ("accumulate", C.c_int32),
                ("t_min", C.c_float), ("accel", C.c_int32), ("deposit", C.c_int32), ("block_size", C.c_int32),
                ("rr_depth", C.c_int32), ("rr_p_max", C.c_float), ("gain_threshold", C.c_float),
                ("seed", C.c_uint32), ("refraction", C.c_int32)]


class rt_records(C.Structure):
    _fields_ = [("hits", C.c_void_p), ("cells", C.c_void_p), ("weights", C.c_void_p), ("stats", C.c_void_p)]


_lib = None


def lib():
    """Load librtmap.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("librtmap.so is not built; run paper_2504_21719_amd/build.py (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.rt_last_error.restype = C.c_char_p
    L.rt_last_error.argtypes = []
    L.rt_build_scene.restype = C.c_int
    L.rt_build_scene.argtypes = [vp, i64, vp, i64, vp, i32, vp, C.POINTER(vp)]
    L.rt_scene_destroy.restype = C.c_int
    L.rt_scene_destroy.argtypes = [vp]
    L.rt_scene_info_get.restype = C.c_int
    L.rt_scene_info_get.argtypes = [vp, C.POINTER(rt_scene_info)]
    L.rt_radio_map.restype = C.c_int
    L.rt_radio_map.argtypes = [vp, rt_materials, C.POINTER(rt_tx), C.POINTER(rt_plane),
                               C.POINTER(rt_sbr_params), vp, vp, C.POINTER(rt_records), vp]
    L.rt_tape_bytes.restype = C.c_size_t
    L.rt_tape_bytes.argtypes = [C.POINTER(rt_sbr_params)]
    L.rt_tape_create.restype = C.c_int
    L.rt_tape_create.argtypes = [C.POINTER(rt_sbr_params), C.POINTER(vp)]
    L.rt_tape_destroy.restype = C.c_int
    L.rt_tape_destroy.argtypes = [vp]
    L.rt_radio_map_backward.restype = C.c_int
    L.rt_radio_map_backward.argtypes = [vp, rt_materials, C.POINTER(rt_tx), C.POINTER(rt_plane),
                                        C.POINTER(rt_sbr_params), vp, vp, vp, vp, vp, vp]
    L.rt_radio_map_backward_noalloc.restype = C.c_int
    L.rt_radio_map_backward_noalloc.argtypes = L.rt_radio_map_backward.argtypes
    L.rt_radio_map_batched.restype = C.c_int
    L.rt_radio_map_batched.argtypes = [vp, rt_materials, i32, C.POINTER(rt_tx), vp, i32,
                                       C.POINTER(rt_plane), C.POINTER(rt_sbr_params), vp, vp, vp, vp]
    L.rt_tune.restype = C.c_int
    L.rt_tune.argtypes = [vp, rt_materials, C.POINTER(rt_tx), C.POINTER(rt_plane), C.POINTER(rt_sbr_params),
                          i64, vp, vp, C.POINTER(i32), C.POINTER(i32)]
    L.rt_set_launch_config.restype = C.c_int
    L.rt_set_launch_config.argtypes = [vp, i32, i32, i32, i32, i32]
    L.rt_scene_export.restype = C.c_int
    L.rt_scene_export.argtypes = [vp, vp, vp, vp, vp, C.POINTER(i64), vp]
    _lib = L
    return L


def _check(status):
    if status != RT_OK:
        raise RtError(status, lib().rt_last_error().decode(errors="replace"))


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _validate(t, name="tensor", dtype=None, numel=None):
    """Check a tensor's type, dtype and that it holds at least ``numel``
    elements (the kernels read or write that many; a smaller buffer would be
    overrun on the device)."""
    if t is None:
        return
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s: expected a torch tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s: expected dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s: needs at least %d elements, got %d" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s: expected a contiguous tensor" % name)


def _ptr(t, name="tensor", dtype=None, numel=None):
    """Device pointer of a checked contiguous device tensor (None for None)."""
    if t is None:
        return None
    _validate(t, name, dtype, numel)
    if not t.is_cuda:
        raise ValueError("%s: expected a device tensor" % name)
    return C.c_void_p(t.data_ptr())


def _ptrs(*specs):
    """Pointers of several (tensor, name, dtype, numel) specs: every dtype and
    size is checked before any device check, so the first error names the
    first wrong tensor."""
    for sp in specs:
        _validate(*sp)
    return [_ptr(*sp) for sp in specs]


def _f32spec(t, name, numel):
    import torch
    return (t, name, torch.float32, numel)


# ----------------------------------------------------------------- structs
def device_array(arr):
    """Device copies of a synthetic transmit array (float64 offsets [n][3],
    float32 (re, im) weights [n][2]), made once and kept on the array object."""
    dev = getattr(arr, "_rt_device", None)
    if dev is None:
        import numpy as np
        import torch
        pos = np.ascontiguousarray(arr.positions, dtype=np.float64).reshape(-1, 3)
        u = np.asarray(arr.precoding).astype(np.complex64).reshape(-1)
        if u.shape[0] != pos.shape[0]:
            raise ValueError("one precoding weight per array element")
        w = np.ascontiguousarray(np.stack([u.real, u.imag], axis=1).astype(np.float32))
        dev = (torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda())
        arr._rt_device = dev
    return dev


def make_tx(tx) -> rt_tx:
    t = rt_tx()
    t.pos[:] = [float(v) for v in tx.pos]
    t.yaw, t.pitch, t.roll = float(tx.yaw), float(tx.pitch), float(tx.roll)
    t.pattern, t.pattern_q, t.pol = int(tx.pattern), float(tx.pattern_q), int(tx.pol)
    arr = getattr(tx, "array", None)
    if arr is not None:
        pos, w = device_array(arr)
        t.n_ant = int(pos.shape[0])
        t.ant_pos, t.precoding = pos.data_ptr(), w.data_ptr()
        t._keep = (pos, w)
    return t


def make_plane(p) -> rt_plane:
    return rt_plane(float(p.z), float(p.x0), float(p.y0), float(p.dx), float(p.dy), int(p.W), int(p.H))


def make_params(p, *, ray_begin=None, ray_end=None, accumulate=0, accel=RT_ACCEL_BVH,
                deposit=RT_DEPOSIT_AUTO, block_size=0) -> rt_sbr_params:
    rb = int(p.ray_begin if ray_begin is None else ray_begin)
    re_ = ray_end if ray_end is not None else getattr(p, "ray_end", None)
    re_ = 0 if re_ is None else int(re_)
    return rt_sbr_params(float(p.freq_hz), int(p.n_rays), rb, re_, int(p.max_depth), int(accumulate),
                         float(p.t_min), int(accel), int(deposit), int(block_size),
                         int(getattr(p, "rr_depth", 1)), float(getattr(p, "rr_p_max", 0.0)),
                         float(getattr(p, "gain_threshold", 0.0)), int(getattr(p, "seed", 0)) & 0xffffffff,
                         int(getattr(p, "refraction", 0)))


# ------------------------------------------------------------------ scene
class RtScene:
    """Owner of an rt_scene* (device-resident triangles + LBVH)."""

    def __init__(self, handle, n_materials):
        self.handle = handle
        self.n_materials = n_materials
        self._pid = os.getpid()

    def info(self) -> rt_scene_info:
        out = rt_scene_info()
        _check(lib().rt_scene_info_get(self.handle, C.byref(out)))
        return out

    def export(self, stream=None):
        """Host copies of the acceleration structure (rt_scene_export):
        morton uint64 [n_tri], nodes float32 [n_tri - 1][16] (binary tree),
        wide float32 [n_wide][32] (4-wide tree, empty if none) and tris
        float32 [n_tri][12] in slot order."""
        import numpy as np
        L = lib()
        n_wide = C.c_int64(0)
        _check(L.rt_scene_export(self.handle, None, None, None, None, C.byref(n_wide), _stream(stream)))
        info = self.info()
        n = int(info.n_triangles)
        morton = np.zeros(n, np.uint64)
        nodes = np.zeros((max(0, n - 1), 16), np.float32)
        wide = np.zeros((int(n_wide.value), 32), np.float32)
        tris = np.zeros((n, 12), np.float32)
        _check(L.rt_scene_export(self.handle, morton.ctypes.data, nodes.ctypes.data, wide.ctypes.data,
                                 tris.ctypes.data, C.byref(n_wide), _stream(stream)))
        return {"morton": morton, "nodes": nodes, "wide": wide, "tris": tris}

    def close(self):
        # a process forked from the owner (a host worker pool) must not call
        # into HIP: there the handle is only dropped, the owner frees it
        if self.handle and os.getpid() == self._pid:
            lib().rt_scene_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rt_build_scene(vertices, triangles, tri_material, n_materials, stream=None) -> RtScene:
    """vertices f32 [n_v,3], triangles i32 [n_t,3], tri_material i32 [n_t] (device tensors)."""
    import torch
    n_v, n_t = int(vertices.shape[0]), int(triangles.shape[0])
    pv, pf, pm = _ptrs((vertices, "vertices", torch.float32, 3 * n_v), (triangles, "triangles", torch.int32, 3 * n_t),
                       (tri_material, "tri_material", torch.int32, n_t))
    h = C.c_void_p()
    _check(lib().rt_build_scene(pv, n_v, pf, n_t, pm, int(n_materials), _stream(stream), C.byref(h)))
    return RtScene(h, int(n_materials))


def scene_from_mesh(scene, device="cuda") -> RtScene:
    """Upload a mesh object (vertices, triangles, tri_material, eps_r) and build it."""
    import torch
    V = torch.as_tensor(scene.vertices, dtype=torch.float32).contiguous().to(device)
    F = torch.as_tensor(scene.triangles, dtype=torch.int32).contiguous().to(device)
    M = torch.as_tensor(scene.tri_material, dtype=torch.int32).contiguous().to(device)
    if F.shape[0] == 0:
        V = torch.zeros((1, 3), dtype=torch.float32, device=device)
    return rt_build_scene(V, F, M, len(scene.eps_r))


def _material_specs(eps_r, sigma, thickness=None, scattering=None, xpd=None, scatter_pattern=None,
                    n_materials=None, n_samples=1):
    nm = None if n_materials is None else int(n_materials)
    ns = None if nm is None else nm * int(n_samples)
    p4 = None if nm is None else 4 * nm
    return [_f32spec(eps_r, "eps_r", ns), _f32spec(sigma, "sigma", ns), _f32spec(thickness, "thickness", nm),
            _f32spec(scattering, "scattering", nm), _f32spec(xpd, "xpd", nm),
            _f32spec(scatter_pattern, "scatter_pattern", p4)]


def materials(eps_r, sigma, thickness=None, scattering=None, xpd=None, scatter_pattern=None, *,
              n_materials=None, n_samples=1) -> rt_materials:
    """Material descriptor.  With ``n_materials`` every array is checked to be
    float32 and long enough: eps_r and sigma [n_samples][n_materials], the
    optional per-material arrays [n_materials], scatter_pattern [n_materials][4]."""
    return rt_materials(*_ptrs(*_material_specs(eps_r, sigma, thickness, scattering, xpd, scatter_pattern,
                                                n_materials, n_samples)))


def _npol(tx):
    return 2 if int(tx.pol) == RT_POL_DUAL else 1


def _range_rays(p):
    b = int(p.ray_begin)
    e = int(p.ray_end) if int(p.ray_end) > 0 else int(p.n_rays)
    return max(0, e - b)


# ----------------------------------------------------------------- forward
def rt_radio_map(scene: RtScene, eps_r, sigma, tx, plane, params, out_map, *, tape=None, hits=None,
                 cells=None, weights=None, stats=None, stream=None, thickness=None, scattering=None, xpd=None,
                 scatter_pattern=None, **pkw):
    """Queue the SBR radio map into ``out_map`` (device f32 [H][W] or [2][H][W]).

    ``thickness`` (device f32 [n_mat], metres) selects slab walls; with
    ``params.refraction`` every hit samples reflection or transmission;
    ``scattering`` and ``xpd`` (device f32 [n_mat]) enable diffuse
    reflection, Lambertian unless ``scatter_pattern`` (device f32 [n_mat][4])
    selects directive or backscattering lobes."""
    import torch
    p = params if isinstance(params, rt_sbr_params) else make_params(params, **pkw)
    pl = plane if isinstance(plane, rt_plane) else make_plane(plane)
    nrec = _range_rays(p) * (int(p.max_depth) + 1)
    ptr = _ptrs(*_material_specs(eps_r, sigma, thickness, scattering, xpd, scatter_pattern, scene.n_materials),
                _f32spec(out_map, "out_map", _npol(tx) * int(pl.W) * int(pl.H)),
                (hits, "hits", torch.int32, nrec), (cells, "cells", torch.int32, nrec),
                _f32spec(weights, "weights", nrec), (stats, "stats", torch.int64, 5))
    mats, pmap, rec = rt_materials(*ptr[:6]), ptr[6], rt_records(*ptr[7:])
    t = tx if isinstance(tx, rt_tx) else make_tx(tx)
    _check(lib().rt_radio_map(scene.handle, mats, C.byref(t), C.byref(pl), C.byref(p), pmap,
                              tape.handle if tape is not None else None, C.byref(rec), _stream(stream)))
    return out_map


class RtTape:
    """Owner of an rt_tape* (device-resident forward records)."""

    def __init__(self, handle, nbytes):
        self.handle = handle
        self.nbytes = nbytes
        self._pid = os.getpid()

    def close(self):
        # as RtScene.close: only the creating process frees the tape
        if self.handle and os.getpid() == self._pid:
            lib().rt_tape_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rt_tape_create(params, **pkw) -> RtTape:
    p = params if isinstance(params, rt_sbr_params) else make_params(params, **pkw)
    h = C.c_void_p()
    _check(lib().rt_tape_create(C.byref(p), C.byref(h)))
    return RtTape(h, int(lib().rt_tape_bytes(C.byref(p))))


def rt_radio_map_backward(scene: RtScene, eps_r, sigma, tx, plane, params, tape: RtTape, grad_map,
                          grad_eps_r=None, grad_sigma=None, grad_orient=None, stream=None, thickness=None,
                          scattering=None, xpd=None, scatter_pattern=None, noalloc=False, **pkw):
    """Adjoint of a forward call recorded on ``tape`` (same materials,
    thickness, scattering, transmitter, plane and parameters).  With
    ``noalloc`` it calls rt_radio_map_backward_noalloc (partial sums in the
    GPU's static workspace; nothing is allocated)."""
    p = params if isinstance(params, rt_sbr_params) else make_params(params, **pkw)
    pl = plane if isinstance(plane, rt_plane) else make_plane(plane)
    nm = scene.n_materials
    ptr = _ptrs(*_material_specs(eps_r, sigma, thickness, scattering, xpd, scatter_pattern, nm),
                _f32spec(grad_map, "grad_map", _npol(tx) * int(pl.W) * int(pl.H)),
                _f32spec(grad_eps_r, "grad_eps_r", nm), _f32spec(grad_sigma, "grad_sigma", nm),
                _f32spec(grad_orient, "grad_orient", 3))
    t = tx if isinstance(tx, rt_tx) else make_tx(tx)
    fn = lib().rt_radio_map_backward_noalloc if noalloc else lib().rt_radio_map_backward
    _check(fn(scene.handle, rt_materials(*ptr[:6]), C.byref(t), C.byref(pl), C.byref(p),
              tape.handle, *ptr[6:], _stream(stream)))


def rt_radio_map_batched(scene: RtScene, eps_r, sigma, txs: Sequence, rays_per_tx: Sequence[int], plane, params,
                         out_maps, grad_maps=None, grads=None, stream=None, thickness=None, scattering=None, xpd=None,
                         scatter_pattern=None, **pkw):
    """eps_r/sigma: device f32 [S][n_mat]; out_maps [T][S][H][W]; grads [T][S][2 n_mat + 3].

    With one material set (S = 1) and no gradients the transmitters may carry
    arrays, and ``thickness``, ``scattering``/``xpd``/``scatter_pattern`` and
    the early-termination and refraction fields of ``params`` apply as in
    ``rt_radio_map``."""
    n_tx = len(txs)
    if len(rays_per_tx) != n_tx:
        raise ValueError("rays_per_tx: one budget per transmitter")
    p = params if isinstance(params, rt_sbr_params) else make_params(params, **pkw)
    pl = plane if isinstance(plane, rt_plane) else make_plane(plane)
    S = int(eps_r.shape[0]) if eps_r.dim() == 2 else 1
    nm = scene.n_materials
    nmap = n_tx * S * int(pl.W) * int(pl.H)
    ptr = _ptrs(*_material_specs(eps_r, sigma, thickness, scattering, xpd, scatter_pattern, nm, S),
                _f32spec(out_maps, "out_maps", nmap), _f32spec(grad_maps, "grad_maps", nmap),
                _f32spec(grads, "grads", n_tx * S * (2 * nm + 3)))
    mats, ptrs = rt_materials(*ptr[:6]), ptr[6:]
    # the descriptors keep the transmit-array tensors alive for the call
    descs = [tx if isinstance(tx, rt_tx) else make_tx(tx) for tx in txs]
    arr = (rt_tx * n_tx)(*descs)
    budgets = (C.c_int64 * n_tx)(*[int(b) for b in rays_per_tx])
    _check(lib().rt_radio_map_batched(scene.handle, mats, S, arr, C.cast(budgets, C.c_void_p),
                                      n_tx, C.byref(pl), C.byref(p), *ptrs, _stream(stream)))
    del descs
    return out_maps


def rt_tune(scene: RtScene, eps_r, sigma, tx, plane, params, n_probe_rays, scratch_map, stream=None, **pkw):
    p = params if isinstance(params, rt_sbr_params) else make_params(params, **pkw)
    pl = plane if isinstance(plane, rt_plane) else make_plane(plane)
    ptr = _ptrs(*_material_specs(eps_r, sigma, n_materials=scene.n_materials),
                _f32spec(scratch_map, "scratch_map", _npol(tx) * int(pl.W) * int(pl.H)))
    mats, pmap = rt_materials(*ptr[:6]), ptr[6]
    t = tx if isinstance(tx, rt_tx) else make_tx(tx)
    b, d = C.c_int32(), C.c_int32()
    _check(lib().rt_tune(scene.handle, mats, C.byref(t), C.byref(pl), C.byref(p),
                         int(n_probe_rays), pmap, _stream(stream), C.byref(b), C.byref(d)))
    return b.value, d.value


def rt_set_launch_config(scene: RtScene, width=0, order=0, block=0, deposit=0, refill=0):
    """Apply a launch configuration (as reported by RtScene.info() after rt_tune)."""
    _check(lib().rt_set_launch_config(scene.handle, int(width), int(order), int(block), int(deposit), int(refill)))
