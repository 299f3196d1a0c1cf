"""Host-side checks of the C ABI (no GPU needed).

* librtmap.so loads and exports every function include/rt.h declares;
* the ctypes structs match the header's field lists;
* argument validation rejects bad inputs on the host, before any device
  work: these calls never reach the device (the scene pointer is an opaque
  dummy that the library does not dereference before validation fails).
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rt_status|const char\*|size_t)\s+(rt_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2504_21719_amd as rt
    L = rt.lib()
    decl = _declared_functions()
    assert len(decl) >= 10, decl
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(rt.EXPORTED) == decl


def _struct_fields(name):
    txt = open(HEADER).read()
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r";", txt)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for f in decl.split(","):
            f = re.sub(r"\[.*?\]", "", f)
            fields.append(re.findall(r"\w+", f)[-1])
    return fields


@pytest.mark.parametrize("cls,name", [("rt_tx", "rt_tx"), ("rt_plane", "rt_plane"), ("rt_sbr_params", "rt_sbr_params"),
                                      ("rt_records", "rt_records"), ("rt_materials", "rt_materials"),
                                      ("rt_scene_info", "rt_scene_info")])
def test_struct_layouts_match_header(cls, name):
    import paper_2504_21719_amd as rt
    py = [f[0] for f in getattr(rt, cls)._fields_]
    assert py == _struct_fields(name)


def _params(**kw):
    import paper_2504_21719_amd as rt
    p = rt.rt_sbr_params(3.5e9, 1000, 0, 0, 3, 0, 1e-4, 0, 0, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [dict(n_rays=0), dict(max_depth=-1), dict(max_depth=65), dict(freq_hz=0.0),
                                 dict(ray_begin=5, ray_end=3), dict(ray_end=2000), dict(accel=4), dict(deposit=7),
                                 dict(block_size=100), dict(accumulate=2), dict(t_min=-1.0), dict(refraction=2),
                                 dict(refraction=1)])
def test_invalid_params_rejected_on_host(bad):
    import paper_2504_21719_amd as rt
    L = rt.lib()
    dummy = C.create_string_buffer(64)            # never dereferenced: validation fails first
    out = C.create_string_buffer(64)
    tx = rt.rt_tx()
    tx.pos[:] = [0.0, 0.0, 10.0]
    pl = rt.rt_plane(1.5, 0, 0, 1, 1, 10, 10)
    m = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p))
    p = _params(**bad)
    st = L.rt_radio_map(C.cast(dummy, C.c_void_p), m, C.byref(tx), C.byref(pl), C.byref(p), C.cast(out, C.c_void_p),
                        None, None, None)
    assert st == rt.RT_EINVAL
    assert L.rt_last_error().decode()


@pytest.mark.parametrize("field,val", [("pattern", 5), ("pol", 3), ("pattern_q", -1.0), ("yaw", float("nan")),
                                       ("n_ant", -1), ("n_ant", 3), ("n_ant", 70000)])
def test_invalid_tx_rejected_on_host(field, val):
    import paper_2504_21719_amd as rt
    L = rt.lib()
    dummy = C.create_string_buffer(64)
    out = C.create_string_buffer(64)
    tx = rt.rt_tx()
    tx.pos[:] = [0.0, 0.0, 10.0]
    setattr(tx, field, val)
    pl = rt.rt_plane(1.5, 0, 0, 1, 1, 10, 10)
    m = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p))
    st = L.rt_radio_map(C.cast(dummy, C.c_void_p), m, C.byref(tx), C.byref(pl), C.byref(_params()),
                        C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL


@pytest.mark.parametrize("plane", [(1.5, 0, 0, 0.0, 1, 10, 10), (1.5, 0, 0, 1, 1, 0, 10), (float("inf"), 0, 0, 1, 1, 4, 4)])
def test_invalid_plane_rejected_on_host(plane):
    import paper_2504_21719_amd as rt
    L = rt.lib()
    dummy = C.create_string_buffer(64)
    out = C.create_string_buffer(64)
    tx = rt.rt_tx()
    pl = rt.rt_plane(*plane)
    m = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p))
    st = L.rt_radio_map(C.cast(dummy, C.c_void_p), m, C.byref(tx), C.byref(pl), C.byref(_params()),
                        C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL


def test_null_arguments_rejected():
    import paper_2504_21719_amd as rt
    L = rt.lib()
    tx = rt.rt_tx()
    pl = rt.rt_plane(1.5, 0, 0, 1, 1, 10, 10)
    m = rt.rt_materials(None, None)
    st = L.rt_radio_map(None, m, C.byref(tx), C.byref(pl), C.byref(_params()), None, None, None, None)
    assert st == rt.RT_EINVAL and "scene" in L.rt_last_error().decode()
    h = C.c_void_p()
    assert L.rt_build_scene(None, -1, None, 0, None, 1, None, C.byref(h)) == rt.RT_EINVAL
    assert L.rt_build_scene(None, 3, None, 5, None, 1, None, C.byref(h)) == rt.RT_EINVAL
    assert L.rt_build_scene(None, 0, None, 0, None, 0, None, C.byref(h)) == rt.RT_EINVAL
    assert L.rt_scene_destroy(None) == rt.RT_OK
    assert L.rt_set_launch_config(None, 4, 1, 256, 2, 48) == rt.RT_EINVAL
    assert L.rt_tape_destroy(None) == rt.RT_OK
    assert L.rt_tape_bytes(C.byref(_params(n_rays=0))) == 0
    assert L.rt_tape_bytes(C.byref(_params(n_rays=100, max_depth=3))) == 100 * 4 * 64 + 100 * 4


@pytest.mark.parametrize("name", ["rt_radio_map_backward", "rt_radio_map_backward_noalloc"])
def test_backward_null_arguments_rejected(name):
    # both backward entry points validate on the host before touching a device
    import paper_2504_21719_amd as rt
    L = rt.lib()
    fn = getattr(L, name)
    dummy = C.create_string_buffer(64)
    out = C.create_string_buffer(64)
    tx = rt.rt_tx()
    tx.pos[:] = [0.0, 0.0, 10.0]
    pl = rt.rt_plane(1.5, 0, 0, 1, 1, 10, 10)
    m = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p))
    o = C.cast(out, C.c_void_p)
    d = C.cast(dummy, C.c_void_p)
    assert fn(None, m, C.byref(tx), C.byref(pl), C.byref(_params()), d, o, o, o, o, None) == rt.RT_EINVAL
    assert "scene" in L.rt_last_error().decode()
    assert fn(d, m, C.byref(tx), C.byref(pl), C.byref(_params()), None, o, o, o, o, None) == rt.RT_EINVAL
    assert "tape" in L.rt_last_error().decode()
    assert fn(d, m, C.byref(tx), C.byref(pl), C.byref(_params()), d, None, o, o, o, None) == rt.RT_EINVAL
    assert fn(d, m, C.byref(tx), C.byref(pl), C.byref(_params(max_depth=-1)), d, o, o, o, o, None) == rt.RT_EINVAL


def test_batched_argument_checks():
    import paper_2504_21719_amd as rt
    L = rt.lib()
    dummy = C.create_string_buffer(64)
    out = C.create_string_buffer(64)
    m = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p))
    txs = (rt.rt_tx * 2)()
    budgets = (C.c_int64 * 2)(10, 0)
    pl = rt.rt_plane(1.5, 0, 0, 1, 1, 10, 10)
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 1, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(_params()), C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL        # zero budget
    budgets[1] = 10
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 0, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(_params()), C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL        # no samples
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 1, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(_params()), C.cast(out, C.c_void_p), C.cast(out, C.c_void_p), None, None)
    assert st == rt.RT_EINVAL        # grad_maps without grads
    txs[0].pol = 2
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 1, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(_params()), C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL        # dual pol not allowed here
    txs[0].pol = 0
    ms = rt.rt_materials(C.cast(out, C.c_void_p), C.cast(out, C.c_void_p), None, C.cast(out, C.c_void_p),
                         C.cast(out, C.c_void_p))
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), ms, 2, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(_params()), C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EUNSUPPORTED  # diffuse reflection changes paths: one material sample only
    pr = _params()
    pr.refraction = 1
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 1, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(pr), C.cast(out, C.c_void_p), None, None, None)
    assert st == rt.RT_EINVAL        # refraction without a thickness
    pr.rr_p_max = 0.5
    pr.refraction = 0
    st = L.rt_radio_map_batched(C.cast(dummy, C.c_void_p), m, 1, txs, C.cast(budgets, C.c_void_p), 2, C.byref(pl),
                                C.byref(pr), C.cast(out, C.c_void_p), C.cast(out, C.c_void_p),
                                C.cast(out, C.c_void_p), None)
    assert st == rt.RT_EUNSUPPORTED  # Russian roulette changes paths: no batched gradients


def test_binding_refuses_host_tensors():
    import torch
    import paper_2504_21719_amd as rt
    with pytest.raises(ValueError):
        rt._ptr(torch.zeros(3))


def test_scene_generators_are_deterministic():
    import scenegen as sg
    a = sg.manhattan_scene()
    b = sg.manhattan_scene()
    assert a.sha256() == b.sha256()
    assert a.n_triangles == 1202 and sg.tiny_scene().n_triangles == 14
    assert set(a.tri_material.tolist()) == {0, 1}
