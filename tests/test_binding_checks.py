"""Host-side argument checks of the Python binding (no GPU needed).

The binding passes raw device pointers to kernels that read or write a fixed
number of elements (the map of every polarisation, per-material arrays, the
batched maps and gradients).  A tensor of the wrong dtype or one that is too
short must be refused before the C call, otherwise the kernels would read or
write past its end.  Every case below uses host tensors: a correctly sized
host tensor gets as far as the device check, so the size and dtype checks are
seen to come first.
"""
import ctypes as C

import pytest

torch = pytest.importorskip("torch")

import paper_2504_21719_amd as rt  # noqa: E402
import scenegen as sg  # noqa: E402


class _FakeScene:
    """Stands in for an RtScene: the checks raise before the handle is used."""
    handle = None
    n_materials = 2


H, W = 4, 5
PLANE = sg.Plane(1.5, 0.0, 0.0, 1.0, 1.0, W, H)
PARAMS = sg.Params(3.5e9, 100, 3)


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def _fwd(tx=None, **kw):
    args = dict(eps_r=f32(2), sigma=f32(2), out_map=f32(1, H, W))
    args.update(kw)
    rt.rt_radio_map(_FakeScene(), args.pop("eps_r"), args.pop("sigma"), tx or sg.Tx((0.0, 0.0, 10.0)), PLANE,
                    PARAMS, args.pop("out_map"), **args)


def test_forward_well_sized_host_tensors_reach_the_device_check():
    with pytest.raises(ValueError, match="device tensor"):
        _fwd()


@pytest.mark.parametrize("kw,what", [
    (dict(eps_r=torch.zeros(2, dtype=torch.float64)), "eps_r: expected dtype"),
    (dict(eps_r=f32(1)), "eps_r: needs at least 2"),
    (dict(sigma=f32(1)), "sigma: needs at least 2"),
    (dict(out_map=f32(H * W - 1)), "out_map: needs at least"),
    (dict(out_map=torch.zeros((1, H, W), dtype=torch.float16)), "out_map: expected dtype"),
    (dict(thickness=f32(1)), "thickness: needs at least 2"),
    (dict(scattering=f32(1), xpd=f32(2)), "scattering: needs at least 2"),
    (dict(scattering=f32(2), xpd=f32(2), scatter_pattern=f32(7)), "scatter_pattern: needs at least 8"),
    (dict(hits=torch.zeros((100, 4), dtype=torch.int64)), "hits: expected dtype"),
    (dict(cells=torch.zeros((99, 4), dtype=torch.int32)), "cells: needs at least 400"),
    (dict(weights=f32(100, 3)), "weights: needs at least 400"),
    (dict(stats=torch.zeros(4, dtype=torch.int64)), "stats: needs at least 5"),
])
def test_forward_rejects_bad_tensors(kw, what):
    with pytest.raises(ValueError, match=what):
        _fwd(**kw)


def test_forward_dual_pol_needs_two_maps():
    with pytest.raises(ValueError, match="out_map: needs at least %d" % (2 * H * W)):
        _fwd(tx=sg.Tx((0.0, 0.0, 10.0), pol=sg.POL_DUAL))


def test_forward_records_follow_the_ray_range():
    # 10 rays of depth 3 need 40 entries, whatever the lattice size
    with pytest.raises(ValueError, match="hits: needs at least 40"):
        rt.rt_radio_map(_FakeScene(), f32(2), f32(2), sg.Tx((0.0, 0.0, 10.0)), PLANE, PARAMS, f32(1, H, W),
                        hits=torch.zeros(39, dtype=torch.int32), ray_begin=50, ray_end=60)


@pytest.mark.parametrize("kw,what", [
    (dict(grad_map=f32(H * W - 1)), "grad_map: needs at least"),
    (dict(grad_eps_r=f32(1)), "grad_eps_r: needs at least 2"),
    (dict(grad_sigma=torch.zeros(2, dtype=torch.float64)), "grad_sigma: expected dtype"),
    (dict(grad_orient=f32(2)), "grad_orient: needs at least 3"),
    (dict(eps_r=f32(1)), "eps_r: needs at least 2"),
])
def test_backward_rejects_bad_tensors(kw, what):
    args = dict(eps_r=f32(2), sigma=f32(2), grad_map=f32(1, H, W), grad_eps_r=f32(2), grad_sigma=f32(2),
                grad_orient=f32(3))
    args.update(kw)
    with pytest.raises(ValueError, match=what):
        rt.rt_radio_map_backward(_FakeScene(), args.pop("eps_r"), args.pop("sigma"), sg.Tx((0.0, 0.0, 10.0)),
                                 PLANE, PARAMS, None, args.pop("grad_map"), **args)


@pytest.mark.parametrize("kw,what", [
    (dict(out_maps=f32(2, 3, H, W - 1)), "out_maps: needs at least %d" % (2 * 3 * H * W)),
    (dict(eps_r=f32(3, 1), sigma=f32(3, 1)), "eps_r: needs at least 6"),
    (dict(grad_maps=f32(2, 3, H, W), grads=f32(2, 3, 6)), "grads: needs at least 42"),
    (dict(grad_maps=f32(2, 2, H, W), grads=f32(2, 3, 7)), "grad_maps: needs at least"),
    (dict(rays_per_tx=[10]), "one budget per transmitter"),
])
def test_batched_rejects_bad_tensors(kw, what):
    args = dict(eps_r=f32(3, 2), sigma=f32(3, 2), out_maps=f32(2, 3, H, W), rays_per_tx=[10, 20])
    args.update(kw)
    txs = [sg.Tx((0.0, 0.0, 10.0)), sg.Tx((5.0, 0.0, 10.0))]
    with pytest.raises(ValueError, match=what):
        rt.rt_radio_map_batched(_FakeScene(), args.pop("eps_r"), args.pop("sigma"), txs, args.pop("rays_per_tx"),
                                PLANE, PARAMS, args.pop("out_maps"), **args)


def test_build_scene_rejects_bad_tensors():
    V = f32(3, 3)
    F = torch.zeros((1, 3), dtype=torch.int32)
    with pytest.raises(ValueError, match="triangles: expected dtype"):
        rt.rt_build_scene(V, F.to(torch.int64), torch.zeros(1, dtype=torch.int32), 1)
    with pytest.raises(ValueError, match="tri_material: needs at least 1"):
        rt.rt_build_scene(V, F, torch.zeros(0, dtype=torch.int32), 1)
    with pytest.raises(ValueError, match="vertices: expected dtype"):
        rt.rt_build_scene(V.double(), F, torch.zeros(1, dtype=torch.int32), 1)


def test_tune_rejects_short_scratch_map():
    with pytest.raises(ValueError, match="scratch_map: needs at least"):
        rt.rt_tune(_FakeScene(), f32(2), f32(2), sg.Tx((0.0, 0.0, 10.0)), PLANE, PARAMS, 1000, f32(H * W - 1))


class _StubLib:
    def __init__(self):
        self.calls = []

    def rt_scene_destroy(self, h):
        self.calls.append(("scene", h))

    def rt_tape_destroy(self, h):
        self.calls.append(("tape", h))


@pytest.mark.parametrize("cls,kind", [("RtScene", "scene"), ("RtTape", "tape")])
def test_handles_are_freed_only_by_their_creating_process(monkeypatch, cls, kind):
    # a host worker pool forks the process: a scene or tape object that is
    # garbage-collected in the child must not call into HIP (doing so crashed
    # the child); only the creating process frees the handle
    import os
    stub = _StubLib()
    monkeypatch.setattr(rt, "lib", lambda: stub)
    obj = getattr(rt, cls)(C.c_void_p(0x1234), 1)
    obj._pid = os.getpid() + 1           # as seen from a forked child
    obj.close()
    assert stub.calls == [] and obj.handle is None
    own = getattr(rt, cls)(C.c_void_p(0x5678), 1)
    own.close()
    assert [c[0] for c in stub.calls] == [kind] and own.handle is None
    own.close()                          # a second close does nothing
    assert len(stub.calls) == 1
