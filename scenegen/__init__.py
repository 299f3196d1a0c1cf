"""Seeded synthetic inputs for the SBR radio-map path.

This module is shared, as input data only, by the FP64 oracle (``oracle/``) and
by the HIP library (``paper_2504_21719_amd``).  It holds no part of the
method's arithmetic: it only builds triangle meshes, material tables,
transmitter poses, measurement planes and run parameters.

Scene model (Sec. "Scene Objects and Meshes"): a scene is a set of triangle
meshes; every triangle carries the index of one radio material, and a radio
material is a (relative permittivity, conductivity) pair (Sec. "Planar
Time-Harmonic Waves", eq. eta).  Vertices are stored as float32 so that the
oracle (which widens them exactly to double) and the GPU see the same geometry.

Workloads (sizes follow the five benchmark configurations of this project):
  * ``tiny``       - ground quad + one box building, 14 triangles
  * ``manhattan``  - 10x10 seeded city blocks, 1,202 triangles
  * ``large``      - fBm terrain + 2,000 subdivided buildings, ~1.0 M triangles
  * ``diff``       - the Manhattan scene with a directional, rotated transmitter
  * ``batch_tx``   - seeded rooftop transmitters with log-uniform ray budgets
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional

import numpy as np

# Material constants at 3.5 GHz used by the workloads (relative permittivity,
# conductivity in S/m).  Metal uses eps_r = 1 and sigma = 1e7 S/m.
CONCRETE = (5.24, 0.12)
GLASS = (6.31, 0.05)
METAL = (1.0, 1.0e7)
# Slab thickness per material (m) for finite-thickness walls: a 20 cm
# concrete wall, a 10 mm glass pane, a 5 mm metal sheet.  The paper prints
# none; these are round values of the usual construction.
THICKNESS = {CONCRETE: 0.2, GLASS: 0.01, METAL: 0.005}


def with_diffuse(scene: "Scene", scattering, xpd=None, pattern=None) -> "Scene":
    """Copy of ``scene`` with a scattering coefficient S (and a
    cross-polarisation share K_x, default 0, and a scattering pattern
    (kind, alpha_R, alpha_I, Lambda), default Lambertian) per material."""
    S = np.broadcast_to(np.asarray(scattering, dtype=np.float64), scene.eps_r.shape).copy()
    K = np.zeros_like(S) if xpd is None else np.broadcast_to(np.asarray(xpd, dtype=np.float64), S.shape).copy()
    P = None if pattern is None else np.broadcast_to(np.asarray(pattern, dtype=np.float64),
                                                     (S.shape[0], 4)).copy()
    return dataclasses.replace(scene, scattering=S, xpd=K, scatter_pattern=P)


def with_thickness(scene: "Scene", thickness=None) -> "Scene":
    """Copy of ``scene`` with slab thickness per material (default THICKNESS
    looked up by (eps_r, sigma))."""
    if thickness is None:
        thickness = [THICKNESS[(float(e), float(s))] for e, s in zip(scene.eps_r, scene.sigma)]
    return dataclasses.replace(scene, thickness=np.asarray(thickness, dtype=np.float64))

PATTERN_ISO = 0          # isotropic, G = 1
PATTERN_DIRECTIONAL = 1  # G(alpha) = (q+1) ((1+cos alpha)/2)^q about local +x
POL_V, POL_H, POL_DUAL = 0, 1, 2


@dataclasses.dataclass
class Scene:
    vertices: np.ndarray          # float32 [n_v, 3], metres
    triangles: np.ndarray         # int32 [n_t, 3]
    tri_material: np.ndarray      # int32 [n_t]
    eps_r: np.ndarray             # float64 [n_mat]
    sigma: np.ndarray             # float64 [n_mat], S/m
    name: str = ""
    thickness: Optional[np.ndarray] = None   # float64 [n_mat] slab thickness (m); None = half-space
    scattering: Optional[np.ndarray] = None  # float64 [n_mat] scattering coefficient S; None = no diffuse
    xpd: Optional[np.ndarray] = None         # float64 [n_mat] cross-polarisation share K_x
    # float64 [n_mat][4] scattering pattern (kind, alpha_R, alpha_I, Lambda):
    # kind 0 Lambertian, 1 directive, 2 backscattering; None = Lambertian
    scatter_pattern: Optional[np.ndarray] = None

    @property
    def n_triangles(self) -> int:
        return int(self.triangles.shape[0])

    @property
    def n_materials(self) -> int:
        return int(self.eps_r.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.vertices, self.triangles, self.tri_material, self.eps_r, self.sigma):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class TxArray:
    """Synthetic transmit array: element offsets from the transmitter position
    (metres, global frame) and one complex precoding weight per element.  The
    weights are stored in float32 (the precision the library takes)."""
    positions: np.ndarray         # [n][3] float64
    precoding: np.ndarray         # [n] complex64


def linear_array(n: int, spacing: float, axis=(1.0, 0.0, 0.0), precoding=None) -> TxArray:
    """n elements spaced `spacing` metres along `axis`, centred on the
    transmitter; equal weights 1/sqrt(n) unless `precoding` is given."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    off = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * spacing
    u = np.full(n, 1.0 / math.sqrt(n), dtype=np.complex64) if precoding is None else np.asarray(precoding)
    return TxArray(off[:, None] * a[None, :], u.astype(np.complex64))


def random_array(n: int, extent: float, seed: int) -> TxArray:
    """n elements at seeded random offsets in a cube of side `extent` metres,
    with seeded random complex weights of unit total power."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5 * extent, 0.5 * extent, size=(n, 3))
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    u = u / np.linalg.norm(u)
    return TxArray(pos, u.astype(np.complex64))


@dataclasses.dataclass
class Tx:
    pos: tuple                    # metres
    yaw: float = 0.0              # radians
    pitch: float = 0.0
    roll: float = 0.0
    pattern: int = PATTERN_ISO
    pattern_q: float = 2.0
    pol: int = POL_V
    array: Optional[TxArray] = None


@dataclasses.dataclass
class Plane:
    z: float                      # horizontal measurement plane z = const
    x0: float
    y0: float
    dx: float
    dy: float
    W: int                        # cells along +x
    H: int                        # cells along +y


@dataclasses.dataclass
class Params:
    freq_hz: float
    n_rays: int                   # N_S, lattice size and estimator normaliser
    max_depth: int                # L
    ray_begin: int = 0
    ray_end: Optional[int] = None  # None -> n_rays
    t_min: float = 1e-4
    # early termination (both off by default): applied before tracing every
    # segment l >= rr_depth; Russian roulette with maximum keep probability
    # rr_p_max, gain thresholding below gain_threshold; draws seeded by seed
    rr_depth: int = 1
    rr_p_max: float = 0.0
    gain_threshold: float = 0.0
    seed: int = 0
    # 1: sample reflection or transmission at every hit (needs slab thickness)
    refraction: int = 0

    def end(self) -> int:
        return self.n_rays if self.ray_end is None else int(self.ray_end)


@dataclasses.dataclass
class Config:
    scene: Scene
    tx: Tx
    plane: Plane
    params: Params
    name: str = ""


# ----------------------------------------------------------------------------
# mesh helpers (pure geometry bookkeeping)
# ----------------------------------------------------------------------------
class _MeshBuilder:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.f: List[np.ndarray] = []
        self.m: List[np.ndarray] = []
        self.nv = 0

    def add(self, verts, faces, mat):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        faces = np.asarray(faces, dtype=np.int64).reshape(-1, 3) + self.nv
        self.v.append(verts)
        self.f.append(faces)
        self.m.append(np.full(faces.shape[0], mat, dtype=np.int32))
        self.nv += verts.shape[0]

    def quad(self, a, b, c, d, mat):
        """Quad a-b-c-d (in order around the boundary) as triangles (a,b,c), (a,c,d)."""
        self.add([a, b, c, d], [[0, 1, 2], [0, 2, 3]], mat)

    def grid_quad(self, origin, u, v, nu, nv, mat):
        """Planar quad origin + s*u + t*v, s,t in [0,1], subdivided nu x nv."""
        o = np.asarray(origin, np.float64)
        u = np.asarray(u, np.float64)
        v = np.asarray(v, np.float64)
        s = np.linspace(0.0, 1.0, nu + 1)
        t = np.linspace(0.0, 1.0, nv + 1)
        pts = o[None, None, :] + s[:, None, None] * u[None, None, :] + t[None, :, None] * v[None, None, :]
        pts = pts.reshape(-1, 3)
        idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
        a = idx[:-1, :-1].ravel()
        b = idx[1:, :-1].ravel()
        c = idx[1:, 1:].ravel()
        d = idx[:-1, 1:].ravel()
        faces = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
        self.add(pts, faces, mat)

    def box(self, lo, hi, mat, bottom=True):
        x0, y0, z0 = lo
        x1, y1, z1 = hi
        p = [(x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0),
             (x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)]
        quads = [(4, 5, 6, 7),  # top
                 (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
        if bottom:
            quads.append((0, 3, 2, 1))
        faces = []
        for a, b, c, d in quads:
            faces += [[a, b, c], [a, c, d]]
        self.add(p, faces, mat)

    def build(self, eps_sigma, name) -> Scene:
        V = np.concatenate(self.v, 0).astype(np.float32)
        F = np.concatenate(self.f, 0).astype(np.int32)
        M = np.concatenate(self.m, 0).astype(np.int32)
        eps = np.array([e for e, _ in eps_sigma], dtype=np.float64)
        sig = np.array([s for _, s in eps_sigma], dtype=np.float64)
        return Scene(V, F, M, eps, sig, name)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def ground_quad(half=100.0, mat_eps_sigma=CONCRETE) -> Scene:
    """Ground quad (+-half, +-half, 0), split along the (-h,-h)->(h,h) diagonal."""
    mb = _MeshBuilder()
    h = float(half)
    mb.quad((-h, -h, 0.0), (h, -h, 0.0), (h, h, 0.0), (-h, h, 0.0), 0)
    return mb.build([mat_eps_sigma], "ground")


def empty_scene() -> Scene:
    return Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32),
                 np.zeros((0,), np.int32), np.array([CONCRETE[0]]), np.array([CONCRETE[1]]), "empty")


def tiny_scene(bottom=True) -> Scene:
    """Ground quad 200x200 m at z=0 plus a 20x20x30 m box centred at (40, 0)
    (bottom=False: without the box's bottom face, which lies on the ground)."""
    mb = _MeshBuilder()
    mb.quad((-100.0, -100.0, 0.0), (100.0, -100.0, 0.0), (100.0, 100.0, 0.0), (-100.0, 100.0, 0.0), 0)
    mb.box((30.0, -10.0, 0.0), (50.0, 10.0, 30.0), 0, bottom=bottom)
    return mb.build([CONCRETE], "tiny")


def tiny_config(n_rays=100_000, max_depth=3) -> Config:
    return Config(tiny_scene(), Tx((0.0, 0.0, 10.0)),
                  Plane(1.5, -100.0, -100.0, 2.0, 2.0, 100, 100),
                  Params(3.5e9, n_rays, max_depth), "tiny")


def manhattan_scene(seed=2, bottoms=True) -> Scene:
    """10x10 blocks on a 100 m pitch over [-500,500]^2 with 20 m streets.

    Streets are centred on x, y = -500 + 100 i; one box per block, centred in
    the block, footprint U(20,60) m per side, height U(10,80) m, concrete or
    glass with p = 0.5.  Draws are row-major over (i, j): w_x, w_y, h, material.
    bottoms=False leaves out the bottom faces, which coincide with the ground
    (for transmitted rays, which can reach them).
    """
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    mb.quad((-500.0, -500.0, 0.0), (500.0, -500.0, 0.0), (500.0, 500.0, 0.0), (-500.0, 500.0, 0.0), 0)
    for i in range(10):
        for j in range(10):
            wx = rng.uniform(20.0, 60.0)
            wy = rng.uniform(20.0, 60.0)
            h = rng.uniform(10.0, 80.0)
            mat = int(rng.uniform() < 0.5)      # 0 concrete, 1 glass
            cx = -450.0 + 100.0 * i
            cy = -450.0 + 100.0 * j
            mb.box((cx - wx / 2, cy - wy / 2, 0.0), (cx + wx / 2, cy + wy / 2, h), mat, bottom=bottoms)
    return mb.build([CONCRETE, GLASS], "manhattan")


def manhattan_config(n_rays=10_000_000, max_depth=5) -> Config:
    return Config(manhattan_scene(), Tx((0.0, 0.0, 30.0)),
                  Plane(1.5, -500.0, -500.0, 1.0, 1.0, 1000, 1000),
                  Params(3.5e9, n_rays, max_depth), "manhattan")


def _value_noise_fbm(n, rng, octaves=8, lacunarity=2.0, gain=0.5):
    """Fractional Brownian motion of bilinear value noise on an n x n grid."""
    out = np.zeros((n, n), np.float64)
    amp = 1.0
    freq = 2.0
    u = np.linspace(0.0, 1.0, n)
    for _ in range(octaves):
        m = int(math.ceil(freq)) + 1
        lattice = rng.standard_normal((m + 1, m + 1))
        x = u * freq
        i0 = np.minimum(np.floor(x).astype(int), m - 1)
        fx = x - i0
        a = lattice[i0][:, i0]
        b = lattice[i0 + 1][:, i0]
        c = lattice[i0][:, i0 + 1]
        d = lattice[i0 + 1][:, i0 + 1]
        fxr = fx[:, None]
        fyc = fx[None, :]
        out += amp * ((a * (1 - fxr) + b * fxr) * (1 - fyc) + (c * (1 - fxr) + d * fxr) * fyc)
        amp *= gain
        freq *= lacunarity
    return out


def large_scene(seed=3, n_buildings=2000, terrain_n=513, half=1000.0,
                footprint=(10.0, 25.0), height=(8.0, 30.0), tile=4.0):
    """fBm terrain (513x513 vertices over [-1000,1000]^2) plus subdivided buildings.

    Returns (scene, terrain_height_fn, buildings) with buildings as
    (x0, y0, x1, y1, roof height) tuples.  Terrain heights are normalised to mean 0,
    std 5 m.  Buildings: centres uniform in [-950,950]^2 with non-overlap
    rejection (5 m gap, 60 m clearing around the origin); facades and roofs are
    subdivided into <= ``tile`` m quads; no bottom faces.  Footprint U(10,25) m
    and height U(8,30) m give 1,021,074 triangles for the default seed.  Materials: 0 concrete
    (terrain and buildings), 1 glass, 2 metal, drawn with p = 0.45/0.45/0.10.
    """
    rng = np.random.default_rng(seed)
    hgt = _value_noise_fbm(terrain_n, rng)
    hgt = (hgt - hgt.mean()) / hgt.std() * 5.0
    xs = np.linspace(-half, half, terrain_n)
    step = xs[1] - xs[0]

    def terrain(x, y):
        fx = (np.asarray(x, np.float64) + half) / step
        fy = (np.asarray(y, np.float64) + half) / step
        i = np.clip(np.floor(fx).astype(int), 0, terrain_n - 2)
        j = np.clip(np.floor(fy).astype(int), 0, terrain_n - 2)
        ax = fx - i
        ay = fy - j
        return ((hgt[i, j] * (1 - ax) + hgt[i + 1, j] * ax) * (1 - ay)
                + (hgt[i, j + 1] * (1 - ax) + hgt[i + 1, j + 1] * ax) * ay)

    mb = _MeshBuilder()
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), hgt.ravel()], 1)
    idx = np.arange(terrain_n * terrain_n).reshape(terrain_n, terrain_n)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    faces = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
    mb.add(verts, faces, 0)

    placed = []   # (x0, y0, x1, y1, roof height)
    tries = 0
    while len(placed) < n_buildings:
        tries += 1
        if tries > 200 * n_buildings:
            raise RuntimeError("building placement did not converge")
        cx, cy = rng.uniform(-950.0, 950.0, 2)
        wx, wy = rng.uniform(footprint[0], footprint[1], 2)
        h = rng.uniform(height[0], height[1])
        mat_u = rng.uniform()
        box = (cx - wx / 2, cy - wy / 2, cx + wx / 2, cy + wy / 2)
        # 60 m clearing around the transmitter at the origin
        nx = min(max(0.0, box[0]), box[2]) if not (box[0] <= 0.0 <= box[2]) else 0.0
        ny = min(max(0.0, box[1]), box[3]) if not (box[1] <= 0.0 <= box[3]) else 0.0
        if math.hypot(nx, ny) < 60.0:
            continue
        ok = True
        for (p0, q0, p1, q1, _) in placed:
            if box[0] < p1 + 5.0 and p0 < box[2] + 5.0 and box[1] < q1 + 5.0 and q0 < box[3] + 5.0:
                ok = False
                break
        if not ok:
            continue
        mat = 0 if mat_u < 0.45 else (1 if mat_u < 0.90 else 2)
        # base below the lowest terrain point under the footprint
        gx = np.linspace(box[0], box[2], 9)
        gy = np.linspace(box[1], box[3], 9)
        GX, GY = np.meshgrid(gx, gy, indexing="ij")
        base = float(terrain(GX, GY).min()) - 1.0
        top = base + h
        placed.append(box + (top,))
        nxq = max(1, int(math.ceil(wx / tile)))
        nyq = max(1, int(math.ceil(wy / tile)))
        nzq = max(1, int(math.ceil((top - base) / tile)))
        x0, y0, x1, y1 = box
        # facades (outward-facing winding is irrelevant: reflection is two-sided)
        mb.grid_quad((x0, y0, base), (x1 - x0, 0, 0), (0, 0, top - base), nxq, nzq, mat)
        mb.grid_quad((x1, y0, base), (0, y1 - y0, 0), (0, 0, top - base), nyq, nzq, mat)
        mb.grid_quad((x1, y1, base), (x0 - x1, 0, 0), (0, 0, top - base), nxq, nzq, mat)
        mb.grid_quad((x0, y1, base), (0, y0 - y1, 0), (0, 0, top - base), nyq, nzq, mat)
        mb.grid_quad((x0, y0, top), (x1 - x0, 0, 0), (0, y1 - y0, 0), nxq, nyq, mat)
    scene = mb.build([CONCRETE, GLASS, METAL], "large")
    return scene, terrain, placed


def large_config(n_rays=100_000_000, max_depth=8, seed=3):
    scene, terrain, _ = large_scene(seed)
    tz = float(terrain(0.0, 0.0)) + 40.0
    return Config(scene, Tx((0.0, 0.0, tz)),
                  Plane(1.5, -1000.0, -1000.0, 2.0, 2.0, 1000, 1000),
                  Params(3.5e9, n_rays, max_depth), "large")


def large_buildings(seed=3):
    """(x0, y0, x1, y1, roof height) of every building of the large scene."""
    return large_scene(seed)[2]


def diff_config(n_rays=1_000_000, max_depth=4) -> Config:
    """Manhattan scene, directional V-pol transmitter (q = 2) at yaw 30 deg, pitch -10 deg."""
    return Config(manhattan_scene(), Tx((0.0, 0.0, 30.0), yaw=math.radians(30.0),
                                        pitch=math.radians(-10.0), roll=0.0,
                                        pattern=PATTERN_DIRECTIONAL, pattern_q=2.0, pol=POL_V),
                  Plane(1.5, -500.0, -500.0, 1.0, 1.0, 1000, 1000),
                  Params(3.5e9, n_rays, max_depth), "diff")


def diff_target_params(scene: Scene, tx: Tx, seed=4):
    """Perturbed parameters for the differentiation target map.

    eps_r scaled by 1+U(-0.1,0.1), sigma by 1+U(-0.2,0.2), yaw/pitch shifted by
    U(-5,5) degrees.
    """
    rng = np.random.default_rng(seed)
    eps = scene.eps_r * (1.0 + rng.uniform(-0.1, 0.1, scene.n_materials))
    sig = scene.sigma * (1.0 + rng.uniform(-0.2, 0.2, scene.n_materials))
    dyaw, dpitch = np.radians(rng.uniform(-5.0, 5.0, 2))
    return eps, sig, tx.yaw + dyaw, tx.pitch + dpitch


def rooftop_transmitters(n_tx=64, seed=5, buildings=None, scene_kind="manhattan",
                         budget_lo=1e5, budget_hi=1e7):
    """Seeded rooftop transmitters (roof centre + 3 m) with log-uniform ray budgets.

    ``buildings`` is a list of (x0, y0, x1, y1, top_z); for the Manhattan scene
    it is derived from the mesh (every 12-triangle box after the ground quad).
    """
    rng = np.random.default_rng(seed)
    sel = rng.choice(len(buildings), size=n_tx, replace=False)
    budgets = np.round(10.0 ** rng.uniform(math.log10(budget_lo), math.log10(budget_hi), n_tx)).astype(np.int64)
    txs = []
    for b in sel:
        x0, y0, x1, y1, top = buildings[b]
        txs.append(Tx(((x0 + x1) / 2, (y0 + y1) / 2, top + 3.0)))
    return txs, budgets


def manhattan_buildings(scene: Scene):
    """(x0, y0, x1, y1, top) for each box of the Manhattan scene."""
    out = []
    V = scene.vertices.astype(np.float64)
    F = scene.triangles
    for b in range((scene.n_triangles - 2) // 12):
        tri = F[2 + 12 * b: 2 + 12 * (b + 1)]
        p = V[np.unique(tri.ravel())]
        out.append((p[:, 0].min(), p[:, 1].min(), p[:, 0].max(), p[:, 1].max(), p[:, 2].max()))
    return out


def random_materials(scene: Scene, n_samples=16, seed=5):
    """Material samples: eps_r ~ U(0.8,1.2) x nominal, sigma ~ U(0.5,2) x nominal."""
    rng = np.random.default_rng(seed)
    eps = scene.eps_r[None, :] * rng.uniform(0.8, 1.2, (n_samples, scene.n_materials))
    sig = scene.sigma[None, :] * rng.uniform(0.5, 2.0, (n_samples, scene.n_materials))
    return eps, sig


def random_soup(n_tri, seed=0, extent=50.0, size=5.0, n_mat=2):
    """Random triangle soup for structural tests of the acceleration structure."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-extent, extent, (n_tri, 1, 3))
    V = (c + rng.uniform(-size, size, (n_tri, 3, 3))).reshape(-1, 3).astype(np.float32)
    F = np.arange(3 * n_tri, dtype=np.int32).reshape(n_tri, 3)
    M = rng.integers(0, n_mat, n_tri).astype(np.int32)
    mats = [CONCRETE, GLASS, METAL][:n_mat]
    return Scene(V, F, M, np.array([e for e, _ in mats]), np.array([s for _, s in mats]), "soup")
