"""Seeded synthetic inputs for the tile-NeRF training step.

This module only draws random numbers and builds scenes, cameras and rays.
It holds none of the method's arithmetic (no sampling, no encoding, no MLP,
no compositing): both the CPU oracle and the HIP path receive exactly the
arrays produced here.

Workloads (all host-side, NumPy ``default_rng(seed)``, FP64 geometry):

* ``tiny_tile``  -- one unit NeRF tile, 3 affine satellite views, rays aimed
  at uniform ground points at z = 0.5 with origins at z = 2, uniform-random
  RGB targets, hash grid L=8/F=2/T=2^14 (16 -> 256), MLP 32->64->16 and
  18->64->3.
* ``full_tile``  -- one unit NeRF tile over a synthetic heightfield (32
  Gaussian bumps, value-noise albedo, hard sun shadows), 8 training views of
  1024^2 px, altitude band z in [0.2, 0.8], hash grid L=16/F=2/T=2^19
  (16 -> 2048), MLP 32->64->16 and 21->64->64->4.
* ``window_2x2`` -- four unit NeRF tiles [i,i+1]x[j,j+1]x[0,1] of a 2x2
  window, each with its own table and networks (small-tile shapes), rays
  drawn per tile from the crop of each of 8 views that holds the projected
  tile corners plus a 10 % margin, ragged per-ray sample budgets.

The satellite views are affine (orthographic): every ray of a view shares one
direction d = (sin th cos ph, sin th sin ph, -cos th) with off-nadir angle
th <= 30 deg, as for pushbroom imagery over a small footprint.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "GridConfig", "MlpConfig", "Workload", "tiny_tile", "full_tile", "window_2x2", "window_rays",
    "full_tile_heldout",
    "init_table", "init_mlp", "mlp_param_shapes", "Heightfield",
]


@dataclasses.dataclass(frozen=True)
class GridConfig:
    n_levels: int
    n_features: int
    log2_table: int
    res_min: int
    res_max: int
    out_width: int = 32

    @property
    def table_size(self) -> int:
        return 1 << self.log2_table


@dataclasses.dataclass(frozen=True)
class MlpConfig:
    feat_width: int = 32       # density-net input width (zero-padded features)
    feat_real: int = 16        # real (non-padding) feature width, for Xavier fan-in
    hidden: int = 64
    dens_out: int = 16         # sigma logit + 15-wide density embedding
    n_dir: int = 3             # 3: view dir; 6: view dir + sun dir
    colour_layers: int = 1     # hidden layers of the colour net
    colour_out: int = 3        # 3: rgb; 4: albedo rgb + sun visibility


def mlp_param_shapes(m: MlpConfig):
    """Row-major [out][in] weight shapes of the packed MLP parameter vector,
    in storage order: density L1, density L2, colour L1, [colour L2], colour out."""
    cin = m.dens_out - 1 + m.n_dir
    shapes = [(m.hidden, m.feat_width), (m.dens_out, m.hidden), (m.hidden, cin)]
    for _ in range(m.colour_layers - 1):
        shapes.append((m.hidden, m.hidden))
    shapes.append((m.colour_out, m.hidden))
    return shapes


def init_table(rng: np.random.Generator, g: GridConfig, n_tiles: int = 1) -> np.ndarray:
    """Hash-table entries U(-1e-4, 1e-4), float32, layout [K][L][T][F]."""
    shape = (n_tiles, g.n_levels, g.table_size, g.n_features)
    return rng.uniform(-1e-4, 1e-4, size=shape).astype(np.float32)


def init_mlp(rng: np.random.Generator, m: MlpConfig) -> np.ndarray:
    """Xavier-uniform weights, bound sqrt(6/(fan_in+fan_out)) with fan_in the
    real input width; padded input columns of the density net are zero."""
    out = []
    for li, (o, i) in enumerate(mlp_param_shapes(m)):
        fan_in = m.feat_real if li == 0 else i
        bound = math.sqrt(6.0 / (fan_in + o))
        w = np.zeros((o, i), dtype=np.float64)
        w[:, :fan_in] = rng.uniform(-bound, bound, size=(o, fan_in))
        out.append(w.astype(np.float32).ravel())
    return np.concatenate(out)


@dataclasses.dataclass
class Workload:
    name: str
    grid: GridConfig
    mlp: MlpConfig
    boxes: np.ndarray            # [K][6] float64: lo xyz, hi xyz
    zband: np.ndarray | None     # [2] float64 or None
    rays_o: np.ndarray           # [R][3] float64
    rays_d: np.ndarray           # [R][3] float64
    sun: np.ndarray | None       # [R][3] float32 unit sun direction (or None)
    target: np.ndarray           # [R][3] float32
    samples_per_ray: int
    early_stop: float            # transmittance threshold, 0 = off
    table: np.ndarray            # [K][L][T][F] float32
    mlp_params: np.ndarray       # [P] float32
    lr: float = 1e-2

    @property
    def n_rays(self) -> int:
        return int(self.rays_o.shape[0])


def _view_dirs(rng, n_views, max_off_nadir_deg):
    th = np.deg2rad(rng.uniform(0.0, max_off_nadir_deg, size=n_views))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_views)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)], axis=1)
    return d


def tiny_tile(seed: int = 0, n_rays: int = 4096, samples: int = 64) -> Workload:
    """Single unit tile, 3 affine views, uniform-random targets."""
    rng = np.random.default_rng(seed)
    grid = GridConfig(n_levels=8, n_features=2, log2_table=14, res_min=16, res_max=256)
    mlp = MlpConfig(feat_width=32, feat_real=16, hidden=64, dens_out=16, n_dir=3,
                    colour_layers=1, colour_out=3)
    dirs = _view_dirs(rng, 3, 30.0)
    view = np.arange(n_rays) % 3
    d = dirs[view]
    g = np.concatenate([rng.uniform(0.0, 1.0, size=(n_rays, 2)),
                        np.full((n_rays, 1), 0.5)], axis=1)
    s = (2.0 - 0.5) / (-d[:, 2])
    o = g - s[:, None] * d
    o[:, 2] = 2.0
    target = rng.uniform(0.0, 1.0, size=(n_rays, 3)).astype(np.float32)
    table = init_table(rng, grid)
    params = init_mlp(rng, mlp)
    boxes = np.array([[0.0, 0.0, 0.0, 1.0, 1.0, 1.0]])
    return Workload("tiny_tile", grid, mlp, boxes, None, o, d, None, target,
                    samples, 0.0, table, params)


# ---------------------------------------------------------------------------
# Heightfield scene for the full-size tile
# ---------------------------------------------------------------------------
class Heightfield:
    """z(x,y) = clip(0.35 + sum_k a_k exp(-|xy-c_k|^2 / (2 s_k^2)), 0.25, 0.75)
    with value-noise albedo in [0.1, 0.9]^3 and a hard-shadow sun term.
    Evaluated through a fine bilinear height grid so that rendering many rays
    stays cheap."""

    GRID = 1024
    LO, HI = -0.5, 1.5

    def __init__(self, rng: np.random.Generator):
        n = 32
        self.a = rng.uniform(0.02, 0.08, size=n)
        self.c = rng.uniform(0.0, 1.0, size=(n, 2))
        self.s = rng.uniform(0.03, 0.12, size=n)
        self.lattice = rng.uniform(0.1, 0.9, size=(9, 9, 3))
        ax = np.linspace(self.LO, self.HI, self.GRID + 1)
        X, Y = np.meshgrid(ax, ax, indexing="ij")
        self.hgrid = self.height_exact(X, Y)

    def height_exact(self, x, y):
        z = np.full(np.shape(x), 0.35)
        for a, c, s in zip(self.a, self.c, self.s):
            z = z + a * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2.0 * s * s))
        return np.clip(z, 0.25, 0.75)

    def height(self, x, y):
        f = (self.HI - self.LO) / self.GRID
        u = np.clip((x - self.LO) / f, 0.0, self.GRID - 1e-9)
        v = np.clip((y - self.LO) / f, 0.0, self.GRID - 1e-9)
        i = np.floor(u).astype(np.int64)
        j = np.floor(v).astype(np.int64)
        fu, fv = u - i, v - j
        h = self.hgrid
        return ((1 - fu) * (1 - fv) * h[i, j] + fu * (1 - fv) * h[i + 1, j]
                + (1 - fu) * fv * h[i, j + 1] + fu * fv * h[i + 1, j + 1])

    def albedo(self, x, y):
        u = np.mod(x, 1.0) * 8.0
        v = np.mod(y, 1.0) * 8.0
        i = np.floor(u).astype(np.int64)
        j = np.floor(v).astype(np.int64)
        fu, fv = u - i, v - j
        fu = fu * fu * (3 - 2 * fu)
        fv = fv * fv * (3 - 2 * fv)
        L = self.lattice
        return ((1 - fu)[:, None] * (1 - fv)[:, None] * L[i, j]
                + fu[:, None] * (1 - fv)[:, None] * L[i + 1, j]
                + (1 - fu)[:, None] * fv[:, None] * L[i, j + 1]
                + fu[:, None] * fv[:, None] * L[i + 1, j + 1])

    def render(self, o, d, sun):
        """Ground-truth colour: albedo x (1 if lit else 0.3); background black."""
        # march from the ray origin down to z = 0.2 (below every surface point)
        t_end = (o[:, 2] - 0.2) / (-d[:, 2])
        t_hit = np.full(o.shape[0], np.inf)
        n_steps = 192
        dt = t_end / n_steps
        alive = np.ones(o.shape[0], dtype=bool)
        for k in range(1, n_steps + 1):
            idx = np.nonzero(alive)[0]
            if idx.size == 0:
                break
            t = k * dt[idx]
            p = o[idx] + t[:, None] * d[idx]
            below = p[:, 2] <= self.height(p[:, 0], p[:, 1])
            hit = idx[below]
            if hit.size:
                lo = (k - 1) * dt[hit]
                hi = k * dt[hit]
                for _ in range(16):
                    mid = 0.5 * (lo + hi)
                    q = o[hit] + mid[:, None] * d[hit]
                    b = q[:, 2] <= self.height(q[:, 0], q[:, 1])
                    hi = np.where(b, mid, hi)
                    lo = np.where(b, lo, mid)
                t_hit[hit] = hi
                alive[hit] = False
        rgb = np.zeros((o.shape[0], 3))
        hit = np.isfinite(t_hit)
        if not hit.any():
            return rgb
        p = o[hit] + t_hit[hit][:, None] * d[hit]
        alb = self.albedo(p[:, 0], p[:, 1])
        # shadow ray toward the sun, from just above the surface up to z = 0.8
        s = sun[hit]
        p0 = p + 1e-3 * s
        ts_end = np.maximum((0.8 - p0[:, 2]) / np.maximum(s[:, 2], 1e-6), 0.0)
        lit = np.ones(p0.shape[0], dtype=bool)
        n_sh = 96
        for k in range(1, n_sh + 1):
            t = ts_end * (k / n_sh)
            q = p0 + t[:, None] * s
            lit &= ~(q[:, 2] < self.height(q[:, 0], q[:, 1]))
        rgb[hit] = alb * np.where(lit, 1.0, 0.3)[:, None]
        return rgb


def full_tile(seed: int = 0, n_rays: int = 1 << 18, samples: int = 128,
              n_views: int = 8, image_px: int = 1024, render_targets: bool = True) -> Workload:
    """Single unit tile over the heightfield scene, altitude band [0.2, 0.8]."""
    rng = np.random.default_rng(seed)
    grid = GridConfig(n_levels=16, n_features=2, log2_table=19, res_min=16, res_max=2048)
    mlp = MlpConfig(feat_width=32, feat_real=32, hidden=64, dens_out=16, n_dir=6,
                    colour_layers=2, colour_out=4)
    scene = Heightfield(rng)
    dirs = _view_dirs(rng, n_views + 1, 30.0)          # last view is held out
    el = np.deg2rad(rng.uniform(40.0, 70.0, size=n_views + 1))
    az = rng.uniform(0.0, 2.0 * np.pi, size=n_views + 1)
    suns = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=1)
    view = rng.integers(0, n_views, size=n_rays)
    px = rng.integers(0, image_px, size=(n_rays, 2))
    g = np.concatenate([(px + 0.5) / image_px, np.full((n_rays, 1), 0.5)], axis=1)
    d = dirs[view]
    s = (1.0 - 0.5) / (-d[:, 2])
    o = g - s[:, None] * d
    o[:, 2] = 1.0
    sun = suns[view]
    if render_targets:
        target = scene.render(o, d, sun).astype(np.float32)
    else:
        target = rng.uniform(0.0, 1.0, size=(n_rays, 3)).astype(np.float32)
    table = init_table(rng, grid)
    params = init_mlp(rng, mlp)
    boxes = np.array([[0.0, 0.0, 0.0, 1.0, 1.0, 1.0]])
    wl = Workload("full_tile", grid, mlp, boxes, np.array([0.2, 0.8]), o, d,
                  sun.astype(np.float32), target, samples, 1e-4, table, params)
    wl.scene = scene
    wl.view_dirs = dirs
    wl.sun_dirs = suns
    return wl


def window_2x2(seed: int = 0, rays_per_tile=None, n_views: int = 8, image_px: int = 1024,
               spr_range=(8, 128), max_off_nadir_deg: float = 30.0) -> Workload:
    """2x2 window of unit tiles covering [0,2]^2 x [0,1] with the small-tile
    hash grid and networks per tile.  Tile k = (i, j) gets rays_per_tile[k]
    rays (default: uniform in 2^15..2^18): each picks a view, then a pixel
    centre of that view's crop of the tile -- the bounding box of the 8 box
    corners projected along the view direction onto the z = 0.5 image plane,
    grown by 10 % of its size on every side (pixels of side 2/image_px over
    [0,2]^2).  Origins sit on z = 2.  Per-ray budgets are uniform in
    spr_range; targets are uniform RGB."""
    rng = np.random.default_rng(seed)
    grid = GridConfig(n_levels=8, n_features=2, log2_table=14, res_min=16, res_max=256)
    mlp = MlpConfig(feat_width=32, feat_real=16, hidden=64, dens_out=16, n_dir=3,
                    colour_layers=1, colour_out=3)
    boxes = np.array([[i, j, 0.0, i + 1.0, j + 1.0, 1.0] for i in range(2) for j in range(2)])
    K = boxes.shape[0]
    if rays_per_tile is None:
        rays_per_tile = rng.integers(1 << 15, (1 << 18) + 1, size=K)
    rays_per_tile = np.asarray(rays_per_tile, dtype=np.int64)
    dirs = _view_dirs(rng, n_views, max_off_nadir_deg)
    px = 2.0 / image_px
    os_, ds_ = [], []
    for k in range(K):
        b = boxes[k]
        corners = np.array([[b[0 + 3 * (q & 1)], b[1 + 3 * ((q >> 1) & 1)], b[2 + 3 * ((q >> 2) & 1)]]
                            for q in range(8)])
        view = rng.integers(0, n_views, size=rays_per_tile[k])
        for v in range(n_views):
            sel = np.nonzero(view == v)[0]
            if sel.size == 0:
                continue
            d = dirs[v]
            proj = corners[:, :2] + ((0.5 - corners[:, 2]) / d[2])[:, None] * d[None, :2]
            lo, hi = proj.min(0), proj.max(0)
            m = 0.1 * (hi - lo)
            lo, hi = lo - m, hi + m
            ilo = np.floor(lo / px).astype(np.int64)
            ihi = np.ceil(hi / px).astype(np.int64)
            pix = np.stack([rng.integers(ilo[a], ihi[a], size=sel.size) for a in range(2)], 1)
            g = np.concatenate([(pix + 0.5) * px, np.full((sel.size, 1), 0.5)], 1)
            s = (2.0 - 0.5) / (-d[2])
            o = g - s * d[None, :]
            o[:, 2] = 2.0
            os_.append(o)
            ds_.append(np.repeat(d[None, :], sel.size, 0))
    rays_o = np.concatenate(os_)
    rays_d = np.concatenate(ds_)
    R = rays_o.shape[0]
    spr = rng.integers(spr_range[0], spr_range[1] + 1, size=R).astype(np.int32)
    target = rng.uniform(0.0, 1.0, size=(R, 3)).astype(np.float32)
    table = init_table(rng, grid, n_tiles=K)
    params = np.stack([init_mlp(rng, mlp) for _ in range(K)])
    wl = Workload("window_2x2", grid, mlp, boxes, None, rays_o, rays_d, None, target, spr, 0.0, table,
                  params)
    wl.rays_per_tile = rays_per_tile
    wl.view_dirs = dirs
    return wl


def window_rays(seed: int, n_rays: int, max_off_nadir_deg: float = 10.0, margin: float = 0.3,
                spr_range=(8, 128)):
    """Rays of one 2x2 window in its local frame ([0,2]^2 x [0,1]): ground
    points uniform in [margin, 2-margin]^2 at z = 0.5, off-nadir at most
    max_off_nadir_deg (with the defaults every ray's chord through the band
    stays inside the window), origins on z = 2, budgets uniform in spr_range,
    uniform RGB targets.  Returns (rays_o, rays_d, target, samples_per_ray)."""
    rng = np.random.default_rng(seed)
    th = np.deg2rad(rng.uniform(0.0, max_off_nadir_deg, size=n_rays))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_rays)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)], axis=1)
    g = np.concatenate([rng.uniform(margin, 2.0 - margin, size=(n_rays, 2)), np.full((n_rays, 1), 0.5)], 1)
    o = g - ((2.0 - 0.5) / np.cos(th))[:, None] * d
    spr = rng.integers(spr_range[0], spr_range[1] + 1, size=n_rays).astype(np.int32)
    target = rng.uniform(0.0, 1.0, size=(n_rays, 3)).astype(np.float32)
    return o, d, target, spr


def tile_init(seed: int, n_levels: int, n_features: int, log2_table: int, m: MlpConfig):
    """init_tile(t) for a sweep over many NeRF tiles: tile t's table U(-1e-4,
    1e-4) (flattened [L][T][F]) and Xavier weights, from the seed and t."""
    def init(t):
        rng = np.random.default_rng([seed, t])
        table = rng.uniform(-1e-4, 1e-4, size=n_levels * (1 << log2_table) * n_features).astype(np.float32)
        return table, init_mlp(rng, m)
    return init


def full_tile_heldout(wl: Workload, n_px: int = 256):
    """Rays and rendered targets of the held-out ninth view of a full_tile
    workload on an n_px x n_px pixel grid over the tile (pixel centres), with
    that view's sun.  Returns (rays_o, rays_d, target, sun)."""
    d = wl.view_dirs[-1]
    sun = wl.sun_dirs[-1]
    ax = (np.arange(n_px) + 0.5) / n_px
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    g = np.stack([X.ravel(), Y.ravel(), np.full(X.size, 0.5)], 1)
    s = (1.0 - 0.5) / (-d[2])
    o = g - s * d[None, :]
    o[:, 2] = 1.0
    dd = np.repeat(d[None, :], o.shape[0], 0)
    su = np.repeat(sun[None, :], o.shape[0], 0)
    target = wl.scene.render(o, dd, su).astype(np.float32)
    return o, dd, target, su.astype(np.float32)
