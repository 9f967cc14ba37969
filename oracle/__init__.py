"""CPU FP64 oracle for one tile-NeRF training step (ctypes over snake_oracle.c).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library (``paper_2507_01631_amd``) and never imports it.

Every function takes and returns NumPy arrays.  Floating-point results are
FP64; sample bounds/positions and hash indices come out at the FP32 / integer
rounding points the library boundary defines, so they compare bit for bit.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snake_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsnake_oracle.so")
_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP over rays)."""
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_level_resolutions.argtypes = [_I, _I, _I, _P]
        L.orc_hash_index.argtypes = [ctypes.c_uint32] * 3 + [_I, _I, _I]
        L.orc_hash_index.restype = ctypes.c_uint32
        L.orc_hash_corners.argtypes = [_P, _I, _I, _I, _P, _P]
        L.orc_sample_segmented.argtypes = [_I, _P, _P, _I, _P, _P, _P, _I, _P,
                                           _P, _P, _P, _P, _P, _P, _P, _I64, _P]
        L.orc_sample_segmented.restype = _I
        L.orc_hashgrid_fwd.argtypes = [_I, _I, _I, _P, _I, _P, _I64, _P, _P, _I, _P, _P]
        L.orc_hashgrid_bwd.argtypes = [_I, _I, _I, _P, _I, _I, _I64, _P, _P, _I, _P, _P]
        L.orc_mlp_param_count.argtypes = [_I] * 6
        L.orc_mlp_param_count.restype = _I64
        L.orc_mlp_fwd.argtypes = [_I] * 6 + [_P, _I64, _P, _P, _P, _P, _P, _P]
        L.orc_mlp_bwd.argtypes = [_I] * 6 + [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_mlp_margin.argtypes = [_I] * 6 + [_P, _I64, _P, _P, _P, _P, _P]
        L.orc_mlp_fwd_bf16emu.argtypes = [_I] * 6 + [_P, _I64, _P, _P, _P, _P, _P, _P]
        L.orc_mlp_bwd_q.argtypes = [_I] * 6 + [_P, _I64, _P, _P, _P, _P, _P, _P, _I, _P, _P]
        L.orc_bf16_round.argtypes = [_I64, _P, _P]
        L.orc_composite_fwd.argtypes = [_I, _P, _P, _P, _P, _P, _D, _P, _P, _D,
                                        _P, _P, _P, _P, _P]
        L.orc_composite_bwd.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P, _D, _P, _P]
        L.orc_adam_step.argtypes = [_I64, _P, _P, _P, _P, _D, _D, _D, _D, _I, _D]
        L.orc_window_accept.argtypes = [_I, _P, _P, _P, _D, _D, _P]
        L.orc_window_accept.restype = _I64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# hash grid
# ---------------------------------------------------------------------------
def level_resolutions(L: int, n_min: int, n_max: int) -> np.ndarray:
    out = np.zeros(L, dtype=np.int32)
    lib().orc_level_resolutions(L, n_min, n_max, _ptr(out))
    return out


def hash_index(i: int, j: int, k: int, N: int, log2T: int, always_hash: bool = False) -> int:
    return int(lib().orc_hash_index(i, j, k, N, log2T, int(always_hash)))


def hash_corners(x, N: int, log2T: int, always_hash: bool = False):
    x = _c(x, np.float32)
    idx = np.zeros(8, dtype=np.uint32)
    w = np.zeros(8, dtype=np.float64)
    lib().orc_hash_corners(_ptr(x), N, log2T, int(always_hash), _ptr(idx), _ptr(w))
    return idx, w


def hashgrid_fwd(res, log2T, table, pos, tile_id=None, out_width=32, always_hash=False,
                 return_index=False):
    """table: float32 [K][L][T][F]; pos: float32 [n][3] -> feat float64 [n][out_width]."""
    res = _c(res, np.int32)
    table = _c(table, np.float32)
    pos = _c(pos, np.float32).reshape(-1, 3)
    L, F = int(table.shape[1]), int(table.shape[3])
    n = pos.shape[0]
    feat = np.zeros((n, out_width), dtype=np.float64)
    idx = np.zeros((n, L, 8), dtype=np.uint32) if return_index else None
    tid = _c(tile_id, np.uint8)
    lib().orc_hashgrid_fwd(L, F, log2T, _ptr(res), int(always_hash), _ptr(table), n,
                           _ptr(pos), _ptr(tid), out_width, _ptr(feat), _ptr(idx))
    return (feat, idx) if return_index else feat


def hashgrid_bwd(res, log2T, table_shape, pos, dfeat, tile_id=None, always_hash=False):
    """Gradient of sum(feat * dfeat) w.r.t. the table: float64 [K][L][T][F]."""
    K, L, T, F = table_shape
    res = _c(res, np.int32)
    pos = _c(pos, np.float32).reshape(-1, 3)
    dfeat = _c(dfeat, np.float64)
    n, W = dfeat.shape
    dtable = np.zeros((K, L, T, F), dtype=np.float64)
    tid = _c(tile_id, np.uint8)
    lib().orc_hashgrid_bwd(L, F, log2T, _ptr(res), int(always_hash), K, n, _ptr(pos),
                           _ptr(tid), W, _ptr(dfeat), _ptr(dtable))
    return dtable


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------
def _mlp_args(m):
    return (int(m.feat_width), int(m.hidden), int(m.dens_out), int(m.n_dir),
            int(m.colour_layers), int(m.colour_out))


def mlp_param_count(m) -> int:
    return int(lib().orc_mlp_param_count(*_mlp_args(m)))


def mlp_fwd(m, weights, feat, view, ray_id, sun=None):
    """feat float64 [n][feat_width]; view/sun float32 [R][3] -> sigma [n], rgb [n][3]."""
    weights = _c(weights, np.float32)
    feat = _c(feat, np.float64)
    n = feat.shape[0]
    sigma = np.zeros(n)
    rgb = np.zeros((n, 3))
    lib().orc_mlp_fwd(*_mlp_args(m), _ptr(weights), n, _ptr(feat), _ptr(_c(view, np.float32)),
                      _ptr(_c(sun, np.float32)), _ptr(_c(ray_id, np.int32)), _ptr(sigma), _ptr(rgb))
    return sigma, rgb


def mlp_margin(m, weights, feat, view, ray_id, sun=None):
    """Per-sample distance from the nearest ReLU kink, min |z| / sum |W x|."""
    weights = _c(weights, np.float32)
    feat = _c(feat, np.float64)
    n = feat.shape[0]
    out = np.zeros(n)
    lib().orc_mlp_margin(*_mlp_args(m), _ptr(weights), n, _ptr(feat), _ptr(_c(view, np.float32)),
                         _ptr(_c(sun, np.float32)), _ptr(_c(ray_id, np.int32)), _ptr(out))
    return out


def mlp_fwd_bf16emu(m, weights, feat, view, ray_id, sun=None):
    """Forward with BF16 rounding emulated at the operand rounding points
    (diagnostic; the reference forward is mlp_fwd)."""
    weights = _c(weights, np.float32)
    feat = _c(feat, np.float64)
    n = feat.shape[0]
    sigma = np.zeros(n)
    rgb = np.zeros((n, 3))
    lib().orc_mlp_fwd_bf16emu(*_mlp_args(m), _ptr(weights), n, _ptr(feat),
                              _ptr(_c(view, np.float32)), _ptr(_c(sun, np.float32)),
                              _ptr(_c(ray_id, np.int32)), _ptr(sigma), _ptr(rgb))
    return sigma, rgb


def mlp_bwd(m, weights, feat, view, ray_id, dsigma, drgb, sun=None):
    weights = _c(weights, np.float32)
    feat = _c(feat, np.float64)
    n = feat.shape[0]
    dW = np.zeros(weights.shape[0])
    dfeat = np.zeros_like(feat)
    lib().orc_mlp_bwd(*_mlp_args(m), _ptr(weights), n, _ptr(feat), _ptr(_c(view, np.float32)),
                      _ptr(_c(sun, np.float32)), _ptr(_c(ray_id, np.int32)),
                      _ptr(_c(dsigma, np.float64)), _ptr(_c(drgb, np.float64)),
                      _ptr(dW), _ptr(dfeat))
    return dW, dfeat


def mlp_bwd_q(m, weights, feat, view, ray_id, dsigma, drgb, sun=None, round16=1):
    """Adjoint of the 16-bit form: mlp_bwd with every matrix-core operand
    rounded to bfloat16 (weights, inputs, post-ReLU activations, colour inputs,
    the output gradient before each transposed product, and both factors of
    each weight-gradient product); round16=0 is mlp_bwd itself, bit for bit."""
    weights = _c(weights, np.float32)
    feat = _c(feat, np.float64)
    n = feat.shape[0]
    dW = np.zeros(weights.shape[0])
    dfeat = np.zeros_like(feat)
    lib().orc_mlp_bwd_q(*_mlp_args(m), _ptr(weights), n, _ptr(feat), _ptr(_c(view, np.float32)),
                        _ptr(_c(sun, np.float32)), _ptr(_c(ray_id, np.int32)),
                        _ptr(_c(dsigma, np.float64)), _ptr(_c(drgb, np.float64)), int(round16),
                        _ptr(dW), _ptr(dfeat))
    return dW, dfeat


def bf16_round(x):
    """x rounded to the nearest bfloat16 (ties to even), as float64."""
    x = _c(x, np.float64)
    out = np.empty_like(x)
    lib().orc_bf16_round(x.size, _ptr(x), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# sampler
# ---------------------------------------------------------------------------
def sample_segmented(rays_o, rays_d, boxes, S, zband=None, samples_per_ray=None,
                     max_count=None, cap=None):
    rays_o = _c(rays_o, np.float64).reshape(-1, 3)
    rays_d = _c(rays_d, np.float64).reshape(-1, 3)
    boxes = _c(boxes, np.float64).reshape(-1, 6)
    R, K = rays_o.shape[0], boxes.shape[0]
    spr = _c(samples_per_ray, np.int32)
    if cap is None:
        cap = int(spr.sum()) if spr is not None else R * int(S)
    cap = max(int(cap), 0)
    info = np.zeros((R, 2), dtype=np.int32)
    t0 = np.zeros(cap, dtype=np.float32)
    t1 = np.zeros(cap, dtype=np.float32)
    pos = np.zeros((cap, 3), dtype=np.float32)
    rid = np.zeros(cap, dtype=np.int32)
    tid = np.zeros(cap, dtype=np.uint8)
    view = np.zeros((R, 3), dtype=np.float32)
    n_out = np.zeros(1, dtype=np.int64)
    rc = lib().orc_sample_segmented(R, _ptr(rays_o), _ptr(rays_d), K, _ptr(boxes),
                                    _ptr(_c(zband, np.float64)), _ptr(spr), int(S),
                                    _ptr(_c(max_count, np.int32)), _ptr(info), _ptr(t0),
                                    _ptr(t1), _ptr(pos), _ptr(rid), _ptr(tid), _ptr(view),
                                    cap, _ptr(n_out))
    n = int(n_out[0])
    if rc != 0:
        raise ValueError("oracle sampler: %d samples exceed capacity %d (rc=%d)" % (n, cap, rc))
    return dict(packed_info=info, t0=t0[:n], t1=t1[:n], pos=pos[:n], ray_id=rid[:n],
                tile_id=tid[:n], view=view, n=n)


def window_accept(rays_o, rays_d, window, zband):
    """Sliding-window ray acceptance (Sec. 4.4): 1 where the ray's chord through
    the altitude band stays inside the closed XY rectangle of the window.
    window = (x_lo, y_lo, x_hi, y_hi)."""
    rays_o = _c(rays_o, np.float64).reshape(-1, 3)
    rays_d = _c(rays_d, np.float64).reshape(-1, 3)
    win = _c(window, np.float64).reshape(4)
    acc = np.zeros(rays_o.shape[0], dtype=np.int32)
    lib().orc_window_accept(rays_o.shape[0], _ptr(rays_o), _ptr(rays_d), _ptr(win),
                            float(zband[0]), float(zband[1]), _ptr(acc))
    return acc


# ---------------------------------------------------------------------------
# coarse occupancy grid (SAT-NGP culling, Sec. 4.1)
# ---------------------------------------------------------------------------
def occupancy_cell(pos, G):
    """Cell of each tile-frame position in a G^3 grid: min(floor(fl32(x G)), G-1)
    per axis (G a power of two, so the product is exact), flattened as
    (i G + j) G + k with i along x."""
    p = np.asarray(pos, dtype=np.float32).reshape(-1, 3)
    c = np.minimum(np.floor(p * np.float32(G)).astype(np.int64), G - 1)
    c = np.maximum(c, 0)
    return (c[:, 0] * G + c[:, 1]) * G + c[:, 2]


def occupancy_cell_centres(G, K=1):
    """Tile-frame centres ((i+0.5)/G, (j+0.5)/G, (k+0.5)/G) of every cell of K
    grids, in cell order, with their tile ids."""
    i = np.arange(G, dtype=np.float64)
    x = (i + 0.5) / G
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    one = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    return np.tile(one, (K, 1)), np.repeat(np.arange(K, dtype=np.uint8), G ** 3)


def occupancy_update(density, sigma, decay, threshold, scale=1.0, mean_cap=False):
    """Decaying maximum of the cells' optical thickness: d = max(decay d,
    scale sigma) (scale = the sample step).  A cell is occupied iff
    d > threshold, or with the mean cap iff d > min(threshold, mean of d).
    The paper names the SAT-NGP culling (Sec. 4.1) without its rule; this is
    the usual I-NGP one, taken as a reading.  FP64."""
    d = np.maximum(np.asarray(density, dtype=np.float64) * decay,
                   scale * np.asarray(sigma, dtype=np.float64))
    thr = min(threshold, float(d.mean())) if mean_cap else threshold
    return d, d > thr


def cull_samples(smp, occupied, G):
    """Keep the samples whose cell (in their own tile's grid) is occupied, in
    order; returns a sampler-like dict over the kept samples."""
    tid = smp["tile_id"].astype(np.int64)
    cell = tid * G ** 3 + occupancy_cell(smp["pos"], G)
    keep = np.asarray(occupied, dtype=bool)[cell]
    info = smp["packed_info"]
    R = info.shape[0]
    counts = np.zeros(R, dtype=np.int32)
    rid = smp["ray_id"]
    np.add.at(counts, rid[keep], 1)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int32)
    out = dict(packed_info=np.stack([starts, counts], 1), view=smp["view"], n=int(keep.sum()))
    for k in ("t0", "t1", "pos", "ray_id", "tile_id"):
        out[k] = smp[k][keep]
    out["keep"] = keep
    return out


def refine_samples(rays_o, rays_d, boxes, budget, kept):
    """Density-driven sampling after culling (Sec. 4.1: the coarse grid's
    occupancy gives each ray segment its sample density).  A ray whose culled
    set ``kept`` (a sampler-like dict, e.g. from cull_samples) holds c > 0
    intervals spends its whole budget B (``budget[r]``, its sample count
    before culling) on them: interval i gets e(i+1) - e(i) equal
    sub-intervals, e(i) = floor((2 B i + c) / (2 c)) (B i / c rounded, halves
    up), so the sample density rises where the grid is occupied.  A ray with
    nothing kept gets no samples.  Sub-interval k of q in [ta, tb] is
    [ta + k h, ta + (k+1) h] with h = (tb - ta) / q (the last one ends at tb),
    and its sample sits at the midpoint, mapped into its tile's frame
    ((o - lo) / ext + m d / ext, clamped to [0, 1]) -- the sampler's own FP32
    rounding points, evaluated one operation at a time here."""
    rays_o = np.asarray(rays_o, dtype=np.float64).reshape(-1, 3)
    rays_d = np.asarray(rays_d, dtype=np.float64).reshape(-1, 3)
    boxes = np.asarray(boxes, dtype=np.float64).reshape(-1, 6)
    budget = np.asarray(budget, dtype=np.int64)
    info = np.asarray(kept["packed_info"], dtype=np.int64)
    R = info.shape[0]
    t0o, t1o, poso, rido, tido = [], [], [], [], []
    counts = np.zeros(R, dtype=np.int32)
    f32 = np.float32
    for r in range(R):
        s0, c = int(info[r, 0]), int(info[r, 1])
        B = int(budget[r]) if c > 0 else 0
        counts[r] = B
        if B == 0:
            continue
        e = [(2 * B * i + c) // (2 * c) for i in range(c + 1)]
        for i in range(c):
            q = e[i + 1] - e[i]
            ta, tb = f32(kept["t0"][s0 + i]), f32(kept["t1"][s0 + i])
            tile = int(kept["tile_id"][s0 + i]) if kept.get("tile_id") is not None else 0
            box = boxes[tile]
            ol = [f32((rays_o[r, a] - box[a]) / (box[3 + a] - box[a])) for a in range(3)]
            dl = [f32(rays_d[r, a] / (box[3 + a] - box[a])) for a in range(3)]
            h = f32(f32(tb - ta) / f32(q))
            for k in range(q):
                a_ = f32(ta + f32(f32(k) * h))
                b_ = tb if k + 1 == q else f32(ta + f32(f32(k + 1) * h))
                m = f32(f32(0.5) * f32(a_ + b_))
                x = [min(max(f32(ol[a] + f32(m * dl[a])), f32(0.0)), f32(1.0)) for a in range(3)]
                t0o.append(a_)
                t1o.append(b_)
                poso.append(x)
                rido.append(r)
                tido.append(tile)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int32)
    n = int(counts.sum())
    return dict(packed_info=np.stack([starts, counts], 1).astype(np.int32), n=n,
                t0=np.asarray(t0o, dtype=np.float32), t1=np.asarray(t1o, dtype=np.float32),
                pos=np.asarray(poso, dtype=np.float32).reshape(n, 3), ray_id=np.asarray(rido, dtype=np.int32),
                tile_id=np.asarray(tido, dtype=np.uint8), view=kept.get("view"))


# ---------------------------------------------------------------------------
# volume rendering
# ---------------------------------------------------------------------------
def composite_fwd(packed_info, sigma, rgb, t0, t1, target=None, loss_scale=0.0,
                  early_stop=0.0, alive=None):
    info = _c(packed_info, np.int32)
    R = info.shape[0]
    rgb_out = np.zeros((R, 3))
    opacity = np.zeros(R)
    depth = np.zeros(R)
    n_alive = np.zeros(R, dtype=np.int32)
    loss = np.zeros(1)
    lib().orc_composite_fwd(R, _ptr(info), _ptr(_c(sigma, np.float64)), _ptr(_c(rgb, np.float64)),
                            _ptr(_c(t0, np.float32)), _ptr(_c(t1, np.float32)), float(early_stop),
                            _ptr(_c(alive, np.int32)), _ptr(_c(target, np.float32)),
                            float(loss_scale), _ptr(rgb_out), _ptr(opacity), _ptr(depth),
                            _ptr(n_alive), _ptr(loss))
    return dict(rgb=rgb_out, opacity=opacity, depth=depth, n_alive=n_alive, loss=float(loss[0]))


def composite_bwd(packed_info, sigma, rgb, t0, t1, target, loss_scale, n_alive=None):
    info = _c(packed_info, np.int32)
    R = info.shape[0]
    n = np.asarray(sigma).shape[0]
    dsigma = np.zeros(n)
    drgb = np.zeros((n, 3))
    lib().orc_composite_bwd(R, _ptr(info), _ptr(_c(sigma, np.float64)), _ptr(_c(rgb, np.float64)),
                            _ptr(_c(t0, np.float32)), _ptr(_c(t1, np.float32)),
                            _ptr(_c(n_alive, np.int32)), _ptr(_c(target, np.float32)),
                            float(loss_scale), _ptr(dsigma), _ptr(drgb))
    return dsigma, drgb


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------
def adam_step(p, g, m, v, lr, step, b1=0.9, b2=0.99, eps=1e-15, l2=0.0):
    """In place on float64 arrays p, m, v."""
    assert p.dtype == m.dtype == v.dtype == np.float64
    g = _c(g, np.float64)
    lib().orc_adam_step(p.size, _ptr(p), _ptr(g), _ptr(m), _ptr(v), float(lr), float(b1),
                        float(b2), float(eps), int(step), float(l2))


# ---------------------------------------------------------------------------
# one training step, composed in the paper's order
# ---------------------------------------------------------------------------
def train_step(wl, res=None, table=None, mlp_params=None, adam_state=None, step=1,
               alive=None, rays=None, timings=None, occupancy=None, bf16=False, refine=False):
    """One step of the tile-NeRF: segmented sampling -> hash encoding -> density
    and colour nets -> volume rendering + MSE loss -> adjoints -> Adam.

    ``wl`` supplies the rays, boxes, band, targets and configs (any object with
    the attributes of ``synth.Workload``).  ``alive`` optionally fixes the
    per-ray early-stop counts (to follow another implementation's decision
    where floating point rounding makes it ambiguous).  ``bf16`` emulates the
    16-bit form: the encoding gathers from the table rounded to bfloat16 (its
    half-precision copy) and both networks round every matrix-core operand to
    bfloat16 (mlp_fwd_bf16emu, mlp_bwd_q); everything else stays FP64.
    Returns a dict of every intermediate, the gradients and the updated FP64
    parameters."""
    t_start = time.perf_counter()
    g, m = wl.grid, wl.mlp
    if res is None:
        res = level_resolutions(g.n_levels, g.res_min, g.res_max)
    table = wl.table if table is None else table
    mlp_params = wl.mlp_params if mlp_params is None else mlp_params
    rays_o, rays_d = (wl.rays_o, wl.rays_d) if rays is None else rays
    target = wl.target if rays is None else rays[2]
    sun = wl.sun if rays is None else rays[3]
    R = rays_o.shape[0]
    out = {}
    spr = wl.samples_per_ray
    if np.ndim(spr) == 0:
        smp = sample_segmented(rays_o, rays_d, wl.boxes, int(spr), zband=wl.zband)
    else:
        smp = sample_segmented(rays_o, rays_d, wl.boxes, 0, zband=wl.zband,
                               samples_per_ray=np.asarray(spr, dtype=np.int32))
    if occupancy is not None:          # (G, occupied cells): SAT-NGP culling before the field
        out["sample_raw"] = smp
        kept = cull_samples(smp, occupancy[1], occupancy[0])
        # with refine, each ray's budget goes to the intervals it kept
        smp = refine_samples(rays_o, rays_d, wl.boxes, smp["packed_info"][:, 1], kept) if refine else kept
    out["sample"] = smp
    table_fwd = bf16_round(table).astype(np.float32).reshape(table.shape) if bf16 else table
    feat = hashgrid_fwd(res, g.log2_table, table_fwd, smp["pos"], smp["tile_id"], g.out_width)
    fwd = mlp_fwd_bf16emu if bf16 else mlp_fwd
    # one weight set ([P]) shared by the tiles, one per tile ([K][P]), or
    # per-tile density nets with one shared colour net ({"density": [K][Pd],
    # "colour": [P-Pd]}): each sample goes through the networks of its tile
    shared_colour = isinstance(mlp_params, dict)
    if shared_colour:
        dens, col = mlp_params["density"], mlp_params["colour"]
        Pd = dens.shape[1]
        full = np.concatenate([dens, np.broadcast_to(col, (dens.shape[0], col.size))], axis=1)
        mlp_flat = np.concatenate([dens.ravel(), col])
    else:
        full = mlp_params
        mlp_flat = np.ravel(mlp_params)
    per_tile = np.ndim(full) == 2
    groups = ([(np.ones(smp["n"], dtype=bool), full)] if not per_tile else
              [(smp["tile_id"] == k, full[k]) for k in range(full.shape[0])])
    sigma, rgb = np.zeros(smp["n"]), np.zeros((smp["n"], 3))
    for sel, w in groups:
        if sel.any():
            sigma[sel], rgb[sel] = fwd(m, w, feat[sel], smp["view"], smp["ray_id"][sel], sun=sun)
    loss_scale = 1.0 / (3.0 * R)
    comp = composite_fwd(smp["packed_info"], sigma, rgb, smp["t0"], smp["t1"], target,
                         loss_scale, early_stop=wl.early_stop, alive=alive)
    n_alive = comp["n_alive"] if alive is None else np.asarray(alive, dtype=np.int32)
    dsigma, drgb = composite_bwd(smp["packed_info"], sigma, rgb, smp["t0"], smp["t1"],
                                 target, loss_scale, n_alive=n_alive)
    dW = np.zeros(np.shape(full))
    dfeat = np.zeros((smp["n"], feat.shape[1]))
    for k, (sel, w) in enumerate(groups):
        if sel.any():
            dWk, dfeat[sel] = mlp_bwd_q(m, w, feat[sel], smp["view"], smp["ray_id"][sel], dsigma[sel], drgb[sel],
                                        sun=sun, round16=int(bf16))
            if per_tile:
                dW[k] += dWk
            else:
                dW += dWk
    if shared_colour:           # the shared colour net collects every tile's gradient
        dW = np.concatenate([dW[:, :Pd].ravel(), dW[:, Pd:].sum(axis=0)])
    dW = dW.ravel()
    dtable = hashgrid_bwd(res, g.log2_table, table.shape, smp["pos"], dfeat, smp["tile_id"])
    if adam_state is None:
        adam_state = dict(m_t=np.zeros(table.size), v_t=np.zeros(table.size),
                          m_w=np.zeros(mlp_flat.size), v_w=np.zeros(mlp_flat.size))
    p_t = table.astype(np.float64).ravel().copy()
    p_w = mlp_flat.astype(np.float64).copy()
    adam_step(p_t, dtable.ravel(), adam_state["m_t"], adam_state["v_t"], wl.lr, step)
    adam_step(p_w, dW, adam_state["m_w"], adam_state["v_w"], wl.lr, step)
    out.update(res=res, feat=feat, sigma=sigma, rgb=rgb, comp=comp, n_alive=n_alive,
               dsigma=dsigma, drgb=drgb, dW=dW, dfeat=dfeat, dtable=dtable,
               table_new=p_t.reshape(table.shape), mlp_new=p_w if shared_colour else p_w.reshape(np.shape(full)),
               adam=adam_state,
               loss=comp["loss"], n_samples=int(n_alive.sum()), n_total=smp["n"])
    if timings is not None:
        timings.append(time.perf_counter() - t_start)
    return out
