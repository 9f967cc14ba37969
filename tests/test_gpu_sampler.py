"""GPU parity of snake_sample_segmented / snake_pack_alive against the FP64
oracle: sample bounds, positions, ray ids, tile ids and packing bit for bit."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, dev, host, run_sampler, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2507_01631_amd import _lib
    _lib.lib()
    return _lib


def _same(g, o, keys=("t0", "t1", "pos", "ray_id")):
    assert g["n"] == o["n"]
    assert np.array_equal(g["packed_info"], o["packed_info"])
    for k in keys:
        assert np.array_equal(g[k], o[k]), k


def _grid_boxes(nx, ny, side=1.0, z=(0.0, 1.0), x0=0.0, y0=0.0):
    return np.array([[x0 + i * side, y0 + j * side, z[0], x0 + (i + 1) * side, y0 + (j + 1) * side, z[1]]
                     for i in range(nx) for j in range(ny)])


def _slanted(rng, n, lo, hi, z_top, max_deg=30.0):
    th = np.deg2rad(rng.uniform(0.0, max_deg, size=n))
    ph = rng.uniform(0, 2 * np.pi, size=n)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)], 1)
    g = np.concatenate([rng.uniform(lo, hi, size=(n, 2)), np.full((n, 1), 0.5)], 1)
    return g - ((z_top - 0.5) / np.cos(th))[:, None] * d, d


def test_tiny_tile_bitexact(L, orc):
    w = synth.tiny_tile(seed=0)
    g = run_sampler(L, w.rays_o, w.rays_d, w.boxes, 64)
    o = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 64)
    _same(g, o)
    assert np.array_equal(g["view"], o["view"])


def test_full_tile_band_bitexact(L, orc):
    w = synth.full_tile(seed=1, n_rays=3000, render_targets=False)
    g = run_sampler(L, w.rays_o, w.rays_d, w.boxes, 128, zband=w.zband)
    o = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 128, zband=w.zband)
    _same(g, o)
    assert np.array_equal(g["view"], o["view"])
    assert g["pos"][:, 2].min() >= 0.2 - 1e-6 and g["pos"][:, 2].max() <= 0.8 + 1e-6


def test_window_ragged_multi_tile_bitexact(L, orc):
    """2x2 window of unit tiles, ragged budgets, misses, vertical and axis rays."""
    rng = np.random.default_rng(2)
    boxes = _grid_boxes(2, 2)
    o, d = _slanted(rng, 4000, -0.3, 2.3, z_top=1.6)
    o[:8] = [[0.5, 0.5, 2], [1.0, 0.5, 2], [1.0, 1.0, 2], [3, 3, 2], [0.25, 0.75, 0.5],
             [-1, 0.5, 0.5], [0.5, -1, 0.25], [1.5, 1.5, 1.0]]
    d[:8] = [[0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [1, 0, 0], [0, 1, 0],
             [0.3, -0.2, -0.9]]
    spr = rng.integers(0, 129, size=4000).astype(np.int32)
    spr[:3] = [1, 2, 3]
    g = run_sampler(L, o, d, boxes, 0, spr=spr)
    r = orc.sample_segmented(o, d, boxes, 0, samples_per_ray=spr)
    _same(g, r, keys=("t0", "t1", "pos", "ray_id", "tile_id"))
    assert np.array_equal(g["view"], r["view"])
    # four-tile windows with an altitude band, scaled world coordinates
    boxes2 = _grid_boxes(2, 2, side=153.6, z=(0.0, 200.0), x0=412345.0, y0=3312345.0)
    o2 = o * np.array([153.6, 153.6, 200.0]) + np.array([412345.0, 3312345.0, 0.0])
    d2 = d * np.array([153.6, 153.6, 200.0])
    g = run_sampler(L, o2, d2, boxes2, 96, zband=[20.0, 180.0])
    r = orc.sample_segmented(o2, d2, boxes2, 96, zband=[20.0, 180.0])
    _same(g, r, keys=("t0", "t1", "pos", "ray_id", "tile_id"))


def test_truncation_prefix_and_capacity(L, orc):
    w = synth.tiny_tile(seed=3, n_rays=777, samples=48)
    mc = np.random.default_rng(4).integers(-2, 60, size=777).astype(np.int32)
    g = run_sampler(L, w.rays_o, w.rays_d, w.boxes, 48, max_count=mc)
    o = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 48, max_count=mc)
    _same(g, o)
    # too small a capacity: nothing past cap is written and the device flags it
    L.snake_check_device_error()
    g = run_sampler(L, w.rays_o, w.rays_d, w.boxes, 48, cap=1000)
    assert g["n"] == 777 * 48
    assert L.snake_check_device_error() == L.SNAKE_DEVERR_CAPACITY
    assert L.snake_check_device_error() == 0


def test_empty_and_all_miss(L):
    g = run_sampler(L, np.zeros((0, 3)), np.zeros((0, 3)), synth.tiny_tile(n_rays=1).boxes, 16)
    assert g["n"] == 0
    o = np.tile([5.0, 5.0, 2.0], (100, 1))
    d = np.tile([0.0, 0.0, -1.0], (100, 1))
    g = run_sampler(L, o, d, np.array([[0, 0, 0, 1, 1, 1.0]]), 16)
    assert g["n"] == 0 and np.all(g["packed_info"][:, 1] == 0)


def test_pack_alive(L):
    rng = np.random.default_rng(5)
    R = 5000
    cnt = rng.integers(0, 130, size=R).astype(np.int32)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int32)
    alive = rng.integers(-3, 140, size=R).astype(np.int32)
    info = dev(np.stack([start, cnt], 1), torch.int32)
    cap = int(cnt.sum())
    idx = torch.full((cap,), -1, dtype=torch.int32, device=DEV)
    n_out = torch.zeros(1, dtype=torch.int64, device=DEV)
    ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=DEV)
    L.snake_pack_alive(info, dev(alive, torch.int32), R, idx, cap, n_out, ws)
    sync()
    keep = np.clip(alive, 0, cnt)
    expect = np.concatenate([np.arange(s, s + k) for s, k in zip(start, keep)]).astype(np.int32)
    assert int(host(n_out)[0]) == expect.size
    assert np.array_equal(host(idx)[:expect.size], expect)


def test_window_accept_bitexact(L, orc):
    """Sliding-window acceptance decisions and the compacted index list match
    the oracle exactly, including rays whose chord ends exactly on the window
    edge, vertical rays, rays parallel to the band and origins inside it."""
    rng = np.random.default_rng(31)
    o, d = _slanted(rng, 5000, -0.4, 2.4, z_top=1.4)
    # exact edge cases: vertical rays on and just off the closed edge
    o[:4] = [[2.0, 1.0, 3.0], [2.0 + 2**-40, 1.0, 3.0], [0.0, 0.0, 3.0], [1.0, 1.0, 0.5]]
    d[:4] = [[0.0, 0.0, -1.0], [0.0, 0.0, -1.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]]
    win, zb = (0.0, 0.0, 2.0, 2.0), (0.0, 1.0)
    R = o.shape[0]
    acc = torch.empty(R, dtype=torch.uint8, device=DEV)
    idx = torch.full((R,), -1, dtype=torch.int32, device=DEV)
    n = torch.zeros(1, dtype=torch.int64, device=DEV)
    ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=DEV)
    L.snake_window_accept(dev(o), dev(d), R, win, zb, acc, idx, n, ws)
    sync()
    ref = orc.window_accept(o, d, win, zb)
    assert np.array_equal(host(acc).astype(np.int32), ref)
    assert int(n.item()) == int(ref.sum())
    assert np.array_equal(host(idx)[:int(ref.sum())], np.nonzero(ref)[0].astype(np.int32))
    assert ref[:4].tolist() == [1, 0, 1, 0]
    assert 1000 < ref.sum() < R - 1000
    # no output array for the flags, and an empty call
    idx2 = torch.full((R,), -1, dtype=torch.int32, device=DEV)
    L.snake_window_accept(dev(o), dev(d), R, win, zb, None, idx2, n, ws)
    sync()
    assert torch.equal(idx2, idx)
    L.snake_window_accept(dev(o), dev(d), 0, win, zb, None, idx2, n, ws)
    sync()
    assert int(n.item()) == 0


@pytest.mark.parametrize("K", [1, 4, 16])
def test_tile_partition_is_stable_sort(L, K):
    """perm is the stable sort of the samples by tile id (bad ids last), inv its
    inverse, tile_start the group bounds; the gathered copies follow perm;
    a device count shorter than n limits every output."""
    rng = np.random.default_rng(40 + K)
    n = 300_001
    tid = rng.integers(0, K, size=n).astype(np.uint8)
    tid[rng.random(n) < 0.3] = min(K - 1, 2)             # uneven group sizes
    if K > 1:
        tid[::997] = K + 3                                 # out-of-range ids go last
    pos = rng.random((n, 3)).astype(np.float32)
    rid = rng.integers(0, 1 << 20, size=n).astype(np.int32)
    ws = torch.empty(L.snake_tile_partition_workspace_bytes(K), dtype=torch.uint8, device=DEV)
    for ne in (n, 123_457):
        perm = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        inv = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        ts = torch.zeros(K + 2, dtype=torch.int64, device=DEV)
        po = torch.zeros((n, 3), device=DEV)
        to = torch.zeros(n, dtype=torch.uint8, device=DEV)
        ro = torch.zeros(n, dtype=torch.int32, device=DEV)
        nd = torch.tensor([ne], dtype=torch.int64, device=DEV)
        L.snake_check_device_error()                     # clear the sticky error word
        L.snake_tile_partition(dev(tid), dev(pos), dev(rid), n, nd, K, perm, inv, ts, po, to, ro, ws)
        sync()
        key = np.minimum(tid[:ne].astype(np.int64), K)
        ref = np.argsort(key, kind="stable").astype(np.int32)
        assert np.array_equal(host(perm)[:ne], ref)
        assert np.all(host(perm)[ne:] == -1)
        assert np.array_equal(host(inv)[ref], np.arange(ne, dtype=np.int32))
        bounds = np.searchsorted(key[ref], np.arange(K + 1))
        assert np.array_equal(host(ts), np.concatenate([bounds, [ne]]))
        assert np.array_equal(host(po)[:ne], pos[ref])
        assert np.array_equal(host(to)[:ne], tid[ref])
        assert np.array_equal(host(ro)[:ne], rid[ref])
        err = L.snake_check_device_error()
        assert bool(err & L.SNAKE_DEVERR_TILE_ID) == (K > 1)


def _run_grouped(L, rays_o, rays_d, boxes, S, zband=None, spr=None, max_count=None):
    R = int(np.asarray(rays_o).shape[0])
    K = np.asarray(boxes).reshape(-1, 6).shape[0]
    cap = max(int(np.sum(spr)) if spr is not None else R * int(S), 1)
    Rb = max(R, 1)
    out = dict(packed_info=torch.full((Rb, 2), -1, dtype=torch.int32, device=DEV),
               t0=torch.zeros(cap, device=DEV), t1=torch.zeros(cap, device=DEV),
               view=torch.zeros((Rb, 3), device=DEV), pos=torch.zeros((cap, 3), device=DEV),
               ray_id=torch.full((cap,), -1, dtype=torch.int32, device=DEV),
               tile_id=torch.full((cap,), 255, dtype=torch.uint8, device=DEV),
               smap=torch.full((cap,), -1, dtype=torch.int32, device=DEV),
               tile_start=torch.full((K + 2,), -1, dtype=torch.int64, device=DEV),
               n_out=torch.full((1,), -1, dtype=torch.int64, device=DEV))
    ws = torch.empty(L.snake_sample_grouped_workspace_bytes(R, K), dtype=torch.uint8, device=DEV)
    ro = dev(np.asarray(rays_o, np.float64).reshape(-1, 3)) if R else None
    rd = dev(np.asarray(rays_d, np.float64).reshape(-1, 3)) if R else None
    L.snake_sample_grouped(ro, rd, R, boxes, zband, None if spr is None else dev(spr, torch.int32), S,
                           None if max_count is None else dev(max_count, torch.int32), out["packed_info"],
                           out["t0"], out["t1"], out["view"], out["pos"], out["ray_id"], out["tile_id"],
                           out["smap"], out["tile_start"], cap, out["n_out"], ws)
    sync()
    res = {k: host(v) for k, v in out.items()}
    n = int(res["n_out"][0])
    res["n"] = n
    for k in ("t0", "t1", "pos", "ray_id", "tile_id", "smap"):
        res[k] = res[k][:n]
    res["packed_info"], res["view"] = res["packed_info"][:R], res["view"][:R]
    return res


def _check_grouped(g, o, K):
    """The grouped outputs are the oracle's packed samples stably sorted by
    tile; t0/t1, packed_info and view stay in packed order."""
    n = o["n"]
    assert g["n"] == n
    assert np.array_equal(g["packed_info"], o["packed_info"])
    assert np.array_equal(g["view"], o["view"])
    assert np.array_equal(g["t0"], o["t0"]) and np.array_equal(g["t1"], o["t1"])
    tid = o["tile_id"] if o.get("tile_id") is not None else np.zeros(n, np.uint8)
    perm = np.argsort(tid, kind="stable")
    assert np.array_equal(g["pos"], o["pos"][perm])
    assert np.array_equal(g["ray_id"], o["ray_id"][perm])
    assert np.array_equal(g["tile_id"], tid[perm])
    assert np.array_equal(g["smap"][perm], np.arange(n))
    bounds = np.searchsorted(tid[perm], np.arange(K + 1))
    assert np.array_equal(g["tile_start"], np.concatenate([bounds, [n]]))


def test_grouped_sampler_matches_oracle(L, orc):
    """snake_sample_grouped: the packed samples of the oracle, written grouped
    by tile, over 2x2 windows (ragged budgets, misses, axis and vertical
    rays; world coordinates with an altitude band), five tiles (the 16-box
    kernels), one tile, truncation by max_count, and no rays."""
    rng = np.random.default_rng(2)
    boxes = _grid_boxes(2, 2)
    o, d = _slanted(rng, 4000, -0.3, 2.3, z_top=1.6)
    o[:8] = [[0.5, 0.5, 2], [1.0, 0.5, 2], [1.0, 1.0, 2], [3, 3, 2], [0.25, 0.75, 0.5],
             [-1, 0.5, 0.5], [0.5, -1, 0.25], [1.5, 1.5, 1.0]]
    d[:8] = [[0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [1, 0, 0], [0, 1, 0],
             [0.3, -0.2, -0.9]]
    spr = rng.integers(0, 129, size=4000).astype(np.int32)
    spr[:3] = [1, 2, 3]
    _check_grouped(_run_grouped(L, o, d, boxes, 0, spr=spr), orc.sample_segmented(o, d, boxes, 0, samples_per_ray=spr), 4)
    mc = rng.integers(-2, 90, size=4000).astype(np.int32)
    _check_grouped(_run_grouped(L, o, d, boxes, 0, spr=spr, max_count=mc),
                   orc.sample_segmented(o, d, boxes, 0, samples_per_ray=spr, max_count=mc), 4)
    boxes2 = _grid_boxes(2, 2, side=153.6, z=(0.0, 200.0), x0=412345.0, y0=3312345.0)
    o2 = o * np.array([153.6, 153.6, 200.0]) + np.array([412345.0, 3312345.0, 0.0])
    d2 = d * np.array([153.6, 153.6, 200.0])
    _check_grouped(_run_grouped(L, o2, d2, boxes2, 96, zband=[20.0, 180.0]),
                   orc.sample_segmented(o2, d2, boxes2, 96, zband=[20.0, 180.0]), 4)
    boxes5 = _grid_boxes(3, 2)[:5]
    o5, d5 = _slanted(rng, 3000, -0.3, 3.3, z_top=1.6)
    _check_grouped(_run_grouped(L, o5, d5, boxes5, 64), orc.sample_segmented(o5, d5, boxes5, 64), 5)
    w = synth.tiny_tile(seed=0)
    _check_grouped(_run_grouped(L, w.rays_o, w.rays_d, w.boxes, 64),
                   orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 64), 1)
    g = _run_grouped(L, np.zeros((0, 3)), np.zeros((0, 3)), boxes, 16)
    assert g["n"] == 0 and np.all(g["tile_start"] == 0)


def test_grouped_sampler_capacity_overflow(L):
    """Too small a capacity: the overflow is flagged, and every map entry of the
    kept packed samples still points inside the arrays."""
    rng = np.random.default_rng(3)
    boxes = _grid_boxes(2, 2)
    o, d = _slanted(rng, 3000, -0.3, 2.3, z_top=1.6)
    R, K, cap = 3000, 4, 20000
    ws = torch.empty(L.snake_sample_grouped_workspace_bytes(R, K), dtype=torch.uint8, device=DEV)
    f = lambda *s, dt=torch.float32: torch.zeros(s, dtype=dt, device=DEV)
    smap = torch.full((cap,), -1, dtype=torch.int32, device=DEV)
    n_out = f(1, dt=torch.int64)
    L.snake_check_device_error()
    L.snake_sample_grouped(dev(o), dev(d), R, boxes, None, None, 64, None, f(R, 2, dt=torch.int32), f(cap), f(cap),
                           f(R, 3), f(cap, 3), f(cap, dt=torch.int32), f(cap, dt=torch.uint8), smap,
                           f(K + 2, dt=torch.int64), cap, n_out, ws)
    sync()
    assert int(n_out.item()) > cap
    assert L.snake_check_device_error() & L.SNAKE_DEVERR_CAPACITY
    m = host(smap)
    assert np.all((m >= 0) & (m < cap))
