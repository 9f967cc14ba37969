"""Coarse occupancy grid and culling (SAT-NGP procedure, Sec. 4.1) on the GPU
against the oracle: cell centres, the decaying-maximum update and the culled
sample packing bit for bit."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, dev, host, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2507_01631_amd import _lib
    _lib.lib()
    return _lib


def test_cells_and_update(L, orc):
    G, K = 32, 3
    n = K * G ** 3
    pos = torch.empty((n, 3), device=DEV)
    tid = torch.empty(n, dtype=torch.uint8, device=DEV)
    L.snake_occupancy_cells(G, K, pos, tid)
    sync()
    rp, rt = orc.occupancy_cell_centres(G, K)
    assert np.array_equal(host(pos), rp) and np.array_equal(host(tid), rt)
    rng = np.random.default_rng(5)
    dens = rng.uniform(0, 2, size=n).astype(np.float32)
    sig = rng.exponential(0.5, size=n).astype(np.float32)
    ws = torch.empty(L.snake_occupancy_workspace_bytes(n), dtype=torch.uint8, device=DEV)
    unpack = lambda bits: ((host(bits).view(np.uint32)[np.arange(n) >> 5] >> (np.arange(n) & 31)) & 1).astype(bool)  # noqa: E731
    for scale, thr, cap in ((1.0, 0.8, 0), (0.25, 0.8, L.SNAKE_OCC_MEAN_CAP), (0.25, 2.0, L.SNAKE_OCC_MEAN_CAP)):
        d, bits = dev(dens), torch.zeros((n + 31) // 32, dtype=torch.int32, device=DEV)
        L.snake_occupancy_update(dev(sig), n, 0.95, scale, thr, cap, d, bits, ws)
        sync()
        ref = np.maximum(dens * np.float32(0.95), np.float32(scale) * sig)     # FP32, as the kernel
        assert np.array_equal(host(d), ref)
        _, occ = orc.occupancy_update(dens, sig, 0.95, thr, scale=scale, mean_cap=bool(cap))
        # the threshold the oracle takes in FP64; cells within FP32 rounding of it may go either way
        t = min(thr, float(ref.astype(np.float64).mean())) if cap else thr
        sure = np.abs(ref.astype(np.float64) - t) > 1e-6 * t
        got = unpack(bits)
        assert np.array_equal(got[sure], occ[sure]) and sure.mean() > 0.999
        assert np.array_equal(got, ref > np.float32(t)) or cap
    # the same call twice gives the same bits (fixed-order mean)
    outs = []
    for _ in range(2):
        d, bits = dev(dens), torch.zeros((n + 31) // 32, dtype=torch.int32, device=DEV)
        L.snake_occupancy_update(dev(sig), n, 0.95, 0.25, 0.1, L.SNAKE_OCC_MEAN_CAP, d, bits, ws)
        outs.append(host(bits))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("K", [1, 4])
def test_cull_matches_oracle(L, orc, K):
    G = 64
    if K == 1:
        w = synth.tiny_tile(seed=4, n_rays=3000, samples=64)
        boxes = w.boxes
        spr = None
        S = 64
    else:
        w = synth.window_2x2(seed=4, rays_per_tile=[800, 700, 900, 600])
        boxes = w.boxes
        spr = w.samples_per_ray
        S = 0
    smp = orc.sample_segmented(w.rays_o, w.rays_d, boxes, S, samples_per_ray=spr)
    rng = np.random.default_rng(9)
    occ = rng.random(K * G ** 3) < 0.35
    bits = np.packbits(occ.reshape(-1, 8)[:, ::-1], axis=1).reshape(-1)      # bit c % 8 of byte c / 8
    words = torch.from_numpy(np.pad(bits, (0, (-bits.size) % 4)).view(np.int32).copy()).to(DEV)
    n, R = smp["n"], w.n_rays
    o = dict(info=torch.zeros((R, 2), dtype=torch.int32, device=DEV), t0=torch.zeros(n, device=DEV),
             t1=torch.zeros(n, device=DEV), pos=torch.zeros((n, 3), device=DEV),
             rid=torch.zeros(n, dtype=torch.int32, device=DEV), tid=torch.zeros(n, dtype=torch.uint8, device=DEV),
             n=torch.zeros(1, dtype=torch.int64, device=DEV))
    ws = torch.empty(L.snake_cull_workspace_bytes(R), dtype=torch.uint8, device=DEV)
    L.snake_cull_samples(G, words, K, R, dev(smp["packed_info"], torch.int32), dev(smp["t0"]), dev(smp["t1"]),
                         dev(smp["pos"]), dev(smp["ray_id"]), dev(smp["tile_id"]) if K > 1 else None,
                         o["info"], o["t0"], o["t1"], o["pos"], o["rid"], o["tid"] if K > 1 else None, n, o["n"], ws)
    sync()
    ref = orc.cull_samples(smp, occ, G)
    m = ref["n"]
    assert int(o["n"].item()) == m and 0 < m < n
    assert np.array_equal(host(o["info"]), ref["packed_info"])
    for k, key in (("t0", "t0"), ("t1", "t1"), ("pos", "pos"), ("rid", "ray_id")):
        assert np.array_equal(host(o[k])[:m], ref[key]), k
    if K > 1:
        assert np.array_equal(host(o["tid"])[:m], ref["tile_id"])


@pytest.mark.parametrize("K", [1, 4])
def test_refine_matches_oracle(L, orc, K):
    """Density-driven sampling after culling: each ray's budget spread over
    its kept intervals, bit for bit against the oracle (counts, bounds,
    positions, ray and tile ids); with every cell occupied it reproduces the
    sampler's own output."""
    G = 64
    if K == 1:
        w = synth.tiny_tile(seed=4, n_rays=1500, samples=48)
        spr, S = None, 48
    else:
        w = synth.window_2x2(seed=4, rays_per_tile=[500, 400, 600, 300])
        spr, S = w.samples_per_ray, 0
    boxes, R = w.boxes, w.n_rays
    smp = orc.sample_segmented(w.rays_o, w.rays_d, boxes, S, samples_per_ray=spr)
    n = smp["n"]
    rng = np.random.default_rng(10)
    for frac in (1.0, 0.3):
        occ = rng.random(K * G ** 3) < frac
        kept = orc.cull_samples(smp, occ, G)
        ref = orc.refine_samples(w.rays_o, w.rays_d, boxes, smp["packed_info"][:, 1], kept)
        o = dict(info=torch.zeros((R, 2), dtype=torch.int32, device=DEV), t0=torch.zeros(n, device=DEV),
                 t1=torch.zeros(n, device=DEV), pos=torch.zeros((n, 3), device=DEV),
                 rid=torch.zeros(n, dtype=torch.int32, device=DEV), tid=torch.zeros(n, dtype=torch.uint8, device=DEV),
                 n=torch.zeros(1, dtype=torch.int64, device=DEV))
        ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=DEV)
        L.snake_sample_refine(dev(w.rays_o), dev(w.rays_d), R, boxes, dev(smp["packed_info"], torch.int32),
                              dev(kept["packed_info"], torch.int32), dev(kept["t0"]), dev(kept["t1"]),
                              dev(kept["tile_id"]) if K > 1 else None, o["info"], o["t0"], o["t1"], o["pos"],
                              o["rid"], o["tid"] if K > 1 else None, n, o["n"], ws)
        sync()
        m = ref["n"]
        assert int(o["n"].item()) == m
        assert np.array_equal(host(o["info"]), ref["packed_info"])
        for k, key in (("t0", "t0"), ("t1", "t1"), ("pos", "pos"), ("rid", "ray_id")):
            assert np.array_equal(host(o[k])[:m], ref[key]), (frac, k)
        if K > 1:
            assert np.array_equal(host(o["tid"])[:m], ref["tile_id"])
        if frac == 1.0:
            assert m == n and np.array_equal(host(o["t0"])[:m], smp["t0"]) and \
                np.array_equal(host(o["pos"])[:m], smp["pos"])
        else:
            assert int(kept["n"]) < m <= n
