"""The no-allocation sampler entry point (snake_sample_segmented_static),
called through the C ABI, against snake_sample_segmented on the same inputs:
every output bit for bit, on two calls in a row, the second with fewer rays
(the shared static scratch keeps the first call's contents)."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, dev, host, sync

pytestmark = pytest.mark.gpu


def _outputs(R, cap, K):
    return dict(packed_info=torch.full((R, 2), -7, dtype=torch.int32, device=DEV),
                t0=torch.full((cap,), -7.0, device=DEV), t1=torch.full((cap,), -7.0, device=DEV),
                pos=torch.full((cap, 3), -7.0, device=DEV),
                ray_id=torch.full((cap,), -7, dtype=torch.int32, device=DEV),
                tile_id=torch.full((cap,), 255, dtype=torch.uint8, device=DEV) if K > 1 else None,
                view=torch.full((R, 3), -7.0, device=DEV),
                n_out=torch.full((1,), -7, dtype=torch.int64, device=DEV))


def _run(L, static, ro, rd, R, boxes, zband, spr, S, cap):
    K = boxes.shape[0]
    out = _outputs(R, cap, K)
    args = (ro, rd, R, boxes, zband, spr, S, None, out["packed_info"], out["t0"], out["t1"], out["pos"],
            out["ray_id"], out["tile_id"], out["view"], cap, out["n_out"])
    if static:
        L.snake_sample_segmented_static(*args)
    else:
        ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=DEV)
        L.snake_sample_segmented(*args, ws)
    return out


@pytest.mark.parametrize("which", ["full_tile", "window"])
def test_static_sampler_matches_workspace_sampler(which):
    from paper_2507_01631_amd import _lib as L
    L.lib()
    if which == "full_tile":
        w = synth.full_tile(seed=3, n_rays=1 << 17, render_targets=False)
        boxes, zband, spr, S = w.boxes, w.zband, None, 128
    else:
        w = synth.window_2x2(seed=3, rays_per_tile=[40000, 30000, 20000, 10000])
        boxes, zband, spr, S = w.boxes, None, w.samples_per_ray, 0
    R0 = w.n_rays
    for R in (R0, R0 // 3 + 17):                   # the second call is smaller
        ro, rd = dev(w.rays_o[:R]), dev(w.rays_d[:R])
        sp = None if spr is None else dev(np.ascontiguousarray(spr[:R]), torch.int32)
        cap = R * 128
        a = _run(L, False, ro, rd, R, boxes, zband, sp, S, cap)
        b = _run(L, True, ro, rd, R, boxes, zband, sp, S, cap)
        sync()
        n = int(host(a["n_out"])[0])
        assert n > 0 and int(host(b["n_out"])[0]) == n
        assert np.array_equal(host(a["packed_info"]), host(b["packed_info"]))
        assert np.array_equal(host(a["view"]), host(b["view"]))
        for k in ("t0", "t1", "pos", "ray_id", "tile_id"):
            if a[k] is not None:
                assert np.array_equal(host(a[k])[:n], host(b[k])[:n]), k
    assert L.snake_check_device_error() == 0


def test_static_sampler_rejects_more_rays_than_its_scratch():
    from paper_2507_01631_amd import _lib as L
    L.lib()
    big = L.snake_sample_segmented_static_max_rays() + 1
    out = _outputs(1, 1, 1)
    with pytest.raises(L.SnakeError) as e:
        L.snake_sample_segmented_static(out["view"], out["view"], big, np.array([0, 0, 0, 1, 1, 1.0]), None,
                                        None, 8, None, out["packed_info"], out["t0"], out["t1"], out["pos"],
                                        out["ray_id"], None, out["view"], 1, out["n_out"])
    assert e.value.code == -1                      # SNAKE_ERR_INVALID_ARG, caught before any launch
    assert "static scratch limit" in str(e.value)
