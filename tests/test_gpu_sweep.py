"""The snake sweep (Sec. 4.4) on the GPU: tiles enter and leave the device
window by asynchronous copies through staging slots while training goes on;
the result must be exactly that of training each window in turn from a
plain per-tile store (same kernels, same order), and each tile must have
taken one Adam step per step of every window that held it."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, dev, host, sync

pytestmark = pytest.mark.gpu

NX, NY, STEPS, R = 3, 3, 2, 700


def _cfg():
    from paper_2507_01631_amd import level_resolutions
    g = synth.GridConfig(n_levels=8, n_features=2, log2_table=14, res_min=16, res_max=256)
    return dict(res=level_resolutions(8, 16, 256), n_features=2, log2_table=14, n_dir=3, colour_layers=1,
                colour_out=3), g


def _batches():
    cache = {}

    def get(pos, k):
        key = (pos, k)
        if key not in cache:
            o, d, t, s = synth.window_rays(1000 * pos[0] + 100 * pos[1] + k, R, spr_range=(8, 48))
            cache[key] = (dev(o), dev(d), dev(t), dev(s))
        return cache[key]
    return get


@pytest.mark.parametrize("graph", [False, True])
def test_sweep_equals_window_by_window(graph):
    from paper_2507_01631_amd import WindowNeRF
    from paper_2507_01631_amd.sweep import SnakeSweep, snake_path
    kw, _ = _cfg()
    batches = _batches()
    sw = SnakeSweep(NX, NY, precision="fp32", max_rays=R, samples=48, seed=3, device=DEV, **kw)
    init = {f: torch.stack(sw.h[f]).clone() for f in sw.h}       # host store: one pinned buffer per tile
    times = sw.run(STEPS, batches, graph=graph)
    assert len(times) == len(snake_path(NX, NY))
    # reference: a plain store on the device, one fresh window per position
    ref = {f: v.to(DEV) for f, v in init.items()}
    boxes = np.array([[i, j, 0.0, i + 1.0, j + 1.0, 1.0] for i in range(2) for j in range(2)])
    for pos in snake_path(NX, NY):
        w = WindowNeRF(boxes=boxes, zband=None, precision="fp32", max_rays=R, samples=48, device=DEV, **kw)
        tiles = [(pos[0] + i) * NY + (pos[1] + j) for i in range(2) for j in range(2)]
        for s, t in enumerate(tiles):
            w.table.view(4, -1)[s].copy_(ref["table"][t])
            w.m_t.view(4, -1)[s].copy_(ref["m_t"][t])
            w.v_t.view(4, -1)[s].copy_(ref["v_t"][t])
            w.params.view(4, -1)[s].copy_(ref["params"][t])
            w.m_w.view(4, -1)[s].copy_(ref["m_w"][t])
            w.v_w.view(4, -1)[s].copy_(ref["v_w"][t])
            w.step_dev[s:s + 1].copy_(ref["step"][t])
        for k in range(STEPS + (1 if graph and pos == snake_path(NX, NY)[0] else 0)):
            # the graph form trains the first window one extra (warm-up) step
            # on the first batch
            b = batches(pos, 0 if (graph and pos == snake_path(NX, NY)[0] and k == 0) else
                        k - (1 if graph and pos == snake_path(NX, NY)[0] else 0))
            w.step(*b)
        for s, t in enumerate(tiles):
            ref["table"][t].copy_(w.table.view(4, -1)[s])
            ref["m_t"][t].copy_(w.m_t.view(4, -1)[s])
            ref["v_t"][t].copy_(w.v_t.view(4, -1)[s])
            ref["params"][t].copy_(w.params.view(4, -1)[s])
            ref["m_w"][t].copy_(w.m_w.view(4, -1)[s])
            ref["v_w"][t].copy_(w.v_w.view(4, -1)[s])
            ref["step"][t].copy_(w.step_dev[s:s + 1])
        del w
    sync()
    for f in ("table", "m_t", "v_t", "params", "m_w", "v_w", "step"):
        assert torch.equal(torch.stack(sw.h[f]), ref[f].cpu()), f
    # corners were trained in 1 window, edges in 2, the centre in 4
    steps = host(sw.trained_steps()).reshape(NX, NY)
    extra = 1 if graph else 0
    want = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) * STEPS
    want[0, 0] += extra; want[0, 1] += extra; want[1, 0] += extra; want[1, 1] += extra
    assert np.array_equal(steps, want)
