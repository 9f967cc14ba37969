"""The snake sweep (Sec. 4.4) on the GPU: tiles enter and leave the device
window by asynchronous copies through staging slots while training goes on;
the result must be exactly that of training each window in turn from a
plain per-tile store (same kernels, same order), each tile must have taken
one Adam step per step of every window that held it, and the whole sweep
must follow the FP64 oracle's step applied window by window."""
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


def _init(kw, seed=3):
    m = synth.MlpConfig(feat_real=16, n_dir=kw["n_dir"], colour_layers=kw["colour_layers"],
                        colour_out=kw["colour_out"])
    return synth.tile_init(seed, len(kw["res"]), kw["n_features"], kw["log2_table"], m)


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
    sw = SnakeSweep(NX, NY, init_tile=_init(kw), precision="fp32", max_rays=R, samples=48, device=DEV, **kw)
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


def test_sweep_matches_oracle_window_by_window(orc):
    """A 3x3 sweep (4 windows, one step each, FP32) against the oracle: the
    oracle keeps every tile's FP64 parameters and Adam moments, takes each
    window's step on the four tiles it holds (their parameters rounded to
    FP32 for the forward, as the GPU stores them) and applies Adam per tile
    with the tile's own step count.  After the sweep every tile's table,
    networks and Adam moments are compared.  A table entry whose gradient is
    near zero at some step can take the other sign of Adam's first move
    (lr sign(g)) in FP32 than in FP64 and then stays about 2 lr away: such
    entries are few, the networks' weights have no near-zero gradients at
    these sizes, so nearly every value must agree to FP32 precision."""
    import types
    from paper_2507_01631_amd.sweep import SnakeSweep, snake_path
    kw, g = _cfg()
    batches = _batches()
    init = _init(kw, seed=11)
    sw = SnakeSweep(NX, NY, init_tile=init, precision="fp32", max_rays=R, samples=48, device=DEV, **kw)
    sw.run(1, batches, graph=False)
    sync()
    m = synth.MlpConfig(feat_real=16, n_dir=3, colour_layers=1, colour_out=3)
    Lv, T, F = len(kw["res"]), 1 << kw["log2_table"], kw["n_features"]
    n = NX * NY
    st = {"p_t": [], "p_w": [], "m_t": [], "v_t": [], "m_w": [], "v_w": [], "step": [0] * n}
    for t in range(n):
        tab, par = init(t)
        st["p_t"].append(tab.astype(np.float64))
        st["p_w"].append(par.astype(np.float64))
        for f, size in (("m_t", tab.size), ("v_t", tab.size), ("m_w", par.size), ("v_w", par.size)):
            st[f].append(np.zeros(size))
    boxes = np.array([[i, j, 0.0, i + 1.0, j + 1.0, 1.0] for i in range(2) for j in range(2)])
    lr = sw.win.lr
    for pos in snake_path(NX, NY):
        tiles = [(pos[0] + i) * NY + (pos[1] + j) for i in range(2) for j in range(2)]
        o, d, tg, spr = (host(x) for x in batches(pos, 0))
        wl = types.SimpleNamespace(grid=g, mlp=m, boxes=boxes, zband=None, rays_o=o, rays_d=d, target=tg, sun=None,
                                   samples_per_ray=spr, early_stop=0.0, lr=lr)
        tab = np.stack([st["p_t"][t] for t in tiles]).astype(np.float32).reshape(4, Lv, T, F)
        par = np.stack([st["p_w"][t] for t in tiles]).astype(np.float32)
        ref = orc.train_step(wl, table=tab, mlp_params=par)
        dW = ref["dW"].reshape(4, -1)
        for s_, t in enumerate(tiles):
            st["step"][t] += 1
            orc.adam_step(st["p_t"][t], ref["dtable"][s_].ravel(), st["m_t"][t], st["v_t"][t], lr, st["step"][t])
            orc.adam_step(st["p_w"][t], dW[s_], st["m_w"][t], st["v_w"][t], lr, st["step"][t])
    assert host(sw.trained_steps()).ravel().tolist() == st["step"]
    frac = lambda got, ref, rel, abs_: float(np.mean(np.abs(got - ref) <= rel * np.abs(ref) + abs_))
    for t in range(n):
        gt, gw = host(sw.h["table"][t]).astype(np.float64), host(sw.h["params"][t]).astype(np.float64)
        touched = st["v_t"][t] > 0
        ft = frac(gt[touched], st["p_t"][t][touched], 1e-4, 1e-6)
        fw = frac(gw, st["p_w"][t], 1e-4, 1e-6)
        print("tile %d (%d steps): table entries within 1e-4: %.5f of %d touched; weights %.5f"
              % (t, st["step"][t], ft, int(touched.sum()), fw))
        assert np.array_equal(gt[~touched], st["p_t"][t][~touched].astype(np.float32))   # never moved
        assert ft >= 0.995 and fw >= 0.999
        assert np.max(np.abs(gt - st["p_t"][t])) <= 3.0 * lr * st["step"][t]
        for f, key in (("m_t", "m_t"), ("m_w", "m_w")):
            got = host(sw.h[f][t]).astype(np.float64)
            assert frac(got, st[key][t], 1e-3, 1e-9) >= 0.99, f
