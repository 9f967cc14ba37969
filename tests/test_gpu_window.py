"""The 2x2 window step (Sec. 4.4) on the GPU: ray acceptance, the segmented
sampler across four tiles with ragged budgets, the tile partition, per-tile
tables and networks, and the whole step captured in one HIP graph."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, assert_grad, assert_values, dev, host, sync

pytestmark = pytest.mark.gpu


def _window(rays_per_tile, seed=0):
    w = synth.window_2x2(seed=seed, rays_per_tile=rays_per_tile)
    return w


PD = 64 * 32 + 16 * 64


def _nerf(w, precision, R, cap=None, shared=False):
    from paper_2507_01631_amd import WindowNeRF, level_resolutions
    g, m = w.grid, w.mlp
    params = (np.concatenate([w.mlp_params[:, :PD].ravel(), w.mlp_params[0, PD:]]) if shared
              else w.mlp_params)
    return WindowNeRF(boxes=w.boxes, zband=None, res=level_resolutions(g.n_levels, g.res_min, g.res_max),
                      n_features=g.n_features, log2_table=g.log2_table, n_dir=m.n_dir,
                      colour_layers=m.colour_layers, colour_out=m.colour_out, precision=precision,
                      tables=w.table, mlp_params=params, max_rays=R, max_samples=cap, samples=128,
                      lr=w.lr, shared_colour=shared, device=DEV)


def _accepted(w, orc):
    acc = orc.window_accept(w.rays_o, w.rays_d, (0.0, 0.0, 2.0, 2.0), (0.0, 1.0)).astype(bool)
    import copy
    wa = copy.copy(w)
    wa.rays_o, wa.rays_d = w.rays_o[acc], w.rays_d[acc]
    wa.target, wa.samples_per_ray = w.target[acc], w.samples_per_ray[acc]
    return wa, acc


def test_window_accept_matches_oracle(orc):
    w = _window([3000, 2000, 2500, 1500])
    nerf = _nerf(w, "fp32", 16)
    idx, n = nerf.accept(dev(w.rays_o), dev(w.rays_d))
    sync()
    ref = orc.window_accept(w.rays_o, w.rays_d, nerf.window_rect(), nerf.band())
    assert int(n.item()) == int(ref.sum())
    assert np.array_equal(host(idx)[:int(ref.sum())], np.nonzero(ref)[0])


def _frac_within(got, ref, rel, abs_):
    got, ref = np.ravel(got).astype(np.float64), np.ravel(ref).astype(np.float64)
    return float(np.mean(np.abs(got - ref) <= rel * np.abs(ref) + abs_))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shared", [False, True])
def test_window_step_matches_oracle(orc, shared, prec):
    """Window step on the accepted rays vs the oracle's step with one weight
    set per tile (or per-tile density nets and one shared colour net).  FP32:
    values within 1e-5, gradients within 1e-4.  BF16: against the oracle's
    emulation of the 16-bit form (bfloat16 table copy, every matrix-core
    operand rounded to bfloat16, FP64 sums), with the bars derived for the
    single-tile step: values 95 % within 1e-5 and all within 1e-2 (log sigma)
    or 5e-3 (colours), gradients within 2e-3 relative L2."""
    w, _ = _accepted(_window([900, 700, 800, 600], seed=1), orc)
    R = w.n_rays
    nerf = _nerf(w, prec, R, shared=shared)
    ro, rd, tg, spr = dev(w.rays_o), dev(w.rays_d), dev(w.target), dev(w.samples_per_ray)
    nerf.step(ro, rd, tg, spr, update=False)
    sync()
    bf = prec == "bf16"
    o = orc.train_step(w, mlp_params=({"density": w.mlp_params[:, :PD], "colour": w.mlp_params[0, PD:]}
                                      if shared else None), bf16=bf)
    smp = o["sample"]
    n = int(host(nerf.n_out)[0])
    assert n == smp["n"]
    assert np.array_equal(host(nerf.packed_info), smp["packed_info"])
    inv = host(nerf.inv)[:n]
    assert np.array_equal(np.sort(inv), np.arange(n))
    # grouped by tile (packed order within a tile), and the same samples
    assert np.all(np.diff(host(nerf.tile_s)[:n].astype(np.int64)) >= 0)
    perm = np.empty(n, np.int64)
    perm[inv] = np.arange(n)
    ts = host(nerf.tile_start)
    for k in range(4):
        assert np.all(np.diff(perm[ts[k]:ts[k + 1]]) > 0)
    assert np.array_equal(host(nerf.tile_s)[inv], smp["tile_id"])
    assert np.array_equal(host(nerf.pos_s)[inv], smp["pos"])
    assert np.array_equal(host(nerf.ray_s)[inv], np.repeat(np.arange(R), smp["packed_info"][:, 1]))
    ts = host(nerf.tile_start)
    assert np.array_equal(np.diff(ts[:5]), np.bincount(smp["tile_id"], minlength=4))
    sig, rgb, rgb_out = host(nerf.sigma)[inv], host(nerf.rgb)[inv], host(nerf.rgb_out)[:R]
    d_step = host(nerf.depth)[:R].copy()
    g_t, r_t = host(nerf.g_t).ravel(), o["dtable"].ravel()
    rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
    print("ERRTAB window_2x2%s %s sigma %.2e rgb %.2e rgb_out %.2e dsigma %.2e dW %.2e dtable %.2e (rel L2 vs %s)" % (
        " shared" if shared else "", prec, rel(sig, o["sigma"]), rel(rgb, o["rgb"]), rel(rgb_out, o["comp"]["rgb"]),
        rel(host(nerf.dsigma)[inv], o["dsigma"]), rel(host(nerf.g_w).ravel(), o["dW"]), rel(g_t, r_t),
        "emu16" if bf else "fp64"))
    if bf:
        assert _frac_within(sig, o["sigma"], 1e-5, 0.0) >= 0.95
        assert_values(np.log(sig), np.log(o["sigma"]), 0.0, 1e-2, "log sigma")
        for name, got, ref in (("rgb", rgb, o["rgb"]), ("rgb_out", rgb_out, o["comp"]["rgb"])):
            assert _frac_within(got, ref, 1e-5, 1e-7) >= 0.95, name
            assert_values(got, ref, 0.0, 5e-3, name)
        assert_values(float(host(nerf.loss)[0]), o["loss"], 1e-4, 0.0, "loss")
        assert rel(host(nerf.dsigma)[inv], o["dsigma"]) <= 2e-3
        assert rel(host(nerf.g_w).ravel(), o["dW"]) <= 2e-3
        assert rel(g_t, r_t) <= 2e-3
        return
    assert_values(sig, o["sigma"], 1e-5, 1e-7, "sigma")
    assert_values(rgb, o["rgb"], 1e-5, 1e-7, "rgb")
    assert_values(rgb_out, o["comp"]["rgb"], 1e-5, 1e-7, "rgb_out")
    assert_values(float(host(nerf.loss)[0]), o["loss"], 1e-5, 0.0, "loss")
    assert_values(d_step, o["comp"]["depth"], 1e-5, 1e-7, "depth")
    # the forward-only renderer gives the step's depth bit for bit
    dep = nerf.render_depth(ro, rd, spr)
    sync()
    assert np.array_equal(host(dep), d_step)
    assert_grad(host(nerf.dsigma)[inv], o["dsigma"], 1e-4, "dsigma")
    assert_grad(host(nerf.g_w).ravel(), o["dW"], 1e-4, "dW per tile")
    assert np.linalg.norm(g_t - r_t) <= 1e-4 * np.linalg.norm(r_t)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_window_graph_replay_equals_eager(orc, prec):
    """One warm-up step, a captured step replayed three times, against four
    eager steps of an identical window: parameters and Adam moments equal bit
    for bit (every reduction in the step has a fixed order)."""
    w, _ = _accepted(_window([1500, 1200, 1400, 1000], seed=2), orc)
    R = w.n_rays
    ro, rd, tg, spr = dev(w.rays_o), dev(w.rays_d), dev(w.target), dev(w.samples_per_ray)
    a = _nerf(w, prec, R)
    for _ in range(4):
        a.step(ro, rd, tg, spr)
    b = _nerf(w, prec, R)
    b.capture(ro, rd, tg, spr, warmup=1)
    for _ in range(3):
        b.replay()
    sync()
    assert host(b.step_dev).tolist() == [4] * 5
    for name in ("table", "params", "m_t", "v_t", "m_w", "v_w"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert torch.equal(a.rgb_out, b.rgb_out)
