"""One whole training step on the GPU against the FP64 oracle's step.

Parameters after Adam are compared where the reference gradient is not tiny
(|g| > 1e-3 max|g|): at step 1 Adam moves every parameter by about lr sign(g),
so a near-zero gradient whose FP32 sign differs from the FP64 one moves a
parameter by 2 lr; that is expected, not an error."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, assert_grad, assert_values, bf16_round, dev, host, sync

pytestmark = pytest.mark.gpu


def make_nerf(w, precision="fp32", max_rays=None, occ_grid=0):
    from paper_2507_01631_amd import TileNeRF, level_resolutions
    g, m = w.grid, w.mlp
    return TileNeRF(res=level_resolutions(g.n_levels, g.res_min, g.res_max), n_features=g.n_features,
                    log2_table=g.log2_table, n_dir=m.n_dir, colour_layers=m.colour_layers,
                    colour_out=m.colour_out, boxes=w.boxes, zband=w.zband, samples=w.samples_per_ray,
                    early_stop=w.early_stop, precision=precision, table=w.table, mlp_params=w.mlp_params,
                    max_rays=max_rays or w.n_rays, lr=w.lr, occ_grid=occ_grid, device=DEV)


def gpu_step(w, precision="fp32", occupancy=None):
    nerf = make_nerf(w, precision, occ_grid=occupancy[0] if occupancy else 0)
    if occupancy:
        occ = occupancy[1]
        by = np.packbits(occ.reshape(-1, 8)[:, ::-1], axis=1).reshape(-1)
        nerf.occ_bits.copy_(torch.from_numpy(by.view(np.int32).copy()))
    ro, rd, tg = dev(w.rays_o), dev(w.rays_d), dev(w.target)
    sun = dev(w.sun) if w.sun is not None else None
    # keep the gradients: run the step by stages and copy before Adam
    R = w.n_rays
    nerf.loss.zero_()
    scale = 1.0 / (3.0 * R)
    nerf.sample(ro, rd, R)
    nerf.field_fwd(sun)
    nerf.render(R, tg, scale)
    n_dev = nerf.field_bwd(R, tg, scale, sun)
    sync()
    out = dict(n=int(host(nerf.n_out)[0]), n_bwd=int(host(n_dev)[0]), loss=float(host(nerf.loss)[0]),
               rgb_out=host(nerf.rgb_out), opacity=host(nerf.opacity), depth=host(nerf.depth),
               n_alive=host(nerf.n_alive), dtable=host(nerf.g_t), dW=host(nerf.g_w))
    n, nb = out["n"], out["n_bwd"]
    out["sigma"], out["rgb"] = host(nerf.sigma)[:n], host(nerf.rgb)[:n]
    out["dsigma"], out["drgb"] = host(nerf.dsigma)[:n], host(nerf.drgb)[:n]
    # dfeat is compact over the samples kept by early stop: scatter back to [n][32]
    idx = host(nerf.alive_idx)[:nb] if w.early_stop > 0 else np.arange(nb)
    df = np.zeros((n, 32))
    W = len(nerf.res) * nerf.F
    df[idx, :W] = host(nerf.dfeat)[:, :nb, :].transpose(1, 0, 2).reshape(nb, W)
    out["dfeat"] = df
    nerf.adam()
    sync()
    out["table_new"], out["mlp_new"] = host(nerf.table), host(nerf.params)
    return out


def _rel(a, b):
    a, b = np.ravel(a).astype(np.float64), np.ravel(b).astype(np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)), \
        float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check_step(g, o, prec, w, orc):
    """FP32: values within 1e-5, gradients within 1e-4 (relative L2 over each
    tensor; elementwise against max|ref| on every sample whose ReLU decisions
    are not within rounding of a kink, and on every table entry such samples do
    not touch).  BF16: values within 1e-2, gradients within 1e-1 relative L2."""
    assert g["n"] == o["n_total"]
    for k, ref in (("dsigma", o["dsigma"]), ("drgb", o["drgb"]), ("dfeat", o["dfeat"]),
                   ("dtable", o["dtable"]), ("dW", o["dW"])):
        print("%-7s rel L2 %.3g  rel max %.3g" % ((k,) + _rel(g[k], ref)))
    if prec == "bf16":
        assert_values(np.log(g["sigma"]), np.log(o["sigma"]), 0.0, 5e-2, "log sigma")
        assert_values(g["rgb"], o["rgb"], 0.0, 1e-2, "rgb")
        assert_values(g["rgb_out"], o["comp"]["rgb"], 0.0, 1e-2, "rgb_out")
        assert_values(g["loss"], o["loss"], 1e-2, 0.0, "loss")
        for k in ("dsigma", "drgb", "dtable", "dW"):
            assert _rel(g[k], o[k])[0] < 1e-1, k
        return
    assert_values(g["sigma"], o["sigma"], 1e-5, 1e-7, "sigma")
    assert_values(g["rgb"], o["rgb"], 1e-5, 1e-7, "rgb")
    assert_values(g["rgb_out"], o["comp"]["rgb"], 1e-5, 1e-7, "rgb_out")
    assert_values(g["loss"], o["loss"], 1e-5, 0.0, "loss")
    assert_grad(g["dsigma"], o["dsigma"], 1e-4, "dsigma")
    assert_grad(g["drgb"], o["drgb"], 1e-4, "drgb")
    assert_grad(g["dW"], o["dW"], 1e-4, "dW")
    # ReLU decisions within FP32 rounding of a kink may go either way
    smp = o["sample"]
    margin = orc.mlp_margin(w.mlp, w.mlp_params, o["feat"], smp["view"], smp["ray_id"], sun=w.sun)
    amb = margin < 1e-5
    print("kink-ambiguous samples: %d of %d" % (amb.sum(), amb.size))
    assert amb.mean() < 2e-2
    ok = ~amb
    assert _rel(g["dfeat"], o["dfeat"])[0] <= 1e-4
    assert_grad(g["dfeat"][ok], o["dfeat"][ok], 1e-4, "dfeat (unambiguous samples)")
    assert _rel(g["dtable"], o["dtable"])[0] <= 1e-4
    mask = np.ones(o["dtable"].shape, dtype=bool)
    if amb.any():
        _, idx = orc.hashgrid_fwd(o["res"], w.grid.log2_table, w.table, smp["pos"][amb],
                                  smp["tile_id"][amb], 32, return_index=True)
        tid = smp["tile_id"][amb].astype(np.int64)
        for lvl in range(idx.shape[1]):
            mask[tid[:, None], lvl, idx[:, lvl, :].astype(np.int64)] = False
    assert_grad(g["dtable"][mask], o["dtable"][mask], 1e-4, "dtable (entries of unambiguous samples)")
    # Adam's first step is lr * sign(g): compare where the sign is not in doubt
    gref = o["dtable"].ravel()
    sel = (np.abs(gref) > 1e-3 * np.abs(gref).max()) & mask.ravel()
    assert_values(g["table_new"].ravel()[sel], o["table_new"].ravel()[sel], 1e-4, 1e-6, "table after Adam")
    gw = o["dW"]
    sel = np.abs(gw) > 1e-3 * np.abs(gw).max()
    assert_values(g["mlp_new"][sel], o["mlp_new"][sel], 1e-4, 1e-6, "MLP after Adam")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tiny_tile_step(orc, prec):
    w = synth.tiny_tile(seed=0)
    g = gpu_step(w, prec)
    o = orc.train_step(w)
    check_step(g, o, prec, w, orc)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_tile_step_reduced_rays(orc, prec):
    """The full-tile configuration (L=16, T=2^19, 128 samples in the band,
    early stop 1e-4, 21->64->64->4 colour net) on 1024 rays, with a random
    table and a steep density head so that early stop truncates most rays."""
    w = synth.full_tile(seed=0, n_rays=1024)
    rng = np.random.default_rng(8)
    w.table = rng.uniform(-1, 1, size=w.table.shape).astype(np.float32)
    row = slice(64 * 32, 64 * 32 + 64)                         # density-logit row
    w.mlp_params[row] = np.abs(w.mlp_params[row]) * np.float32(4.0)
    g = gpu_step(w, prec)
    assert np.sum(g["n_alive"]) < 0.9 * g["n"]               # early stop is active
    o = orc.train_step(w, alive=g["n_alive"])
    if prec == "fp32":
        ref_alive = orc.train_step(w)["n_alive"]
        assert np.mean(g["n_alive"] != ref_alive) < 0.01
    check_step(g, o, prec, w, orc)


def test_autograd_function_matches_oracle_and_fd(orc):
    from paper_2507_01631_amd import SnakeTileStep, level_resolutions
    w = synth.tiny_tile(seed=5, n_rays=1024, samples=32)
    rng = np.random.default_rng(6)
    w.table = rng.uniform(-0.5, 0.5, size=w.table.shape).astype(np.float32)
    nerf = make_nerf(w)
    table = nerf.table.requires_grad_(True)
    params = nerf.params.requires_grad_(True)
    loss = SnakeTileStep.apply(table, params, nerf, dev(w.rays_o), dev(w.rays_d), dev(w.target), None)
    loss.backward()
    sync()
    o = orc.train_step(w)
    assert abs(float(loss) - o["loss"]) <= 1e-5 * o["loss"]
    assert_grad(host(table.grad), o["dtable"], 1e-4, "dtable")
    assert_grad(host(params.grad), o["dW"], 1e-4, "dW")
    # central differences of the FP64 oracle loss, h = 1e-3
    res = level_resolutions(8, 16, 256)

    def oracle_loss(tab, par):
        s = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, w.samples_per_ray)
        f = orc.hashgrid_fwd(res, w.grid.log2_table, tab, s["pos"], None, 32)
        sg, c = orc.mlp_fwd(w.mlp, par, f, s["view"], s["ray_id"])
        return orc.composite_fwd(s["packed_info"], sg, c, s["t0"], s["t1"], w.target,
                                 1.0 / (3 * w.n_rays))["loss"]

    gt = host(table.grad).ravel()
    cand = np.nonzero(np.abs(gt) > 1e-2 * np.abs(gt).max())[0]
    pick = rng.choice(cand, size=min(64, cand.size), replace=False)
    bad = 0
    for i in pick:
        tp, tm = w.table.copy().ravel(), w.table.copy().ravel()
        tp[i] += np.float32(1e-3)
        tm[i] -= np.float32(1e-3)
        fd = (oracle_loss(tp.reshape(w.table.shape), w.mlp_params)
              - oracle_loss(tm.reshape(w.table.shape), w.mlp_params)) / float(tp[i] - tm[i])
        bad += abs(fd - gt[i]) > 2e-3 * np.abs(gt).max() + 1e-2 * abs(fd)
    assert bad <= 2
    gw = host(params.grad)
    cand = np.nonzero(np.abs(gw) > 1e-2 * np.abs(gw).max())[0]
    pick = rng.choice(cand, size=min(64, cand.size), replace=False)
    bad = 0
    for i in pick:
        wp, wm = w.mlp_params.copy(), w.mlp_params.copy()
        wp[i] += np.float32(1e-3)
        wm[i] -= np.float32(1e-3)
        fd = (oracle_loss(w.table, wp) - oracle_loss(w.table, wm)) / float(wp[i] - wm[i])
        bad += abs(fd - gw[i]) > 2e-3 * np.abs(gw).max() + 1e-2 * abs(fd)
    assert bad <= 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_sampled(orc, prec):
    """Full-size step (2^18 rays x 128 samples, L=16, T=2^19) in the launch
    configuration of the benchmark; outputs checked on samples the oracle can
    compute one by one."""
    w = synth.full_tile(seed=0, n_rays=1 << 18, render_targets=False)
    nerf = make_nerf(w, prec)
    ro, rd, tg, sun = dev(w.rays_o), dev(w.rays_d), dev(w.target), dev(w.sun)
    nerf.loss.zero_()
    R = w.n_rays
    scale = 1.0 / (3 * R)
    nerf.sample(ro, rd, R)
    nerf.field_fwd(sun)
    nerf.render(R, tg, scale)
    sync()
    rng = np.random.default_rng(7)
    rays = np.sort(rng.choice(R, size=512, replace=False))
    info = host(nerf.packed_info)
    o = orc.sample_segmented(w.rays_o[rays], w.rays_d[rays], w.boxes, 128, zband=w.zband)
    sel = np.concatenate([np.arange(info[r, 0], info[r, 0] + info[r, 1]) for r in rays])
    sd = torch.as_tensor(sel, device=DEV)
    assert np.array_equal(info[rays, 1], o["packed_info"][:, 1])
    assert np.array_equal(host(nerf.t0[sd]), o["t0"]) and np.array_equal(host(nerf.t1[sd]), o["t1"])
    assert np.array_equal(host(nerf.pos[sd]), o["pos"])
    assert np.array_equal(rays[o["ray_id"]], host(nerf.ray_id[sd]))
    # field on those samples
    # the BF16 form gathers from the BF16 mirror of the table
    tref = bf16_round(w.table) if nerf.table_bf16 else w.table
    feat = orc.hashgrid_fwd(nerf.res, w.grid.log2_table, tref, o["pos"], None, 32)
    gf = host(nerf.feat[:, sd, :]).transpose(1, 0, 2).reshape(sel.size, -1)
    vt = 1e-2 if prec == "bf16" else 1e-5
    assert_values(gf, feat, 2 ** -8 if prec == "bf16" else 1e-5, 1e-7, "feat")
    s_ref, c_ref = orc.mlp_fwd(w.mlp, w.mlp_params, feat, o["view"], o["ray_id"], sun=w.sun[rays])
    sig, rgb = host(nerf.sigma[sd]), host(nerf.rgb[sd])
    assert_values(sig, s_ref, vt, vt * 1e-2, "sigma")
    assert_values(rgb, c_ref, vt, vt * 1e-2, "rgb")
    comp = orc.composite_fwd(o["packed_info"], sig, rgb, o["t0"], o["t1"], alive=host(nerf.n_alive)[rays])
    assert_values(host(nerf.rgb_out)[rays], comp["rgb"], 1e-5, 1e-7, "rgb_out")
    # the adjoint at full size: properties that hold at any size
    n_dev = nerf.field_bwd(R, tg, scale, sun)
    sync()
    nb = int(host(n_dev)[0])
    assert nb == int(host(nerf.n_alive).astype(np.int64).sum())
    assert bool(torch.isfinite(nerf.g_t).all()) and bool(torch.isfinite(nerf.g_w).all())
    # trilinear weights sum to 1, so each level's table gradient sums to the
    # sum of that level's feature gradients over the samples
    for lvl in (0, 7, 15):
        got = nerf.g_t[0, lvl].double().sum(0)
        d = nerf.dfeat[lvl, :nb].double()
        ref = d.sum(0)
        tol = 2e-3 * ref.abs() + 1e-6 * d.abs().sum(0)
        assert bool(((got - ref).abs() <= tol).all()), (lvl, host(got), host(ref))


def test_tiny_tile_step_with_occupancy_culling(orc):
    """Samples in unoccupied cells of a 32^3 grid are culled before the field:
    the whole FP32 step matches the oracle step that culls with the same grid."""
    w = synth.tiny_tile(seed=7)
    G = 32
    rng = np.random.default_rng(31)
    occ = rng.random(G ** 3) < 0.5
    g = gpu_step(w, "fp32", occupancy=(G, occ))
    o = orc.train_step(w, occupancy=(G, occ))
    assert 0 < o["sample"]["n"] < o["sample_raw"]["n"]
    check_step(g, o, "fp32", w, orc)


def test_occupancy_update_from_the_field(orc):
    """update_occupancy evaluates the density networks at the cell centres:
    the decayed maxima match the oracle's sigma there (FP32 tolerance)."""
    w = synth.tiny_tile(seed=8)
    G = 16
    nerf = make_nerf(w, "fp32", occ_grid=G)
    nerf.update_occupancy()
    nerf.update_occupancy()
    sync()
    pos, _ = orc.occupancy_cell_centres(G)
    feat = orc.hashgrid_fwd(orc.level_resolutions(8, 16, 256), 14, w.table, pos)
    sig, _ = orc.mlp_fwd(w.mlp, w.mlp_params, feat, np.array([[0.0, 0.0, -1.0]], np.float32),
                         np.zeros(G ** 3, np.int32))
    # the grid starts at zero: after two updates it holds sigma * step
    ref = np.maximum(sig * nerf.occ_step * 0.95, sig * nerf.occ_step)
    assert_values(host(nerf.occ_density), ref, 1e-5, 1e-9, "occupancy density")
    frac = nerf.occupied_fraction()
    mean_occ = (ref > min(0.01, ref.mean())).mean()
    assert abs(frac - mean_occ) < 0.01, (frac, mean_occ)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_step_with_no_samples(orc, prec):
    """Every ray misses the tile: no samples anywhere in the step.  The
    composite is the background 0, the loss is the targets' mean square, all
    gradients are zero and Adam leaves the table and the networks unchanged
    (the full-tile shapes and launch configuration, early stop on)."""
    w = synth.full_tile(seed=0, n_rays=2048, render_targets=False)
    w.rays_o = np.tile([5.0, 5.0, 2.0], (w.n_rays, 1))
    w.rays_d = np.tile([0.0, 0.0, -1.0], (w.n_rays, 1))
    nerf = make_nerf(w, prec)
    g = gpu_step(w, prec)
    assert g["n"] == 0 and g["n_bwd"] == 0
    assert np.all(g["rgb_out"] == 0.0) and np.all(g["opacity"] == 0.0)
    ref_loss = float(np.sum(w.target.astype(np.float64) ** 2) / (3.0 * w.n_rays))
    assert_values(g["loss"], ref_loss, 1e-5, 0.0, "loss")
    assert not np.any(g["dtable"]) and not np.any(g["dW"])
    assert np.array_equal(g["table_new"], host(nerf.table)) and np.array_equal(g["mlp_new"], host(nerf.params))
    from paper_2507_01631_amd import _lib as L
    assert L.snake_check_device_error() == 0
