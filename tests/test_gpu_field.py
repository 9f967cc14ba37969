"""GPU parity of the hash encoding and the density/colour networks against the
FP64 oracle: hash indices bit for bit, features and network outputs within
the FP32 (1e-5) or BF16 (1e-2) tolerance, gradients within 1e-4 (FP32) or
3e-2 (BF16)."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, assert_binned_bound, assert_grad, binned_floor, assert_values, bf16_round, dev, host, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2507_01631_amd import _lib
    _lib.lib()
    return _lib


GRIDS = {
    "tiny": dict(L=8, F=2, log2T=14, lo=16, hi=256),
    "full": dict(L=16, F=2, log2T=19, lo=16, hi=2048),
    "f1": dict(L=12, F=1, log2T=12, lo=4, hi=600),
    "f4": dict(L=4, F=4, log2T=10, lo=8, hi=64),
}


def _positions(rng, n):
    p = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    p[:6] = [[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [1, 0, 1], [np.float32(1) - np.float32(6e-8), 0.25, 0.75],
             [0.0625, 0.125, 0.999]]
    return p


def _grid_setup(L, orc, name, rng, K=1):
    c = GRIDS[name]
    res = orc.level_resolutions(c["L"], c["lo"], c["hi"])
    table = rng.uniform(-1, 1, size=(K, c["L"], 1 << c["log2T"], c["F"])).astype(np.float32)
    return c, res, table


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("bf16", [False, True])
def test_hashgrid_fwd(L, orc, name, bf16):
    rng = np.random.default_rng(10)
    n = 20011
    K = 2 if name == "tiny" else 1
    c, res, table = _grid_setup(L, orc, name, rng, K)
    pos = _positions(rng, n)
    tid = rng.integers(0, K, size=n).astype(np.uint8) if K > 1 else None
    g = L.grid_desc(res, c["F"], c["log2T"], L.SNAKE_BF16 if bf16 else L.SNAKE_F32)
    feat = torch.zeros((c["L"], n, c["F"]), dtype=torch.bfloat16 if bf16 else torch.float32, device=DEV)
    idx = torch.zeros((n, c["L"], 8), dtype=torch.int32, device=DEV)
    L.snake_hashgrid_fwd(g, K, dev(table), dev(pos), None if tid is None else dev(tid), None, n, None, feat,
                         idx)
    sync()
    ref, ridx = orc.hashgrid_fwd(res, c["log2T"], table, pos, tid, 32, return_index=True)
    assert np.array_equal(host(idx).astype(np.uint32), ridx)
    got = host(feat).transpose(1, 0, 2).reshape(n, -1)
    W = c["L"] * c["F"]
    if bf16:
        assert_values(got, ref[:, :W], rel=2 ** -8, abs_=1e-6, what="feat bf16")
    else:
        assert_values(got, ref[:, :W], rel=1e-5, abs_=1e-6, what="feat")


def test_convert_bf16_matches_torch(L):
    """The table mirror: round to nearest even, bit for bit against torch's
    conversion, over random values, ties, subnormals, infinities and NaN."""
    rng = np.random.default_rng(12)
    with np.errstate(over="ignore", under="ignore"):
        x = (rng.standard_normal(40000) * 10.0 ** rng.integers(-42, 39, 40000)).astype(np.float32)
    bits = rng.integers(0, 2 ** 32, size=4000, dtype=np.uint64).astype(np.uint32)
    ties = (rng.integers(0, 2 ** 16, size=4000).astype(np.uint32) << 16) | np.uint32(0x8000)
    special = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 3.4e38, -3.4e38, 1e-40, -1e-40, 1e-45],
                       np.float32)
    x = np.concatenate([x, bits.view(np.float32), ties.view(np.float32), special])
    x = x[: x.size // 4 * 4]
    out = torch.empty(x.size, dtype=torch.bfloat16, device=DEV)
    L.snake_convert_bf16(dev(x), x.size, out)
    sync()
    got = out.cpu().view(torch.int16).numpy().view(np.uint16)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.all((got[nan] & 0x7f80) == 0x7f80) and np.all((got[nan] & 0x7f) != 0)


@pytest.mark.parametrize("name", ["tiny", "full", "f1", "f4"])
@pytest.mark.parametrize("bf16", [False, True])
def test_hashgrid_fwd_bf16_table(L, orc, name, bf16):
    """Gathers from the BF16 mirror: the same corner slots, and features equal
    the oracle's on the BF16-rounded table (the blend itself stays FP32)."""
    rng = np.random.default_rng(13)
    n = 20011
    K = 2 if name == "tiny" else 1
    c, res, table = _grid_setup(L, orc, name, rng, K)
    pos = _positions(rng, n)
    tid = rng.integers(0, K, size=n).astype(np.uint8) if K > 1 else None
    g = L.grid_desc(res, c["F"], c["log2T"], L.SNAKE_BF16 if bf16 else L.SNAKE_F32, L.SNAKE_GRID_TABLE_BF16)
    th = torch.empty(table.shape, dtype=torch.bfloat16, device=DEV)
    L.snake_convert_bf16(dev(table), table.size, th)
    feat = torch.zeros((c["L"], n, c["F"]), dtype=torch.bfloat16 if bf16 else torch.float32, device=DEV)
    idx = torch.zeros((n, c["L"], 8), dtype=torch.int32, device=DEV)
    L.snake_hashgrid_fwd(g, K, th, dev(pos), None if tid is None else dev(tid), None, n, None, feat, idx)
    sync()
    ref, ridx = orc.hashgrid_fwd(res, c["log2T"], bf16_round(table), pos, tid, 32, return_index=True)
    assert np.array_equal(host(idx).astype(np.uint32), ridx)
    got = host(feat).transpose(1, 0, 2).reshape(n, -1)
    W = c["L"] * c["F"]
    if bf16:
        assert_values(got, ref[:, :W], rel=2 ** -8, abs_=1e-6, what="feat bf16 (bf16 table)")
    else:
        assert_values(got, ref[:, :W], rel=1e-5, abs_=1e-6, what="feat (bf16 table)")


def test_hashgrid_fwd_superchunk_order(L, orc):
    """The forward's work order (level by level over all samples, or
    super-chunks of 2^20 samples with every level of one before the next)
    changes nothing: the same bits, with a partial last super-chunk."""
    rng = np.random.default_rng(14)
    c, res, table = _grid_setup(L, orc, "full", rng)
    n = 3 * (1 << 20) + 4097
    pos = _ray_positions(rng, n)
    g = L.grid_desc(res, c["F"], c["log2T"], L.SNAKE_BF16)
    outs = []
    saved = L.snake_tune_get("hash_fwd_superchunk")
    try:
        for v in (0, 1, 2):
            L.snake_tune_set("hash_fwd_superchunk", v)
            feat = torch.empty((c["L"], n, c["F"]), dtype=torch.bfloat16, device=DEV)
            L.snake_hashgrid_fwd(g, 1, dev(table), dev(pos), None, None, n, None, feat, None)
            outs.append(feat)
        sync()
    finally:
        L.snake_tune_set("hash_fwd_superchunk", saved)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    sel = rng.choice(n, size=2000, replace=False)
    ref = orc.hashgrid_fwd(res, c["log2T"], table, pos[sel], None, 32)
    got = host(outs[0][:, torch.as_tensor(sel, device=DEV), :]).transpose(1, 0, 2).reshape(sel.size, -1)
    assert_values(got, ref, 2 ** -8, 1e-6, "feat (sampled)")


@pytest.mark.parametrize("name", ["tiny", "full", "f1", "f4"])
@pytest.mark.parametrize("table_bf16", [False, True])
def test_hashgrid_fwd_lds_path_matches_cache_path(L, orc, name, table_bf16):
    """Levels whose slice fits in LDS are gathered from an LDS copy unless the
    hash_fwd_lds tunable is 0.  Both paths give the same bits and corner
    slots: tiles grouped in runs (as a window's partition leaves them, with
    runs ending inside a block's samples), in random order, an id past the
    last tile, an index array and a device count below the host bound, over
    several blocks of samples and a ragged tail; sampled features against the
    oracle."""
    rng = np.random.default_rng(19)
    K = 3
    c, res, table = _grid_setup(L, orc, name, rng, K)
    n = 5 * 4096 + 1234
    pos = _ray_positions(rng, n)
    runs = np.repeat(np.arange(K), [6000, 9000, n - 15000]).astype(np.uint8)
    rand = rng.integers(0, K, size=n).astype(np.uint8)
    rand[::101] = K                                  # no such tile
    sel = rng.permutation(n).astype(np.int32)
    flags = L.SNAKE_GRID_TABLE_BF16 if table_bf16 else 0
    g = L.grid_desc(res, c["F"], c["log2T"], L.SNAKE_BF16, flags)
    if table_bf16:
        tab = torch.empty(table.shape, dtype=torch.bfloat16, device=DEV)
        L.snake_convert_bf16(dev(table), table.size, tab)
        reft = bf16_round(table)
    else:
        tab, reft = dev(table), table
    nd = torch.tensor([n - 777], dtype=torch.int64, device=DEV)
    cases = [(runs, None, None), (rand, None, None), (runs, sel, nd)]
    saved = L.snake_tune_get("hash_fwd_lds")
    try:
        for tid, idxs, ndev in cases:
            outs = []
            for v in (0, 1):
                L.snake_tune_set("hash_fwd_lds", v)
                feat = torch.full((c["L"], n, c["F"]), 3.0, dtype=torch.bfloat16, device=DEV)
                idx = torch.zeros((n, c["L"], 8), dtype=torch.int32, device=DEV)
                L.snake_hashgrid_fwd(g, K, tab, dev(pos), dev(tid), None if idxs is None else dev(idxs), n, ndev,
                                     feat, idx)
                outs.append((feat, idx))
            sync()
            assert torch.equal(outs[0][0], outs[1][0])
            assert torch.equal(outs[0][1], outs[1][1])
            ne = n if ndev is None else n - 777
            s = rng.choice(ne, size=1500, replace=False)
            src = s if idxs is None else idxs[s]
            ok = tid[src] < K
            ref = orc.hashgrid_fwd(res, c["log2T"], reft, pos[src[ok]], tid[src[ok]], 32)
            got = host(outs[1][0][:, torch.as_tensor(s[ok], device=DEV), :]).transpose(1, 0, 2).reshape(ok.sum(), -1)
            assert_values(got, ref[:, :c["L"] * c["F"]], 2 ** -8, 1e-6, "feat (sampled, %s)" % name)
            assert np.all(host(outs[1][0][:, torch.as_tensor(s[~ok], device=DEV), :]) == 0.0)
    finally:
        L.snake_tune_set("hash_fwd_lds", saved)
    L.snake_check_device_error()


def test_hashgrid_fwd_indexed_and_device_count(L, orc):
    rng = np.random.default_rng(11)
    c, res, table = _grid_setup(L, orc, "full", rng)
    N = 9000
    pos = _positions(rng, N)
    sel = rng.choice(N, size=5000, replace=False).astype(np.int32)
    g = L.grid_desc(res, c["F"], c["log2T"])
    n_host = 6000                       # host bound; device count says 4321
    nd = torch.tensor([4321], dtype=torch.int64, device=DEV)
    feat = torch.full((c["L"], n_host, c["F"]), 7.0, device=DEV)
    L.snake_hashgrid_fwd(g, 1, dev(table), dev(pos), None, dev(np.pad(sel, (0, 1000)), torch.int32), n_host,
                         nd, feat, None)
    sync()
    got = host(feat).transpose(1, 0, 2).reshape(n_host, -1)
    ref = orc.hashgrid_fwd(res, c["log2T"], table, pos[sel[:4321]], None, 32)
    assert_values(got[:4321], ref, rel=1e-5, abs_=1e-6, what="indexed feat")
    assert np.all(got[4321:] == 7.0)     # untouched past the device count


@pytest.mark.parametrize("name", ["tiny", "full", "f1", "f4"])
@pytest.mark.parametrize("mode", ["atomic", "binned", "binned-1level"])
def test_hashgrid_bwd(L, orc, name, mode):
    rng = np.random.default_rng(12)
    n = 30001
    K = 2 if name == "tiny" else 1
    c, res, table = _grid_setup(L, orc, name, rng, K)
    pos = _positions(rng, n)
    tid = rng.integers(0, K, size=n).astype(np.uint8) if K > 1 else None
    W = c["L"] * c["F"]
    dfeat = rng.normal(size=(n, W))
    dfeat[::7] = 0.0                     # zero-gradient samples are skipped
    g = L.grid_desc(res, c["F"], c["log2T"])
    dtab = torch.zeros(table.shape, device=DEV)
    dfd = dev(dfeat.reshape(n, c["L"], c["F"]).transpose(1, 0, 2).astype(np.float32))
    ws = None
    if mode != "atomic":
        lg = 1 if mode == "binned-1level" else c["L"]
        ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, K, n, lg), dtype=torch.uint8, device=DEV)
    L.snake_hashgrid_bwd(g, K, dev(pos), None if tid is None else dev(tid), None, n, None, dfd, dtab, ws)
    sync()
    assert L.snake_check_device_error() == 0
    dpad = np.zeros((n, 32))
    dpad[:, :W] = dfeat.astype(np.float32)
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, dpad, tid)
    assert_grad(host(dtab), ref, 1e-4, "dtable")


# ---------------------------------------------------------------------------
MLPS = {
    "tiny": (synth.MlpConfig(feat_real=16, n_dir=3, colour_layers=1, colour_out=3), 8, 2),
    "full": (synth.MlpConfig(feat_real=32, n_dir=6, colour_layers=2, colour_out=4), 16, 2),
}


def _mlp_inputs(rng, cfg, Lv, F, n, R, wscale=2.0):
    w = synth.init_mlp(rng, cfg) * np.float32(wscale)
    feat = rng.normal(scale=0.7, size=(n, Lv * F)).astype(np.float32)
    view = rng.normal(size=(R, 3)).astype(np.float32)
    view /= np.linalg.norm(view, axis=1, keepdims=True)
    sun = rng.normal(size=(R, 3)).astype(np.float32)
    rid = rng.integers(0, R, size=n).astype(np.int32)
    return w, feat, view, sun, rid


def _pad32(f):
    out = np.zeros((f.shape[0], 32))
    out[:, :f.shape[1]] = f
    return out


@pytest.mark.parametrize("name", list(MLPS))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mlp_fwd(L, orc, name, prec):
    rng = np.random.default_rng(13)
    cfg, Lv, F = MLPS[name]
    n, R = 5003, 701
    bf = prec == "bf16"
    # BF16 is checked at the Xavier scale the networks are initialised with
    w, feat, view, sun, rid = _mlp_inputs(rng, cfg, Lv, F, n, R, 1.0 if bf else 2.0)
    m = L.mlp_desc(Lv, F, cfg.n_dir, cfg.colour_layers, cfg.colour_out,
                   L.SNAKE_BF16 if bf else L.SNAKE_F32, L.SNAKE_F32)
    fd = dev(feat.reshape(n, Lv, F).transpose(1, 0, 2))
    sigma = torch.zeros(n, device=DEV)
    rgb = torch.zeros((n, 3), device=DEV)
    L.snake_mlp_fwd(m, dev(w), fd, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), R, None, n,
                    None, sigma, rgb)
    sync()
    rs, rc = orc.mlp_fwd(cfg, w, _pad32(feat), view, rid, sun=sun if cfg.n_dir == 6 else None)
    if bf:
        # sigma = exp(o_0): the logit's bf16 error is absolute, so compare log sigma
        assert_values(np.log(host(sigma)), np.log(rs), rel=0.0, abs_=2e-2, what="log sigma")
        assert_values(host(rgb), rc, rel=0.0, abs_=1e-2, what="rgb")
        # against the same rounding points emulated in FP64: only FP32 summation
        # order differs, except where it tips an intermediate to the next bf16
        es, ec = orc.mlp_fwd_bf16emu(cfg, w, _pad32(feat), view, rid, sun=sun if cfg.n_dir == 6 else None)
        d_rgb = np.abs(host(rgb) - ec).max(axis=1)
        d_sig = np.abs(np.log(host(sigma)) - np.log(es))
        assert np.mean(d_rgb > 1e-5) < 0.05 and d_rgb.max() < 5e-3, (np.mean(d_rgb > 1e-5), d_rgb.max())
        assert np.mean(d_sig > 1e-5) < 0.05 and d_sig.max() < 5e-3, (np.mean(d_sig > 1e-5), d_sig.max())
    else:
        assert_values(host(sigma), rs, rel=1e-5, abs_=1e-7, what="sigma")
        assert_values(host(rgb), rc, rel=1e-5, abs_=1e-7, what="rgb")


@pytest.mark.parametrize("name", list(MLPS))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mlp_bwd(L, orc, name, prec):
    rng = np.random.default_rng(14)
    cfg, Lv, F = MLPS[name]
    N, R = 7000, 900
    w, feat, view, sun, rid = _mlp_inputs(rng, cfg, Lv, F, N, R)
    ds = rng.normal(size=N).astype(np.float32)
    dr = rng.normal(size=(N, 3)).astype(np.float32)
    sel = np.sort(rng.choice(N, size=4099, replace=False)).astype(np.int32)
    n = sel.size
    bf = prec == "bf16"
    m = L.mlp_desc(Lv, F, cfg.n_dir, cfg.colour_layers, cfg.colour_out,
                   L.SNAKE_BF16 if bf else L.SNAKE_F32, L.SNAKE_F32)
    fd = dev(feat.reshape(N, Lv, F).transpose(1, 0, 2))
    dW = torch.zeros(w.size, device=DEV)
    dfeat = torch.zeros((Lv, n, F), device=DEV)
    ws = torch.empty(L.snake_mlp_bwd_workspace_bytes(m), dtype=torch.uint8, device=DEV)
    L.snake_mlp_bwd(m, dev(w), fd, N, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), R,
                    dev(sel), n, None, dev(ds), dev(dr), dW, dfeat, ws)
    sync()
    rW, rf = orc.mlp_bwd(cfg, w, _pad32(feat[sel]), view, rid[sel], ds[sel], dr[sel],
                         sun=sun if cfg.n_dir == 6 else None)
    tol = 3e-2 if bf else 1e-4
    assert_grad(host(dW), rW, tol, "dW")
    got_f = host(dfeat).transpose(1, 0, 2).reshape(n, -1)
    assert_grad(got_f, rf[:, :Lv * F], tol, "dfeat")
    # the sum is deterministic: a second call adds exactly the same values
    dW2 = dW.clone()
    L.snake_mlp_bwd(m, dev(w), fd, N, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), R,
                    dev(sel), n, None, dev(ds), dev(dr), dW2, dfeat, ws)
    sync()
    assert torch.equal(dW2 - dW, dW)
    # stored activations (forward over all N samples, adjoint reads them through
    # the index list) give bit-identical gradients to recomputation
    act = torch.empty((N, L.snake_mlp_act_width(m)), device=DEV)
    sig, rgb = torch.empty(N, device=DEV), torch.empty((N, 3), device=DEV)
    L.snake_mlp_fwd(m, dev(w), fd, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), R, None, N,
                    None, sig, rgb, act=act)
    dW3 = torch.zeros_like(dW)
    dfeat3 = torch.zeros_like(dfeat)
    L.snake_mlp_bwd(m, dev(w), fd, N, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), R,
                    dev(sel), n, None, dev(ds), dev(dr), dW3, dfeat3, ws, act=act)
    sync()
    assert torch.equal(dW3, dW)
    assert torch.equal(dfeat3, dfeat)


def test_hashgrid_bwd_binned_indexed_ray_ordered(L, orc):
    """Binned adjoint on sampler-ordered positions (long runs of equal slots on
    coarse levels) read through an index list, with a device count."""
    import synth as sy
    rng = np.random.default_rng(15)
    w = sy.full_tile(seed=2, n_rays=300, render_targets=False)
    s = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 128, zband=w.zband)
    c, res, table = _grid_setup(L, orc, "full", rng)
    N = s["n"]
    sel = np.sort(rng.choice(N, size=N // 2, replace=False)).astype(np.int32)
    n = sel.size
    dfeat = rng.normal(size=(n, 32)).astype(np.float32)
    g = L.grid_desc(res, 2, c["log2T"])
    dtab = torch.zeros(table.shape, device=DEV)
    ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, 1, n + 100, 5), dtype=torch.uint8, device=DEV)
    nd = torch.tensor([n], dtype=torch.int64, device=DEV)
    dfd = torch.zeros((16, n + 100, 2), device=DEV)
    dfd[:, :n, :] = dev(dfeat.reshape(n, 16, 2).transpose(1, 0, 2))
    L.snake_hashgrid_bwd(g, 1, dev(s["pos"]), None, dev(np.pad(sel, (0, 100))), n + 100, nd, dfd, dtab, ws)
    sync()
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, s["pos"][sel], dfeat.astype(np.float64))
    assert_grad(host(dtab), ref, 1e-4, "dtable")


def test_hashgrid_bwd_workspace_too_small(L):
    g = L.grid_desc([16, 32], 2, 14)
    need = L.snake_hashgrid_bwd_workspace_bytes(g, 1, 1000, 1)
    ws = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    with pytest.raises(L.SnakeError):
        L.snake_hashgrid_bwd(g, 1, torch.zeros((1000, 3), device=DEV), None, None, 1000, None,
                             torch.zeros((2, 1000, 2), device=DEV), torch.zeros((1, 2, 1 << 14, 2), device=DEV),
                             ws)


def test_bad_tile_and_ray_ids_are_dropped_and_flagged(L, orc):
    """Out-of-range ids from the device never index out of bounds: the sample
    is dropped and a device error bit is raised."""
    rng = np.random.default_rng(18)
    c, res, table = _grid_setup(L, orc, "tiny", rng, K=2)
    n = 1000
    pos = _positions(rng, n)
    tid = rng.integers(0, 2, size=n).astype(np.uint8)
    tid[::97] = 7                                   # no tile 7
    g = L.grid_desc(res, 2, c["log2T"])
    L.snake_check_device_error()
    feat = torch.full((8, n, 2), 5.0, device=DEV)
    L.snake_hashgrid_fwd(g, 2, dev(table), dev(pos), dev(tid), None, n, None, feat)
    sync()
    f = host(feat)
    assert np.all(f[:, ::97, :] == 0.0) and np.all(f[:, 1::97, :] != 5.0)
    assert L.snake_check_device_error() & L.SNAKE_DEVERR_TILE_ID
    dtab = torch.zeros(table.shape, device=DEV)
    ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, 2, n, 8), dtype=torch.uint8, device=DEV)
    L.snake_hashgrid_bwd(g, 2, dev(pos), dev(tid), None, n, None, torch.ones((8, n, 2), device=DEV), dtab, ws)
    sync()
    ok = tid < 2
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos[ok], np.ones((ok.sum(), 32)), tid[ok])
    ref[:, :, :, :] *= 1.0
    assert_grad(host(dtab), ref, 1e-4, "dtable without the bad samples")
    assert L.snake_check_device_error() & L.SNAKE_DEVERR_TILE_ID
    # MLP: ray ids outside [0, R)
    cfg, Lv, F = MLPS["tiny"]
    w, fe, view, sun, rid = _mlp_inputs(rng, cfg, Lv, F, 256, 50)
    rid[::9] = 50
    m = L.mlp_desc(Lv, F, 3, 1, 3)
    sig = torch.full((256,), 3.0, device=DEV)
    rgb = torch.full((256, 3), 3.0, device=DEV)
    L.snake_mlp_fwd(m, dev(w), dev(fe.reshape(256, Lv, F).transpose(1, 0, 2)), dev(view), None, dev(rid), 50,
                    None, 256, None, sig, rgb)
    sync()
    assert np.all(host(sig)[::9] == 0) and np.all(host(rgb)[::9] == 0) and np.all(host(sig)[1::9] > 0)
    assert L.snake_check_device_error() & L.SNAKE_DEVERR_RAY_ID


@pytest.mark.parametrize("shared", [0, 1])
@pytest.mark.parametrize("name", list(MLPS))
def test_mlp_per_tile_weights(L, orc, name, shared):
    """Window form: K = 4 weight sets selected by each sample's tile after the
    tile partition, with uneven group sizes (one empty), 16-sample tiles that
    would straddle groups, and a few invalid tile ids (dropped: sigma = rgb = 0,
    dfeat = 0).  Each group matches the oracle run on its own samples with its
    own weights; dW is [K][P].  With a shared colour net the weights are the
    four density sets then one colour set, and the colour gradient sums over
    the tiles."""
    rng = np.random.default_rng(77)
    cfg, Lv, F = MLPS[name]
    K, n, R = 4, 6007, 900
    P = orc.mlp_param_count(cfg)
    ws_ = [synth.init_mlp(rng, cfg) * np.float32(2.0) for _ in range(K)]
    W = np.stack(ws_)
    _, feat, view, sun, rid = _mlp_inputs(rng, cfg, Lv, F, n, R)
    tid = rng.choice([0, 1, 3], size=n, p=[0.6, 0.3, 0.1]).astype(np.uint8)   # group 2 empty
    tid[::611] = 9
    sun_d = dev(sun) if cfg.n_dir == 6 else None
    # partition on the GPU, then run the networks in the partitioned order
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    ts = torch.empty(K + 2, dtype=torch.int64, device=DEV)
    rs = torch.empty(n, dtype=torch.int32, device=DEV)
    pws = torch.empty(L.snake_tile_partition_workspace_bytes(K), dtype=torch.uint8, device=DEV)
    L.snake_check_device_error()
    L.snake_tile_partition(dev(tid), None, dev(rid), n, None, K, perm, None, ts, None, None, rs, pws)
    sync()
    assert L.snake_check_device_error() & L.SNAKE_DEVERR_TILE_ID
    pm = host(perm)
    bounds = host(ts)
    fs = feat[pm]
    m = L.mlp_desc(Lv, F, cfg.n_dir, cfg.colour_layers, cfg.colour_out, shared_colour=shared)
    Pd = 64 * 32 + 16 * 64
    if shared:
        W[:, Pd:] = W[0, Pd:]                                  # one colour set for every tile
        Wg = np.concatenate([W[:, :Pd].ravel(), W[0, Pd:]])
    else:
        Wg = W.reshape(-1)
    assert Wg.size == L.snake_mlp_weight_count(m, K)
    fd = dev(fs.reshape(n, Lv, F).transpose(1, 0, 2))
    sig = torch.full((n,), 7.0, device=DEV)
    rgb = torch.full((n, 3), 7.0, device=DEV)
    L.snake_mlp_fwd(m, dev(Wg), fd, dev(view), sun_d, rs, R, None, n, None, sig, rgb, K=K,
                    tile_start=ts)
    ds = rng.normal(size=n).astype(np.float32)
    dr = rng.normal(size=(n, 3)).astype(np.float32)
    dW = torch.zeros(Wg.size, device=DEV)
    dfeat = torch.full((Lv, n, F), 7.0, device=DEV)
    wsb = torch.empty(L.snake_mlp_bwd_workspace_bytes(m, K), dtype=torch.uint8, device=DEV)
    L.snake_mlp_bwd(m, dev(Wg), fd, n, dev(view), sun_d, rs, R, None, n, None, dev(ds), dev(dr),
                    dW, dfeat, wsb, K=K, tile_start=ts)
    sync()
    g_sig, g_rgb = host(sig), host(rgb)
    g_all = host(dW)
    g_dw = np.zeros((K, P))
    if shared:
        g_dw[:, :Pd] = g_all[:K * Pd].reshape(K, Pd)
    else:
        g_dw[:] = g_all.reshape(K, P)
    r_col = np.zeros(P - Pd)
    g_df = host(dfeat).transpose(1, 0, 2).reshape(n, -1)
    for k in range(K + 1):
        sl = slice(bounds[k], bounds[k + 1])
        if k == K:
            assert np.all(g_sig[sl] == 0) and np.all(g_rgb[sl] == 0) and np.all(g_df[sl] == 0)
            assert bounds[k + 1] - bounds[k] == len(range(0, n, 611))
            continue
        if bounds[k + 1] == bounds[k]:
            assert np.all(g_dw[k] == 0)
            continue
        r_sig, r_rgb = orc.mlp_fwd(cfg, W[k], _pad32(fs[sl]), view, host(rs)[sl],
                                   sun=sun if cfg.n_dir == 6 else None)
        assert_values(g_sig[sl], r_sig, rel=1e-5, abs_=1e-7, what="sigma tile %d" % k)
        assert_values(g_rgb[sl], r_rgb, rel=1e-5, abs_=1e-7, what="rgb tile %d" % k)
        rW, rf = orc.mlp_bwd(cfg, W[k], _pad32(fs[sl]), view, host(rs)[sl], ds[sl], dr[sl],
                             sun=sun if cfg.n_dir == 6 else None)
        if shared:
            assert_grad(g_dw[k, :Pd], rW[:Pd], 1e-4, "density dW tile %d" % k)
            r_col += rW[Pd:]
        else:
            assert_grad(g_dw[k], rW, 1e-4, "dW tile %d" % k)
        assert_grad(g_df[sl], rf[:, :Lv * F], 1e-4, "dfeat tile %d" % k)
    assert bounds[3] == bounds[2]
    if shared:
        assert_grad(g_all[K * Pd:], r_col, 1e-4, "shared colour dW")


def _ray_positions(rng, n, per_ray=128):
    """Positions of consecutive samples along straight rays through the unit
    cube (the sampler's order), so that neighbouring samples share cells on
    the coarse levels; a ragged last ray."""
    r = (n + per_ray - 1) // per_ray
    a = rng.uniform(0, 1, size=(r, 1, 3))
    b = rng.uniform(0, 1, size=(r, 1, 3))
    t = ((np.arange(per_ray) + 0.5) / per_ray)[None, :, None]
    return (a + t * (b - a)).reshape(-1, 3)[:n].astype(np.float32)


def _heavy_tailed(rng, n, W):
    """Feature gradients spread over many decades, like transmittance-weighted
    gradients behind an opaque surface: log-normal magnitudes (sigma 3, so the
    largest of a million values is about 2^22 times the median), random
    signs, a tenth of the samples zero."""
    g = rng.lognormal(0.0, 3.0, size=(n, W)) * rng.choice([-1.0, 1.0], size=(n, W))
    g[rng.random(n) < 0.1] = 0.0
    return g.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("name", ["full", "tiny"])
def test_hashgrid_bwd_binned_heavy_tailed(L, orc, name):
    """Heavy-tailed feature gradients (log-normal, sigma 3) on ray-ordered
    samples: the binned adjoint matches the FP64 oracle per tensor (1e-4
    relative L2), per element against max|ref| (1e-4) and per element within
    its own rounding bound; no entry larger than that bound loses its sign,
    and nearly every entry is within 1e-4 of its own value (only entries whose
    contributions cancel to far below their absolute sum can lose more, as in
    any summation)."""
    rng = np.random.default_rng(29)
    n = 1 << 21
    c, res, table = _grid_setup(L, orc, name, rng)
    W = c["L"] * c["F"]
    pos = _ray_positions(rng, n)
    dfeat = _heavy_tailed(rng, n, W)
    g = L.grid_desc(res, c["F"], c["log2T"])
    dfd = dev(dfeat.reshape(n, c["L"], c["F"]).transpose(1, 0, 2).astype(np.float32))
    ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, 1, n, c["L"]), dtype=torch.uint8, device=DEV)
    dtab = torch.zeros(table.shape, device=DEV)
    L.snake_hashgrid_bwd(g, 1, dev(pos), None, None, n, None, dfd, dtab, ws)
    sync()
    assert L.snake_check_device_error() == 0
    dpad = np.zeros((n, 32))
    dpad[:, :W] = dfeat
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, dpad)
    absref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, np.abs(dpad))
    got = host(dtab)
    assert_grad(got, ref, 1e-4, "dtable (heavy-tailed)")
    floor = binned_floor(orc, res, c["log2T"], pos, dfeat, c["F"])[None]
    lim = assert_binned_bound(got, ref, absref, floor, "dtable (heavy-tailed)").reshape(ref.shape)
    # every entry larger than its error bound keeps its sign
    big = np.abs(ref) > lim
    assert np.all(np.sign(got[big]) == np.sign(ref[big])), "sign lost"
    # entries down to 2^-30 of the largest: the 20-bit values and exact sums
    # keep nearly all of them within 1e-4 of their own value
    nz = np.abs(ref) > 2.0 ** -30 * np.abs(ref).max()
    rel = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    print("heavy-tailed %s: %d entries above 2^-30 of the largest, rel err median %.2e, 99.9%% %.2e, max %.2e, "
          ">1e-4: %.2e; %d entries at the absolute floor" % (name, nz.sum(), np.median(rel), np.quantile(rel, 0.999),
                                                           rel.max(), np.mean(rel > 1e-4), int((~big).sum())))
    assert np.mean(rel > 1e-4) < 1e-2
    # the FP32-atomic form on the same input, for comparison (its order, hence
    # its last bits, vary from run to run)
    dtab.zero_()
    L.snake_hashgrid_bwd(g, 1, dev(pos), None, None, n, None, dfd, dtab, None)
    sync()
    ga = host(dtab)
    rela = np.abs(ga[nz] - ref[nz]) / np.abs(ref[nz])
    print("heavy-tailed %s, FP32 atomics: rel L2 %.2e, rel err median %.2e, 99.9%% %.2e, max %.2e, >1e-4: %.2e" % (
        name, np.linalg.norm(ga - ref) / np.linalg.norm(ref), np.median(rela), np.quantile(rela, 0.999), rela.max(),
        np.mean(rela > 1e-4)))
    print("heavy-tailed %s, binned: rel L2 %.2e" % (name, np.linalg.norm(got - ref) / np.linalg.norm(ref)))


def test_hashgrid_bwd_binned_is_deterministic(L, orc):
    """The binned adjoint sums exactly in integers, and its count/scatter blocks
    take whole 64-sample wavefronts (so runs merge the same way), so the grid
    shape and the number of levels per pass change nothing: the same bits
    every time.  Its rounding stays within the oracle bound."""
    rng = np.random.default_rng(19)
    n = 200_003
    c, res, table = _grid_setup(L, orc, "full", rng)
    pos = _positions(rng, n)
    pos[n // 2:] = _ray_positions(rng, n - n // 2)   # runs of equal slots on the coarse levels
    dfeat = (rng.normal(size=(n, 32)) * rng.uniform(0, 3, size=(n, 1))).astype(np.float32)
    g = L.grid_desc(res, 2, c["log2T"])
    dfd = dev(dfeat.reshape(n, 16, 2).transpose(1, 0, 2))
    ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, 1, n, 16), dtype=torch.uint8, device=DEV)
    saved = {k: L.snake_tune_get(k) for k in ("bin_blocks", "bin_levels_per_pass")}
    outs = []
    try:
        for blocks, lg in ((2048, 0), (1024, 0), (256, 0), (512, 3), (64, 1)):
            L.snake_tune_set("bin_blocks", blocks)
            L.snake_tune_set("bin_levels_per_pass", lg)
            dtab = torch.zeros(table.shape, device=DEV)
            L.snake_hashgrid_bwd(g, 1, dev(pos), None, None, n, None, dfd, dtab, ws)
            outs.append(dtab)
        sync()
    finally:
        for k, v in saved.items():
            L.snake_tune_set(k, v)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, dfeat.astype(np.float64))
    assert_grad(host(outs[0]), ref, 1e-4, "dtable")
    absref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, np.abs(dfeat.astype(np.float64)))
    floor = binned_floor(orc, res, c["log2T"], pos, dfeat.astype(np.float64), 2)[None]
    assert_binned_bound(host(outs[0]), ref, absref, floor, "dtable")


@pytest.mark.parametrize("lg", [1, 3, 0])
def test_hashgrid_bwd_binned_nonfinite_level_adds_nothing(L, orc, lg):
    """A level whose feature gradient holds an inf or a NaN leaves its table
    gradient untouched and raises the non-finite flag; the other levels are
    summed as usual, in every split of the levels into passes."""
    rng = np.random.default_rng(23)
    n = 20011
    c, res, table = _grid_setup(L, orc, "tiny", rng)
    pos = _positions(rng, n)
    dfeat = rng.normal(size=(n, c["L"] * c["F"]))
    bad = 3
    dfeat[17, bad * 2] = np.inf
    dfeat[9001, bad * 2 + 1] = np.nan
    g = L.grid_desc(res, c["F"], c["log2T"])
    dfd = dev(dfeat.reshape(n, c["L"], c["F"]).transpose(1, 0, 2).astype(np.float32))
    ws = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(g, 1, n, c["L"]), dtype=torch.uint8, device=DEV)
    saved = L.snake_tune_get("bin_levels_per_pass")
    try:
        L.snake_tune_set("bin_levels_per_pass", lg)
        dtab = torch.zeros(table.shape, device=DEV)
        L.snake_hashgrid_bwd(g, 1, dev(pos), None, None, n, None, dfd, dtab, ws)
        sync()
    finally:
        L.snake_tune_set("bin_levels_per_pass", saved)
    assert L.snake_check_device_error() == L.SNAKE_DEVERR_NONFINITE
    got = host(dtab)
    assert np.all(got[:, bad] == 0.0)
    clean = dfeat.astype(np.float32).astype(np.float64)
    clean[:, bad * 2:bad * 2 + 2] = 0.0
    dpad = np.zeros((n, 32))
    dpad[:, :clean.shape[1]] = clean
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, dpad)
    assert_grad(got, ref, 1e-4, "dtable")
