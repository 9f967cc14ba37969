"""GPU parity of the hash encoding and the density/colour networks against the
FP64 oracle: hash indices bit for bit, features and network outputs within
the FP32 (1e-5) or BF16 (1e-2) tolerance, gradients within 1e-4 (FP32) or
3e-2 (BF16)."""
import numpy as np
import pytest
import torch

import synth
from _helpers import DEV, assert_grad, assert_values, dev, host, sync

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
    L.snake_hashgrid_fwd(g, dev(table), dev(pos), None if tid is None else dev(tid), None, n, None, feat,
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
    L.snake_hashgrid_fwd(g, dev(table), dev(pos), None, dev(np.pad(sel, (0, 1000)), torch.int32), n_host,
                         nd, feat, None)
    sync()
    got = host(feat).transpose(1, 0, 2).reshape(n_host, -1)
    ref = orc.hashgrid_fwd(res, c["log2T"], table, pos[sel[:4321]], None, 32)
    assert_values(got[:4321], ref, rel=1e-5, abs_=1e-6, what="indexed feat")
    assert np.all(got[4321:] == 7.0)     # untouched past the device count


@pytest.mark.parametrize("name", ["tiny", "full", "f1", "f4"])
def test_hashgrid_bwd(L, orc, name):
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
    L.snake_hashgrid_bwd(g, dev(pos), None if tid is None else dev(tid), None, n, None, dfd, dtab)
    sync()
    dpad = np.zeros((n, 32))
    dpad[:, :W] = dfeat.astype(np.float32)
    ref = orc.hashgrid_bwd(res, c["log2T"], table.shape, pos, dpad, tid)
    assert_grad(host(dtab), ref, 1e-4, "dtable")


# ---------------------------------------------------------------------------
MLPS = {
    "tiny": (synth.MlpConfig(feat_real=16, n_dir=3, colour_layers=1, colour_out=3), 8, 2),
    "full": (synth.MlpConfig(feat_real=32, n_dir=6, colour_layers=2, colour_out=4), 16, 2),
}


def _mlp_inputs(rng, cfg, Lv, F, n, R):
    w = synth.init_mlp(rng, cfg) * np.float32(2.0)
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
    w, feat, view, sun, rid = _mlp_inputs(rng, cfg, Lv, F, n, R)
    bf = prec == "bf16"
    m = L.mlp_desc(Lv, F, cfg.n_dir, cfg.colour_layers, cfg.colour_out,
                   L.SNAKE_BF16 if bf else L.SNAKE_F32, L.SNAKE_F32)
    fd = dev(feat.reshape(n, Lv, F).transpose(1, 0, 2))
    sigma = torch.zeros(n, device=DEV)
    rgb = torch.zeros((n, 3), device=DEV)
    L.snake_mlp_fwd(m, dev(w), fd, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), None, n,
                    None, sigma, rgb)
    sync()
    rs, rc = orc.mlp_fwd(cfg, w, _pad32(feat), view, rid, sun=sun if cfg.n_dir == 6 else None)
    tol = 1e-2 if bf else 1e-5
    assert_values(host(sigma), rs, rel=tol, abs_=tol * 1e-2, what="sigma")
    assert_values(host(rgb), rc, rel=tol, abs_=tol * 1e-2, what="rgb")


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
    L.snake_mlp_bwd(m, dev(w), fd, N, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), dev(sel),
                    n, None, dev(ds), dev(dr), dW, dfeat, ws)
    sync()
    rW, rf = orc.mlp_bwd(cfg, w, _pad32(feat[sel]), view, rid[sel], ds[sel], dr[sel],
                         sun=sun if cfg.n_dir == 6 else None)
    tol = 3e-2 if bf else 1e-4
    assert_grad(host(dW), rW, tol, "dW")
    got_f = host(dfeat).transpose(1, 0, 2).reshape(n, -1)
    assert_grad(got_f, rf[:, :Lv * F], tol, "dfeat")
    # the sum is deterministic: a second call adds exactly the same values
    dW2 = dW.clone()
    L.snake_mlp_bwd(m, dev(w), fd, N, dev(view), dev(sun) if cfg.n_dir == 6 else None, dev(rid), dev(sel),
                    n, None, dev(ds), dev(dr), dW2, dfeat, ws)
    sync()
    assert torch.equal(dW2 - dW, dW)
