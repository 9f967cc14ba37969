"""GPU parity of volume rendering, its adjoint and Adam against the FP64 oracle."""
import numpy as np
import pytest
import torch

from _helpers import DEV, assert_grad, assert_values, dev, host, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2507_01631_amd import _lib
    _lib.lib()
    return _lib


def _rays(rng, counts, sigma_scale=3.0):
    counts = np.asarray(counts, np.int32)
    R = counts.size
    start = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int32)
    n = int(counts.sum())
    t0 = np.zeros(n, np.float32)
    t1 = np.zeros(n, np.float32)
    for r in range(R):
        if counts[r]:
            t = np.sort(rng.uniform(0.5, 1.5, size=counts[r] + 1)).astype(np.float32)
            t0[start[r]:start[r] + counts[r]] = t[:-1]
            t1[start[r]:start[r] + counts[r]] = t[1:]
    sigma = (rng.exponential(sigma_scale, size=n)).astype(np.float32)
    rgb = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    tgt = rng.uniform(0, 1, size=(R, 3)).astype(np.float32)
    return np.stack([start, counts], 1), t0, t1, sigma, rgb, tgt


def _gpu_composite(L, info, t0, t1, sigma, rgb, tgt, thr, scale):
    R = info.shape[0]
    o = dict(rgb_out=torch.zeros((R, 3), device=DEV), opacity=torch.zeros(R, device=DEV),
             depth=torch.zeros(R, device=DEV), n_alive=torch.zeros(R, dtype=torch.int32, device=DEV),
             loss=torch.zeros(1, device=DEV))
    args = [dev(sigma), dev(rgb), dev(t0), dev(t1), dev(info, torch.int32)]
    L.snake_composite_fwd(*args, R, thr, dev(tgt), scale, o["rgb_out"], o["opacity"], o["depth"],
                          o["n_alive"], o["loss"])
    n = sigma.size
    ds = torch.full((max(n, 1),), 9.0, device=DEV)
    dr = torch.full((max(n, 1), 3), 9.0, device=DEV)
    L.snake_composite_bwd(*args, R, o["n_alive"], dev(tgt), scale, ds, dr)
    sync()
    out = {k: host(v) for k, v in o.items()}
    out["dsigma"], out["drgb"] = host(ds)[:n], host(dr)[:n]
    return out


@pytest.mark.parametrize("thr", [0.0, 1e-4, 0.05])
def test_composite_fwd_bwd(L, orc, thr):
    rng = np.random.default_rng(20)
    counts = np.concatenate([[0, 1, 2, 63, 64, 65, 127, 128, 129, 200, 333],
                             rng.integers(0, 140, size=3000)])
    # denser media for the early-stop cases, so that T falls below the threshold
    info, t0, t1, sigma, rgb, tgt = _rays(rng, counts, sigma_scale=30.0 if thr > 0 else 3.0)
    R = info.shape[0]
    scale = 1.0 / (3 * R)
    g = _gpu_composite(L, info, t0, t1, sigma, rgb, tgt, thr, scale)
    ref = orc.composite_fwd(info, sigma, rgb, t0, t1, tgt, scale, early_stop=thr)
    # early-stop counts: equal, except where T sits within rounding of the threshold
    diff = np.nonzero(g["n_alive"] != ref["n_alive"])[0]
    for r in diff:
        st = info[r, 0]
        k = min(g["n_alive"][r], ref["n_alive"][r])
        tau = float(np.sum(sigma[st:st + k].astype(np.float64) * (t1[st:st + k].astype(np.float64)
                                                                  - t0[st:st + k])))
        assert abs(np.exp(-tau) / thr - 1.0) < 1e-4, (r, g["n_alive"][r], ref["n_alive"][r])
    assert diff.size <= max(2, R // 1000)
    ref = orc.composite_fwd(info, sigma, rgb, t0, t1, tgt, scale, alive=g["n_alive"])
    assert_values(g["rgb_out"], ref["rgb"], 1e-5, 1e-7, "rgb_out")
    assert_values(g["opacity"], ref["opacity"], 1e-5, 1e-7, "opacity")
    assert_values(g["depth"], ref["depth"], 1e-5, 1e-7, "depth")
    assert_values(g["loss"][0], ref["loss"], 1e-5, 0.0, "loss")
    rds, rdr = orc.composite_bwd(info, sigma, rgb, t0, t1, tgt, scale, n_alive=g["n_alive"])
    assert_grad(g["dsigma"], rds, 1e-4, "dsigma")
    assert_grad(g["drgb"], rdr, 1e-4, "drgb")
    if thr > 0:
        assert np.any(g["n_alive"] < counts)


def test_composite_thin_and_dense_samples(L, orc):
    """Very thin samples (alpha ~ 1e-7) and saturated ones (alpha = 1)."""
    rng = np.random.default_rng(21)
    info, t0, t1, sigma, rgb, tgt = _rays(rng, [128] * 64)
    sigma[::3] = 1e-5
    sigma[1::5] = 1e4
    R = 64
    g = _gpu_composite(L, info, t0, t1, sigma, rgb, tgt, 0.0, 1.0 / (3 * R))
    ref = orc.composite_fwd(info, sigma, rgb, t0, t1, tgt, 1.0 / (3 * R))
    assert_values(g["rgb_out"], ref["rgb"], 1e-5, 1e-7, "rgb_out")
    assert_values(g["opacity"], ref["opacity"], 1e-5, 1e-7, "opacity")


def test_adam_matches_oracle(L, orc):
    rng = np.random.default_rng(22)
    n = 100003                         # not a multiple of 4: exercises the tail
    p = rng.normal(size=n).astype(np.float32)
    P, M, V = dev(p), torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        g[:100] = 0.0
        G = dev(g)
        L.snake_adam_step(P, G, M, V, n, 1e-2, 0.9, 0.99, 1e-15, step, 1e-3, L.SNAKE_ADAM_ZERO_GRAD)
        orc.adam_step(pr, g, mr, vr, 1e-2, step, l2=1e-3)
        sync()
        assert torch.count_nonzero(G).item() == 0       # zero-grad flag
        assert_values(host(P), pr, 1e-6, 1e-7, "p step %d" % step)
        # m and v are running sums of terms of either sign: FP32 rounding is
        # relative to the terms (|g| ~ 1, g^2 ~ 1), not to the result
        assert_values(host(M), mr, 1e-5, 1e-6, "m")
        assert_values(host(V), vr, 1e-5, 1e-6, "v")
    # the step read on the device (graph replays): same bits as the host step
    P2, M2, V2 = dev(p), torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    P3, M3, V3 = dev(p), torch.zeros(n, device=DEV), torch.zeros(n, device=DEV)
    step_dev = torch.zeros(1, dtype=torch.int32, device=DEV)
    for step in range(1, 6):
        g = rng.normal(size=n).astype(np.float32)
        L.snake_counter_add(step_dev, 1)
        L.snake_adam_step(P2, dev(g), M2, V2, n, 1e-2, 0.9, 0.99, 1e-15, 0, 1e-3, 0, step_dev=step_dev)
        L.snake_adam_step(P3, dev(g), M3, V3, n, 1e-2, 0.9, 0.99, 1e-15, step, 1e-3, 0)
    sync()
    assert int(step_dev.item()) == 5
    assert torch.equal(P2, P3) and torch.equal(M2, M3) and torch.equal(V2, V3)


def test_composite_sample_map(L):
    """With a sample map the per-sample values live in another order: the
    result equals the identity-order call on the permuted arrays, bit for bit,
    and the adjoints land at the mapped positions."""
    rng = np.random.default_rng(23)
    counts = rng.integers(0, 150, size=2000)
    info, t0, t1, sigma, rgb, tgt = _rays(rng, counts, sigma_scale=30.0)
    n, R = sigma.size, info.shape[0]
    inv = rng.permutation(n).astype(np.int32)            # packed p -> stored at inv[p]
    s_perm = np.empty_like(sigma)
    s_perm[inv] = sigma
    c_perm = np.empty_like(rgb)
    c_perm[inv] = rgb
    ref = _gpu_composite(L, info, t0, t1, sigma, rgb, tgt, 1e-4, 1.0 / (3 * R))
    o = dict(rgb_out=torch.zeros((R, 3), device=DEV), n_alive=torch.zeros(R, dtype=torch.int32, device=DEV),
             loss=torch.zeros(1, device=DEV))
    args = [dev(s_perm), dev(c_perm), dev(t0), dev(t1), dev(info, torch.int32)]
    L.snake_composite_fwd(*args, R, 1e-4, dev(tgt), 1.0 / (3 * R), o["rgb_out"], None, None, o["n_alive"],
                          o["loss"], sample_map=dev(inv))
    ds = torch.full((n,), 9.0, device=DEV)
    dr = torch.full((n, 3), 9.0, device=DEV)
    L.snake_composite_bwd(*args, R, o["n_alive"], dev(tgt), 1.0 / (3 * R), ds, dr, sample_map=dev(inv))
    sync()
    assert np.array_equal(host(o["rgb_out"]), ref["rgb_out"])
    assert np.array_equal(host(o["n_alive"]), ref["n_alive"])
    assert np.array_equal(host(ds)[inv], ref["dsigma"])
    assert np.array_equal(host(dr)[inv], ref["drgb"])


def test_adam_tiles_equals_separate_calls(L):
    """Adam over K tiles in one launch, each tile with its own step count,
    gives the bits of K separate calls (tile length not a multiple of 4)."""
    rng = np.random.default_rng(23)
    K, tn = 5, 33331
    steps = np.array([1, 4, 2, 7, 3], dtype=np.int32)
    p = rng.normal(size=K * tn).astype(np.float32)
    m = (rng.normal(size=K * tn) * 0.1).astype(np.float32)
    v = np.abs(rng.normal(size=K * tn) * 0.01).astype(np.float32)
    g = rng.normal(size=K * tn).astype(np.float32)
    A = [dev(x) for x in (p, g, m, v)]
    sd = dev(steps, torch.int32)
    L.snake_adam_step_tiles(*A, tn, K, 1e-2, 0.9, 0.99, 1e-15, sd, 1e-3, L.SNAKE_ADAM_ZERO_GRAD)
    for k in range(K):
        sl = slice(k * tn, (k + 1) * tn)
        B = [dev(x[sl]) for x in (p, g, m, v)]             # separate, aligned tensors per tile
        L.snake_adam_step(*B, tn, 1e-2, 0.9, 0.99, 1e-15, int(steps[k]), 1e-3, L.SNAKE_ADAM_ZERO_GRAD)
        sync()
        for a, b in zip(A, B):
            assert torch.equal(a[sl], b)
    assert torch.count_nonzero(A[1]).item() == 0
