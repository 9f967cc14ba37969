"""Shared helpers for the GPU parity tests: run one libsnake call on seeded
NumPy inputs and bring its outputs back, plus the tolerance checks.

Tolerances (FP32 forms): sample bounds, positions, ray ids and hash indices
bit-exact; values |d| <= 1e-5 |ref| + 1e-7; gradients per tensor
||d||_2 / ||ref||_2 <= 1e-4 and elementwise |d| <= 1e-4 max|ref|.  BF16 MLP
forms: 1e-2 on values, 3e-2 on gradients (bf16 keeps 8 mantissa bits, so each
rounded operand carries up to 2^-9 relative error)."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    if t.dtype == torch.bfloat16:
        t = t.float()
    return t.detach().cpu().numpy()


def sync():
    torch.cuda.synchronize()


def bf16_round(a):
    """FP32 values rounded to bfloat16 (nearest, ties to even) by torch's CPU
    conversion, returned as FP32."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def assert_values(got, ref, rel=1e-5, abs_=1e-7, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    err = np.abs(got - ref)
    lim = rel * np.abs(ref) + abs_
    bad = err > lim
    if bad.any():
        i = np.argmax(err - lim)
        raise AssertionError("%s: %d/%d outside tolerance; worst idx %d got %r ref %r"
                             % (what, int(bad.sum()), bad.size, i, got.ravel()[i], ref.ravel()[i]))


def assert_grad(got, ref, tol=1e-4, what=""):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    nr = np.linalg.norm(ref)
    assert nr > 0, what
    rel = np.linalg.norm(got - ref) / nr
    assert rel <= tol, "%s: relative L2 error %.3g > %.1g" % (what, rel, tol)
    worst = np.max(np.abs(got - ref))
    assert worst <= tol * np.max(np.abs(ref)), "%s: max error %.3g > %.1g * %.3g" % (
        what, worst, tol, np.max(np.abs(ref)))


def binned_floor(orc, res, log2T, pos, dfeat, F):
    """Per table entry, the absolute part of the binned adjoint's error bound:
    (number of corner contributions it receives) x 2^(e_l - 56), where
    2^(e_l - 1) <= max|dfeat| of level l < 2^e_l.  Each value is stored with
    its exponent counted down from the level's largest gradient, so a value
    more than 37 binades below it is rounded to a multiple of 2^(e_l - 56)
    and one more than 56 below it is stored as 0.  dfeat float64 [n][L*F];
    returns float64 [L][T][F]."""
    Lv, T = len(res), 1 << log2T
    out = np.zeros((Lv, T))
    _, idx = orc.hashgrid_fwd(res, log2T, np.zeros((1, Lv, T, F), np.float32), pos, None, Lv * F,
                              return_index=True)
    for l in range(Lv):
        d = dfeat[:, l * F:(l + 1) * F]
        m = float(np.max(np.abs(d)))
        if m == 0.0:
            continue
        e = np.frexp(m)[1]
        act = np.any(d != 0.0, axis=1)
        cnt = np.bincount(idx[act, l, :].ravel().astype(np.int64), minlength=T)
        out[l] = cnt * 2.0 ** (e - 56)
    return np.repeat(out[:, :, None], F, axis=2)


def assert_binned_bound(got, ref, absref, floor, what):
    """The binned adjoint's own error bound, entry by entry: every stored value
    is rounded once to 20 significant bits after at most a 64-term FP32 run
    sum (at most about 2^-18 of the run's absolute sum), or below 2^-37 of the
    level's largest gradient to the absolute unit in `floor` (binned_floor);
    the sums are exact and the entry is rounded once to FP32, so
    |got - ref| <= 2^-17 sum|w g| + 2^-22 |ref| + floor (absref = sum|w g|
    per entry, from the oracle)."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    absref = np.asarray(absref, np.float64).ravel()
    floor = np.asarray(floor, np.float64).ravel()
    err = np.abs(got - ref)
    lim = 2.0 ** -17 * absref + 2.0 ** -22 * np.abs(ref) + floor + 1e-38
    bad = err > lim
    w = np.argmax(err / lim)
    assert not bad.any(), "%s: %d entries outside the rounding bound; worst got %r ref %r sum|c| %r floor %r" % (
        what, int(bad.sum()), got[w], ref[w], absref[w], floor[w])
    return lim


def run_sampler(L, rays_o, rays_d, boxes, S, zband=None, spr=None, max_count=None, cap=None):
    R = int(np.asarray(rays_o).shape[0])
    if cap is None:
        cap = int(np.sum(spr)) if spr is not None else R * int(S)
    Rb = max(R, 1)
    out = dict(
        packed_info=torch.full((Rb, 2), -1, dtype=torch.int32, device=DEV),
        t0=torch.zeros(max(cap, 1), device=DEV), t1=torch.zeros(max(cap, 1), device=DEV),
        pos=torch.zeros((max(cap, 1), 3), device=DEV),
        ray_id=torch.full((max(cap, 1),), -1, dtype=torch.int32, device=DEV),
        tile_id=torch.full((max(cap, 1),), 255, dtype=torch.uint8, device=DEV),
        view=torch.zeros((Rb, 3), device=DEV),
        n_out=torch.full((1,), -1, dtype=torch.int64, device=DEV))
    ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=DEV)
    ro = dev(np.asarray(rays_o, np.float64).reshape(-1, 3)) if R else None
    rd = dev(np.asarray(rays_d, np.float64).reshape(-1, 3)) if R else None
    L.snake_sample_segmented(ro, rd, R, boxes, zband, None if spr is None else dev(spr, torch.int32),
                             S, None if max_count is None else dev(max_count, torch.int32),
                             out["packed_info"], out["t0"], out["t1"], out["pos"], out["ray_id"],
                             out["tile_id"] if np.asarray(boxes).reshape(-1, 6).shape[0] > 1 else None,
                             out["view"], cap, out["n_out"], ws)
    sync()
    res = {k: host(v) for k, v in out.items()}
    n = int(res["n_out"][0])
    res["n"] = n
    for k in ("t0", "t1", "pos", "ray_id", "tile_id"):
        res[k] = res[k][:min(n, cap)]
    res["packed_info"] = res["packed_info"][:R]
    res["view"] = res["view"][:R]
    return res
