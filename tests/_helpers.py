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
