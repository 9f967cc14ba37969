"""Pins of the CPU FP64 oracle against what the mathematics fixes.

Nothing here re-types an oracle formula: every check is a closed form, an
invariant, a brute-force count, a library routine or a finite difference of
the oracle's own forward pass.  CPU only.
"""
import math

import numpy as np
import pytest

import synth

P2, P3 = 2654435761, 805459861


# ---------------------------------------------------------------------------
# hash grid: indices, cells, weights
# ---------------------------------------------------------------------------
def test_level_resolutions_geometric(orc):
    for L, lo, hi in [(8, 16, 256), (16, 16, 2048), (4, 8, 64), (1, 16, 16)]:
        res = orc.level_resolutions(L, lo, hi)
        assert res[0] == lo and res[-1] == hi
        assert np.all(np.diff(res) > 0) if L > 1 else True
        if L > 1:
            b = (hi / lo) ** (1.0 / (L - 1))
            exact = lo * b ** np.arange(L)
            assert np.all(res <= exact + 1e-6) and np.all(res > exact - 1.0)


def test_hash_index_bruteforce_bigint(orc):
    """Prime-XOR hash with uint32 wrap-around, checked with Python big ints."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        i, j, k = (int(v) for v in rng.integers(0, 1 << 12, size=3))
        log2T = int(rng.integers(4, 25))
        h = ((i * 1) ^ (j * P2) ^ (k * P3)) % (1 << 32) % (1 << log2T)
        assert orc.hash_index(i, j, k, 2048, log2T) == h
        assert orc.hash_index(i, j, k, 4, log2T, always_hash=True) == h


def test_hash_index_pairs_x_neighbours(orc):
    """With the x prime equal to 1, corners i and i^1 land in adjacent slots."""
    rng = np.random.default_rng(2)
    for _ in range(500):
        i, j, k = (int(v) for v in rng.integers(0, 4096, size=3))
        a = orc.hash_index(i, j, k, 2048, 19)
        b = orc.hash_index(i ^ 1, j, k, 2048, 19)
        assert a ^ b == 1


def test_dense_level_is_a_bijection(orc):
    """A level whose (N+1)^3 corners fit the table is indexed without collisions,
    x fastest."""
    N, log2T = 16, 14          # 17^3 = 4913 <= 16384
    seen = set()
    for k in range(N + 1):
        for j in range(N + 1):
            for i in range(N + 1):
                idx = orc.hash_index(i, j, k, N, log2T)
                assert idx < (N + 1) ** 3
                seen.add(idx)
                if i > 0:
                    assert idx == orc.hash_index(i - 1, j, k, N, log2T) + 1
    assert len(seen) == (N + 1) ** 3
    # one more level of resolution and the grid no longer fits -> hashed
    assert (25 + 1) ** 3 > (1 << 14)
    assert orc.hash_index(3, 5, 7, 25, 14) == ((3 ^ 5 * P2 ^ 7 * P3) % (1 << 32)) % (1 << 14)


def test_trilinear_weights_partition_of_unity(orc):
    rng = np.random.default_rng(3)
    for _ in range(300):
        x = rng.uniform(0, 1, size=3).astype(np.float32)
        N = int(rng.integers(2, 3000))
        _, w = orc.hash_corners(x, N, 19)
        assert np.all(w >= 0.0)
        assert abs(w.sum() - 1.0) < 1e-12


def test_cell_rounding_points_fp32(orc):
    """p = fl32(x N) decides the cell; at x = 1 the last cell takes weight 1."""
    N = 256
    idx, w = orc.hash_corners(np.array([1.0, 1.0, 1.0], np.float32), N, 30)
    assert w[7] == 1.0 and np.all(w[:7] == 0.0)
    # corner (N, N, N) of the dense level
    assert idx[7] == N + N * (N + 1) + N * (N + 1) ** 2
    # a value whose float32 product lands exactly on an integer
    x = np.float32(0.5)
    idx, w = orc.hash_corners(np.array([x, 0.0, 0.0], np.float32), 16, 14)
    assert idx[0] == 8 and w[0] == 1.0


def test_hashgrid_reproduces_linear_field(orc):
    """Trilinear interpolation reproduces a linear function of the corner
    coordinates exactly: table(i,j,k) = a i + b j + c k  =>  feat = a p_x + b p_y + c p_z."""
    res = np.array([16, 23], np.int32)           # both dense for T = 2^14
    log2T, F = 14, 2
    T = 1 << log2T
    table = np.zeros((1, 2, T, F), np.float32)
    coef = [(0.25, -0.5, 1.0), (0.125, 0.75, -0.25)]
    for l, N in enumerate(res):
        side = N + 1
        ii, jj, kk = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
        idx = ii + jj * side + kk * side * side
        a, b, c = coef[l]
        table[0, l, idx.ravel(), 0] = (a * ii + b * jj + c * kk).ravel()
        table[0, l, idx.ravel(), 1] = 1.0
    pos = np.random.default_rng(4).uniform(0, 1, size=(500, 3)).astype(np.float32)
    pos[:5] = [[0, 0, 0], [1, 1, 1], [0.5, 0.25, 1.0], [1, 0, 0.5], [0.999999, 0.0, 0.3]]
    feat = orc.hashgrid_fwd(res, log2T, table, pos, out_width=8)
    for l, N in enumerate(res):
        p = (pos * np.float32(N)).astype(np.float64)        # fl32(x N), then exact
        a, b, c = coef[l]
        np.testing.assert_allclose(feat[:, 2 * l], a * p[:, 0] + b * p[:, 1] + c * p[:, 2],
                                   rtol=0, atol=1e-12)
        np.testing.assert_allclose(feat[:, 2 * l + 1], 1.0, rtol=0, atol=1e-12)
    assert np.all(feat[:, 4:] == 0.0)               # zero padding past L*F


def test_hashgrid_bwd_is_adjoint_of_fwd(orc):
    """<J^T y, x> = <y, J x>: the encoding is linear in the table."""
    rng = np.random.default_rng(5)
    res = orc.level_resolutions(8, 16, 256)
    log2T = 10                                        # small table: plenty of collisions
    table = rng.normal(size=(2, 8, 1 << log2T, 2)).astype(np.float32)
    dx = rng.normal(size=table.shape).astype(np.float32)
    pos = rng.uniform(0, 1, size=(3000, 3)).astype(np.float32)
    tid = rng.integers(0, 2, size=3000).astype(np.uint8)
    y = rng.normal(size=(3000, 32))
    y[:, 16:] = 0.0
    Jx = orc.hashgrid_fwd(res, log2T, dx, pos, tid, 32)
    JTy = orc.hashgrid_bwd(res, log2T, table.shape, pos, y, tid)
    lhs = float(np.sum(JTy * dx.astype(np.float64)))
    rhs = float(np.sum(y * Jx))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs))
    # samples of tile 0 never touch tile 1's table
    y0 = np.where(tid[:, None] == 0, y, 0.0)
    g0 = orc.hashgrid_bwd(res, log2T, table.shape, pos, y0, tid)
    assert np.all(g0[1] == 0.0) and np.any(g0[0] != 0.0)


# ---------------------------------------------------------------------------
# segmented sampler
# ---------------------------------------------------------------------------
UNIT = np.array([[0.0, 0.0, 0.0, 1.0, 1.0, 1.0]])


def _ray(o, d):
    return np.array([o], np.float64), np.array([d], np.float64)


def test_sampler_vertical_ray_closed_form(orc):
    o, d = _ray([0.3, 0.4, 2.0], [0.0, 0.0, -1.0])
    s = orc.sample_segmented(o, d, UNIT, 8)
    assert s["n"] == 8 and tuple(s["packed_info"][0]) == (0, 8)
    assert s["t0"][0] == np.float32(1.0) and s["t1"][-1] == np.float32(2.0)
    assert np.all(s["t1"][:-1] == s["t0"][1:])                  # intervals abut
    np.testing.assert_allclose(s["t1"] - s["t0"], 1.0 / 8, rtol=0, atol=1e-6)
    assert np.all(s["pos"][:, 0] == np.float32(0.3)) and np.all(s["pos"][:, 1] == np.float32(0.4))
    mid = 1.0 + (np.arange(8) + 0.5) / 8.0
    np.testing.assert_allclose(s["pos"][:, 2], 2.0 - mid, rtol=0, atol=2e-7)
    assert np.all(s["view"][0] == np.float32([0, 0, -1]))
    # the altitude band clips the chord to [z_hi, z_lo] = t in [1.2, 1.8]
    s = orc.sample_segmented(o, d, UNIT, 4, zband=[0.2, 0.8])
    assert s["t0"][0] == np.float32((0.8 - 2.0) / -1.0) and s["t1"][-1] == np.float32(1.8)
    np.testing.assert_allclose(s["pos"][:, 2], [0.725, 0.575, 0.425, 0.275], atol=2e-7)


def test_sampler_axis_aligned_rays_each_axis(orc):
    for a in range(3):
        for sgn in (1.0, -1.0):
            o = np.array([0.25, 0.5, 0.75])
            o[a] = -0.5 if sgn > 0 else 1.5
            d = np.zeros(3)
            d[a] = sgn * 2.0                                  # non-unit direction
            s = orc.sample_segmented(o[None], d[None], UNIT, 5)
            assert s["t0"][0] == np.float32(0.25) and s["t1"][-1] == np.float32(0.75)
            assert np.all(s["view"][0] == np.float32(d / 2.0))


def test_sampler_misses_and_origin_inside(orc):
    o = np.array([[2.0, 2.0, 2.0], [0.5, 0.5, 0.5], [0.5, 0.5, 2.0], [1.0, 0.5, 2.0]])
    d = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    s = orc.sample_segmented(o, d, UNIT, 16)
    cnt = s["packed_info"][:, 1]
    assert list(cnt) == [0, 16, 0, 0]        # miss, inside (t_near = 0), pointing away, on the hi face
    assert s["t0"][0] == 0.0 and s["t1"][15] == np.float32(0.5)
    # a ray through an edge only (t_far == t_near) is a miss
    s = orc.sample_segmented([[0.5, -0.5, 0.5]], [[1.0, 1.0, 0.0]], UNIT, 4)
    assert s["n"] == 0


def _grid_boxes(nx, ny, side=1.0, z=(0.0, 1.0), x0=0.0, y0=0.0):
    b = []
    for ix in range(nx):
        for iy in range(ny):
            b.append([x0 + ix * side, y0 + iy * side, z[0],
                      x0 + (ix + 1) * side, y0 + (iy + 1) * side, z[1]])
    return np.array(b)


def _slanted_rays(rng, n, lo, hi, z_top=1.5, max_deg=30.0):
    th = np.deg2rad(rng.uniform(1.0, max_deg, size=n))
    ph = rng.uniform(0, 2 * np.pi, size=n)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)], 1)
    g = np.concatenate([rng.uniform(lo, hi, size=(n, 2)), np.full((n, 1), 0.5)], 1)
    o = g - ((z_top - 0.5) / np.cos(th))[:, None] * d
    return o, d


def test_sampler_segments_meet_on_shared_faces(orc):
    """Adjacent NeRF tiles: the far bound of one segment is bit-for-bit the
    near bound of the next, and the segments together cover the chord through
    the union of the tiles."""
    rng = np.random.default_rng(6)
    boxes = _grid_boxes(2, 2)
    window = np.array([[0.0, 0.0, 0.0, 2.0, 2.0, 1.0]])
    o, d = _slanted_rays(rng, 400, 0.2, 1.8)
    S = rng.integers(8, 129, size=400).astype(np.int32)
    s = orc.sample_segmented(o, d, boxes, 0, samples_per_ray=S)
    whole = orc.sample_segmented(o, d, window, 0, samples_per_ray=S)
    shared = 0
    for r in range(400):
        st, c = s["packed_info"][r]
        wst, wc = whole["packed_info"][r]
        assert c == S[r] == wc                          # the budget is spent exactly
        t0, t1, tid = s["t0"][st:st + c], s["t1"][st:st + c], s["tile_id"][st:st + c]
        assert np.all(t1[:-1] == t0[1:])                 # abut, across tile changes too
        assert t0[0] == whole["t0"][wst] and t1[-1] == whole["t1"][wst + wc - 1]
        changes = np.nonzero(tid[1:] != tid[:-1])[0]
        shared += len(changes) > 0
        for ch in changes:                                # positions cross the face
            a = 0 if boxes[tid[ch]][3] == boxes[tid[ch + 1]][0] or boxes[tid[ch]][0] == boxes[tid[ch + 1]][3] else 1
            assert 0.0 <= s["pos"][st + ch][a] <= 1.0 and 0.0 <= s["pos"][st + ch + 1][a] <= 1.0
        # each tile's samples lie inside its box (world position from local)
        for j in range(c):
            b = boxes[tid[j]]
            m = 0.5 * (float(t0[j]) + float(t1[j]))
            pw = o[r] + m * d[r]
            assert np.all(pw >= b[:3] - 1e-5) and np.all(pw <= b[3:] + 1e-5)
    assert shared > 50


def test_sampler_budget_split_proportional(orc):
    """Sum of per-segment counts equals the ray budget; every segment gets a
    sample, and each count is within one sample of 1 + its length-proportional
    share of the rest."""
    rng = np.random.default_rng(7)
    boxes = _grid_boxes(2, 2)
    o, d = _slanted_rays(rng, 300, 0.3, 1.7)
    S = 64
    s = orc.sample_segmented(o, d, boxes, S)
    for r in range(300):
        st, c = s["packed_info"][r]
        assert c == S
        tid = s["tile_id"][st:st + c]
        lens, counts = [], []
        for k in np.unique(tid):
            sel = tid == k
            lens.append(float(s["t1"][st:st + c][sel][-1]) - float(s["t0"][st:st + c][sel][0]))
            counts.append(int(sel.sum()))
        nseg = len(lens)
        share = 1 + (S - nseg) * np.array(lens) / np.sum(lens)
        assert np.all(np.array(counts) >= 1)
        assert np.all(np.abs(np.array(counts) - share) <= 1.0 + 1e-6)


def test_sampler_at_most_three_tiles_for_low_off_nadir(orc):
    """A ray crossing the band with (z_hi - z_lo) tan(theta) <= tile side meets
    at most 3 tiles of a regular grid."""
    rng = np.random.default_rng(8)
    boxes = _grid_boxes(4, 4, side=1.0, z=(0.0, 1.0))
    o, d = _slanted_rays(rng, 2000, 0.5, 3.5, z_top=1.2, max_deg=44.0)
    s = orc.sample_segmented(o, d, boxes, 32)
    for r in range(2000):
        st, c = s["packed_info"][r]
        assert len(np.unique(s["tile_id"][st:st + c])) <= 3


def test_sampler_truncation_is_a_prefix(orc):
    w = synth.tiny_tile(seed=3, n_rays=64, samples=32)
    full = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 32)
    mc = np.random.default_rng(9).integers(-1, 40, size=64).astype(np.int32)
    tr = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 32, max_count=mc)
    for r in range(64):
        fs, fc = full["packed_info"][r]
        ts, tc = tr["packed_info"][r]
        assert tc == min(fc, max(mc[r], 0))
        for key in ("t0", "t1", "pos", "ray_id"):
            assert np.array_equal(tr[key][ts:ts + tc], full[key][fs:fs + tc])


def test_window_accept_closed_forms(orc):
    """Vertical rays accept inside or on the window edge (closed rectangle)
    and reject outside; a slanted ray's band chord end points are
    o + t d at t = (z - o_z) / d_z; rays parallel to the band are rejected;
    an origin inside the band starts the chord at t = 0."""
    win = (0.0, 0.0, 2.0, 2.0)
    o = np.array([[1.0, 1.0, 3.0], [2.0, 0.5, 3.0], [2.0 + 2**-40, 0.5, 3.0], [-0.25, 1.0, 3.0],
                  [0.5, 0.5, 2.0], [0.5, 0.5, 2.0], [0.5, 0.5, 2.0], [1.0, 1.0, 0.5], [1.0, 1.0, 0.5],
                  [1.0, 1.0, 0.5]])
    d = np.array([[0, 0, -1.0], [0, 0, -1.0], [0, 0, -1.0], [0, 0, -1.0],
                  # band [0.5, 1.5]: chord t in [0.5, 1.5], x from 0.625 to 0.875 (all exact)
                  [0.25, 0, -1.0], [-0.375, 0, -1.0], [-0.5, 0, -1.0],
                  [1.0, 0, 0.0],                               # parallel to the band
                  [1.5, 0, 1.0],                               # inside, going up: t in [0, 1]
                  [0.75, 0, 1.0]])
    acc = orc.window_accept(o, d, win, (0.5, 1.5))
    # x at chord ends: ray 5: 0.5-0.1875=0.3125, 0.5-0.5625=-0.0625 -> out;
    # ray 6: 0.25, -0.25 -> out; ray 8: 1, 2.5 -> out; ray 9: 1, 1.75 -> in
    assert acc.tolist() == [1, 1, 0, 0, 1, 0, 0, 0, 0, 1]
    acc2 = orc.window_accept(o[4:5], d[4:5], (0.0, 0.0, 0.875, 1.0), (0.5, 1.5))
    acc3 = orc.window_accept(o[4:5], d[4:5], (0.0, 0.0, 0.875 - 2**-40, 1.0), (0.5, 1.5))
    assert acc2.tolist() == [1] and acc3.tolist() == [0]


def test_window_accept_equals_chord_covered_by_window_tiles(orc):
    """A ray is accepted exactly when the 2x2 window's tiles cover its whole
    chord through the band: the sampler's intervals inside the window then
    span the same length as over a 4x4 grid around it (checked through the
    independently pinned segmented sampler)."""
    rng = np.random.default_rng(21)
    win_boxes = _grid_boxes(2, 2)                         # [0,2]^2 x [0,1]
    big = _grid_boxes(4, 4, x0=-1.0, y0=-1.0)             # [-1,3]^2 x [0,1]
    o, d = _slanted_rays(rng, 3000, -0.3, 2.3, z_top=1.4, max_deg=30.0)
    acc = orc.window_accept(o, d, (0.0, 0.0, 2.0, 2.0), (0.0, 1.0))
    sw = orc.sample_segmented(o, d, win_boxes, 16)
    sb = orc.sample_segmented(o, d, big, 16)
    n_acc = n_rej_partial = 0
    for r in range(3000):
        ws, wc = sw["packed_info"][r]
        bs, bc = sb["packed_info"][r]
        assert bc > 0
        lw = float(np.sum(sw["t1"][ws:ws + wc].astype(np.float64) - sw["t0"][ws:ws + wc]))
        lb = float(np.sum(sb["t1"][bs:bs + bc].astype(np.float64) - sb["t0"][bs:bs + bc]))
        # band end points, to skip rays that graze the window edge
        t = np.array([(1.0 - o[r, 2]) / d[r, 2], (0.0 - o[r, 2]) / d[r, 2]])
        xy = o[r, :2][None, :] + t[:, None] * d[r, :2][None, :]
        edge = np.min(np.abs(np.concatenate([xy.ravel(), xy.ravel() - 2.0])))
        if edge < 1e-6:
            continue
        if acc[r]:
            n_acc += 1
            assert abs(lw - lb) <= 1e-6 * lb
        else:
            assert lw < lb - 1e-6
            n_rej_partial += wc > 0
    assert n_acc > 500 and n_rej_partial > 200


def test_sampler_capacity_error(orc):
    w = synth.tiny_tile(seed=0, n_rays=16, samples=8)
    with pytest.raises(ValueError):
        orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 8, cap=100)


# ---------------------------------------------------------------------------
# volume rendering
# ---------------------------------------------------------------------------
def _single_ray(n, t_a, t_b):
    t = np.linspace(t_a, t_b, n + 1).astype(np.float32)
    return np.array([[0, n]], np.int32), t[:-1].copy(), t[1:].copy()


def test_composite_constant_density_closed_form(orc):
    for n in (1, 3, 64, 128):
        info, t0, t1 = _single_ray(n, 0.5, 1.25)
        ell = float(t1[-1]) - float(t0[0])
        sig = np.full(n, 2.5)
        c = np.array([0.2, 0.5, 0.9])
        out = orc.composite_fwd(info, sig, np.tile(c, (n, 1)), t0, t1)
        T_final = math.exp(-2.5 * ell)
        assert abs(out["opacity"][0] - (1 - T_final)) < 1e-13
        np.testing.assert_allclose(out["rgb"][0], c * (1 - T_final), rtol=0, atol=1e-13)
        assert out["n_alive"][0] == n


def test_composite_depth_geometric_series(orc):
    """Uniform intervals of width h and constant sigma: w_i = q^i (1-q) with
    q = exp(-sigma h); depth = sum w_i (t_a + (i + 1/2) h) in closed form."""
    n, t_a, h, sig = 40, 0.25, 1.0 / 64, 7.0
    t = (t_a + h * np.arange(n + 1)).astype(np.float32)      # exact in FP32
    info = np.array([[0, n]], np.int32)
    out = orc.composite_fwd(info, np.full(n, sig), np.ones((n, 3)), t[:-1], t[1:])
    q = math.exp(-sig * h)
    s0 = (1 - q ** n) / (1 - q)
    s1 = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    depth = (1 - q) * ((t_a + 0.5 * h) * s0 + h * s1)
    assert abs(out["depth"][0] - depth) < 1e-12


def test_composite_segments_associate(orc):
    """Compositing two consecutive segments separately and combining them with
    C = C1 + T1 C2, T = T1 T2 equals compositing their concatenation (the
    segmented rendering identity for rays split between NeRF tiles)."""
    rng = np.random.default_rng(10)
    n1, n2 = 17, 29
    t = np.sort(rng.uniform(0, 2, size=n1 + n2 + 1)).astype(np.float32)
    sig = rng.uniform(0, 5, size=n1 + n2)
    rgb = rng.uniform(0, 1, size=(n1 + n2, 3))
    whole = orc.composite_fwd(np.array([[0, n1 + n2]], np.int32), sig, rgb, t[:-1], t[1:])
    a = orc.composite_fwd(np.array([[0, n1]], np.int32), sig[:n1], rgb[:n1], t[:n1], t[1:n1 + 1])
    b = orc.composite_fwd(np.array([[0, n2]], np.int32), sig[n1:], rgb[n1:], t[n1:-1], t[n1 + 1:])
    T1, T2 = 1 - a["opacity"][0], 1 - b["opacity"][0]
    np.testing.assert_allclose(whole["rgb"][0], a["rgb"][0] + T1 * b["rgb"][0], atol=1e-14)
    assert abs((1 - whole["opacity"][0]) - T1 * T2) < 1e-14
    assert whole["opacity"][0] <= 1.0


def test_composite_early_stop_and_loss(orc):
    info, t0, t1 = _single_ray(10, 0.0, 1.0)
    sig = np.full(10, 0.01)
    sig[4] = 1e3                    # T drops to ~0 after sample 4
    rgb = np.full((10, 3), 0.5)
    out = orc.composite_fwd(info, sig, rgb, t0, t1, early_stop=1e-4)
    assert out["n_alive"][0] == 5
    off = orc.composite_fwd(info, sig, rgb, t0, t1)
    assert off["n_alive"][0] == 10
    assert abs(out["rgb"][0, 0] - off["rgb"][0, 0]) < 1e-6       # the tail carries ~no weight
    tgt = out["rgb"].astype(np.float32)
    assert orc.composite_fwd(info, sig, rgb, t0, t1, target=tgt, loss_scale=1.0)["loss"] < 1e-12
    tgt2 = tgt + np.float32(0.5)
    l2 = orc.composite_fwd(info, sig, rgb, t0, t1, target=tgt2, loss_scale=1 / 3)["loss"]
    assert abs(l2 - 0.25) < 1e-6


def test_composite_bwd_single_sample_closed_form(orc):
    """C = (1 - exp(-sigma d)) c: dC/dsigma = d exp(-sigma d) c."""
    info = np.array([[0, 1]], np.int32)
    t0, t1 = np.array([0.5], np.float32), np.array([0.75], np.float32)
    sig, c = np.array([3.0]), np.array([[0.2, 0.4, 0.6]])
    tgt = np.zeros((1, 3), np.float32)
    ds, dc = orc.composite_bwd(info, sig, c, t0, t1, tgt, 0.5)
    C = (1 - math.exp(-0.75)) * c[0]
    g = 2 * 0.5 * C
    assert abs(ds[0] - np.sum(g * 0.25 * math.exp(-0.75) * c[0])) < 1e-14
    np.testing.assert_allclose(dc[0], g * (1 - math.exp(-0.75)), atol=1e-15)


def test_composite_bwd_matches_central_fd(orc):
    rng = np.random.default_rng(11)
    R = 6
    cnt = np.array([1, 5, 12, 0, 30, 7], np.int32)
    st = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int32)
    info = np.stack([st, cnt], 1)
    n = int(cnt.sum())
    t0 = np.zeros(n, np.float32)
    t1 = np.zeros(n, np.float32)
    for r in range(R):
        t = np.sort(rng.uniform(0, 1, size=cnt[r] + 1)).astype(np.float32)
        t0[st[r]:st[r] + cnt[r]], t1[st[r]:st[r] + cnt[r]] = t[:-1], t[1:]
    sig = rng.uniform(0.1, 8, size=n)
    rgb = rng.uniform(0, 1, size=(n, 3))
    tgt = rng.uniform(0, 1, size=(R, 3)).astype(np.float32)
    scale = 1 / (3 * R)
    ds, dc = orc.composite_bwd(info, sig, rgb, t0, t1, tgt, scale)
    L = lambda s_, c_: orc.composite_fwd(info, s_, c_, t0, t1, target=tgt, loss_scale=scale)["loss"]
    h = 1e-6
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd = (L(sig + e, rgb) - L(sig - e, rgb)) / (2 * h)
        assert abs(fd - ds[i]) <= 1e-7 * max(1e-3, abs(ds[i]))
        for c in range(3):
            E = np.zeros_like(rgb)
            E[i, c] = h
            fd = (L(sig, rgb + E) - L(sig, rgb - E)) / (2 * h)
            assert abs(fd - dc[i, c]) <= 1e-7 * max(1e-3, abs(dc[i, c]))


def test_composite_bwd_early_stop_zero_tail(orc):
    info, t0, t1 = _single_ray(10, 0.0, 1.0)
    sig = np.full(10, 0.5)
    rgb = np.full((10, 3), 0.5)
    tgt = np.zeros((1, 3), np.float32)
    ds, dc = orc.composite_bwd(info, sig, rgb, t0, t1, tgt, 1.0, n_alive=np.array([6], np.int32))
    assert np.all(ds[6:] == 0) and np.all(dc[6:] == 0) and np.all(dc[:6] > 0)


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------
def _numpy_mlp(m, w, feat, view, sun):
    """Textbook forward with NumPy FP64 matmuls."""
    shapes = synth.mlp_param_shapes(m)
    mats, o = [], 0
    for (a, b) in shapes:
        mats.append(w[o:o + a * b].astype(np.float64).reshape(a, b))
        o += a * b
    relu = lambda x: np.maximum(x, 0.0)
    sig = lambda x: 1.0 / (1.0 + np.exp(-x))
    h = relu(feat @ mats[0].T)
    out = h @ mats[1].T
    sigma = np.exp(out[:, 0])
    cin = [out[:, 1:], view.astype(np.float64)]
    if m.n_dir == 6:
        cin.append(sun.astype(np.float64))
    g = relu(np.concatenate(cin, 1) @ mats[2].T)
    for li in range(m.colour_layers - 1):
        g = relu(g @ mats[3 + li].T)
    y = g @ mats[-1].T
    rgb = sig(y[:, :3]) if m.colour_out == 3 else sig(y[:, :3]) * sig(y[:, 3:4])
    return sigma, rgb


@pytest.mark.parametrize("which", ["tiny", "full"])
def test_mlp_fwd_matches_numpy_chain(orc, which):
    rng = np.random.default_rng(12)
    m = synth.tiny_tile().mlp if which == "tiny" else synth.MlpConfig(
        feat_real=32, n_dir=6, colour_layers=2, colour_out=4)
    w = synth.init_mlp(rng, m) * 3.0
    n = 257
    feat = rng.normal(size=(n, 32))
    view = rng.normal(size=(n, 3)).astype(np.float32)
    sun = rng.normal(size=(n, 3)).astype(np.float32)
    rid = np.arange(n, dtype=np.int32)
    sigma, rgb = orc.mlp_fwd(m, w, feat, view, rid, sun=sun if m.n_dir == 6 else None)
    s_ref, c_ref = _numpy_mlp(m, w, feat, view, sun)
    np.testing.assert_allclose(sigma, s_ref, rtol=1e-12)
    np.testing.assert_allclose(rgb, c_ref, rtol=1e-12, atol=1e-15)
    assert orc.mlp_param_count(m) == w.size


@pytest.mark.parametrize("which", ["tiny", "full"])
def test_mlp_bwd_matches_central_fd(orc, which):
    rng = np.random.default_rng(13)
    m = synth.tiny_tile().mlp if which == "tiny" else synth.MlpConfig(
        feat_real=32, n_dir=6, colour_layers=2, colour_out=4)
    w = (synth.init_mlp(rng, m) * 2.0).astype(np.float32)
    n = 9
    feat = rng.normal(size=(n, 32))
    view = rng.normal(size=(n, 3)).astype(np.float32)
    sun = rng.normal(size=(n, 3)).astype(np.float32)
    sun_arg = sun if m.n_dir == 6 else None
    rid = np.arange(n, dtype=np.int32)
    ys, yc = rng.normal(size=n), rng.normal(size=(n, 3))
    dW, dfeat = orc.mlp_bwd(m, w, feat, view, rid, ys, yc, sun=sun_arg)

    # FD over the FP64 weights through the NumPy chain (independent of the oracle)
    def J(wd, fd_):
        s, c = _numpy_mlp(m, wd, fd_, view, sun)
        return float(np.sum(s * ys) + np.sum(c * yc))
    wd = w.astype(np.float64)
    h = 1e-6
    idx = rng.choice(w.size, size=200, replace=False)
    # FD round-off is ~eps |J| / h; allow it on top of a 1e-6 relative error
    tol_w = 1e-6 * np.abs(dW).max() + 1e-15 * abs(J(wd, feat)) / h
    for i in idx:
        e = np.zeros_like(wd)
        e[i] = h
        fd = (J(wd + e, feat) - J(wd - e, feat)) / (2 * h)
        assert abs(fd - dW[i]) <= tol_w, (i, fd, dW[i])
    tol_f = 1e-6 * np.abs(dfeat).max() + 1e-15 * abs(J(wd, feat)) / h
    for s in range(n):
        for i in range(32):
            e = np.zeros_like(feat)
            e[s, i] = h
            fd = (J(wd, feat + e) - J(wd, feat - e)) / (2 * h)
            assert abs(fd - dfeat[s, i]) <= tol_f


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------
def test_adam_constant_gradient_closed_form(orc):
    """With a constant gradient g, bias correction makes m_hat = g and
    v_hat = g^2 at every step, so each step moves p by lr g / (|g| + eps)."""
    rng = np.random.default_rng(14)
    n = 1000
    p0 = rng.normal(size=n)
    g = rng.normal(size=n)
    g[:10] = 0.0
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    lr, eps = 1e-2, 1e-15
    for t in range(1, 6):
        orc.adam_step(p, g, m, v, lr, t, eps=eps)
        expect = p0 - t * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(p, expect, rtol=0, atol=1e-13)
    assert np.all(p[:10] == p0[:10])                 # zero gradient, zero update


def test_adam_l2_and_first_step(orc):
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.0, 0.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    orc.adam_step(p, g, m, v, 0.1, 1, eps=0.0, l2=0.5)
    # first step: p - lr sign(g + l2 p)
    np.testing.assert_allclose(p, [0.9, -1.9, 0.4], atol=1e-14)


# ---------------------------------------------------------------------------
# end-to-end step: gradients of the whole chain against central FD
# ---------------------------------------------------------------------------
def _small_workload(seed=0, n_rays=48, samples=24):
    w = synth.tiny_tile(seed=seed, n_rays=n_rays, samples=samples)
    rng = np.random.default_rng(seed + 100)
    # larger table values so that the encoding matters in the loss
    w.table = rng.uniform(-1.0, 1.0, size=w.table.shape).astype(np.float32)
    return w


def _loss(orc, w, res, table, params):
    s = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, w.samples_per_ray)
    f = orc.hashgrid_fwd(res, w.grid.log2_table, table, s["pos"], s["tile_id"], 32)
    sg, c = orc.mlp_fwd(w.mlp, params, f, s["view"], s["ray_id"])
    return orc.composite_fwd(s["packed_info"], sg, c, s["t0"], s["t1"], w.target,
                             1.0 / (3 * w.n_rays))["loss"]


def test_train_step_gradients_match_central_fd(orc):
    w = _small_workload()
    out = orc.train_step(w)
    res = out["res"]
    rng = np.random.default_rng(15)
    g = out["dtable"].ravel()
    nz = np.nonzero(np.abs(g) > 1e-3 * np.abs(g).max())[0]
    pick = rng.choice(nz, size=min(64, nz.size), replace=False)
    h = 1e-4
    base = w.table.astype(np.float64)
    bad = 0
    for i in pick:
        tp, tm = base.ravel().copy(), base.ravel().copy()
        tp[i] += h
        tm[i] -= h
        # the oracle takes float32 tables: perturb through float64 -> use exact deltas
        lp = _loss(orc, w, res, tp.reshape(base.shape).astype(np.float32), w.mlp_params)
        lm = _loss(orc, w, res, tm.reshape(base.shape).astype(np.float32), w.mlp_params)
        hp = float(np.float32(tp[i]) - np.float32(base.ravel()[i]))
        hm = float(np.float32(base.ravel()[i]) - np.float32(tm[i]))
        fd = (lp - lm) / (hp + hm)
        if abs(fd - g[i]) > 2e-3 * abs(g).max():
            bad += 1
    assert bad <= 2, bad
    gw = out["dW"]
    pick = rng.choice(np.nonzero(np.abs(gw) > 1e-3 * np.abs(gw).max())[0], size=64, replace=False)
    bad = 0
    for i in pick:
        wp, wm = w.mlp_params.copy(), w.mlp_params.copy()
        hh = np.float32(1e-3) * max(1.0, abs(float(wp[i])))
        wp[i] += hh
        wm[i] -= hh
        fd = (_loss(orc, w, res, w.table, wp) - _loss(orc, w, res, w.table, wm)) / float(wp[i] - wm[i])
        if abs(fd - gw[i]) > 2e-3 * abs(gw).max():
            bad += 1
    assert bad <= 2, bad


def test_train_step_thread_count_independent(orc, monkeypatch):
    """The oracle's reductions are ordered, so its step is deterministic."""
    w = _small_workload(seed=1)
    a = orc.train_step(w)
    b = orc.train_step(w)
    assert np.array_equal(a["dtable"], b["dtable"]) and np.array_equal(a["dW"], b["dW"])


# ---------------------------------------------------------------------------
# diagnostics: ReLU margin and BF16-rounding emulation
# ---------------------------------------------------------------------------
def test_mlp_margin_invariances(orc):
    rng = np.random.default_rng(16)
    m = synth.tiny_tile().mlp
    w = synth.init_mlp(rng, m)
    feat = rng.normal(size=(50, 32))
    feat[:, 16:] = 0.0
    view = rng.normal(size=(50, 3)).astype(np.float32)
    rid = np.arange(50, dtype=np.int32)
    mg = orc.mlp_margin(m, w, feat, view, rid)
    assert np.all(mg >= 0) and np.all(mg <= 1)
    # doubling the first density layer and halving the second is exact (powers
    # of two): every ratio and the embedding are unchanged, so is the margin
    w2 = w.copy()
    w2[:64 * 32] *= np.float32(2.0)
    w2[64 * 32:64 * 32 + 16 * 64] *= np.float32(0.5)
    mg2 = orc.mlp_margin(m, w2, feat, view, rid)
    np.testing.assert_allclose(mg, mg2, rtol=1e-12)
    # a uniformly shifted input that keeps every sign changes the margin
    assert not np.allclose(mg, orc.mlp_margin(m, w, feat + 3.0 * (feat != 0), view, rid))
    # a pre-activation that is exactly zero gives margin 0
    f0 = np.zeros((1, 32))
    f0[0, 0], f0[0, 1] = 1.0, 1.0
    w0 = w.copy()
    w0[0], w0[1] = np.float32(0.5), np.float32(-0.5)       # unit 0: 0.5 - 0.5 = 0
    assert orc.mlp_margin(m, w0, f0, view[:1], rid[:1])[0] == 0.0


@pytest.mark.parametrize("which", ["tiny", "full"])
def test_bf16_emulation_matches_torch_rounding(orc, which):
    """The emulated BF16 forward equals a NumPy chain whose rounding points use
    torch's float32 -> bfloat16 conversion (round to nearest even)."""
    import torch
    rng = np.random.default_rng(17)
    m = synth.tiny_tile().mlp if which == "tiny" else synth.MlpConfig(
        feat_real=32, n_dir=6, colour_layers=2, colour_out=4)
    w = synth.init_mlp(rng, m)
    n = 300
    feat = rng.normal(scale=0.5, size=(n, 32))
    view = rng.normal(size=(n, 3)).astype(np.float32)
    sun = rng.normal(size=(n, 3)).astype(np.float32)
    rid = np.arange(n, dtype=np.int32)
    bf = lambda a: torch.tensor(np.asarray(a, np.float64)).float().bfloat16().double().numpy()
    shapes = synth.mlp_param_shapes(m)
    mats, o = [], 0
    for (a, b) in shapes:
        mats.append(bf(w[o:o + a * b]).reshape(a, b))
        o += a * b
    h = bf(np.maximum(bf(feat) @ mats[0].T, 0))
    out = h @ mats[1].T
    cin = [bf(out[:, 1:]), bf(view)] + ([bf(sun)] if m.n_dir == 6 else [])
    g = bf(np.maximum(np.concatenate(cin, 1) @ mats[2].T, 0))
    for li in range(m.colour_layers - 1):
        g = bf(np.maximum(g @ mats[3 + li].T, 0))
    y = g @ mats[-1].T
    sg = lambda v: 1 / (1 + np.exp(-v))
    rgb = sg(y[:, :3]) if m.colour_out == 3 else sg(y[:, :3]) * sg(y[:, 3:4])
    s_e, c_e = orc.mlp_fwd_bf16emu(m, w, feat, view, rid, sun=sun if m.n_dir == 6 else None)
    np.testing.assert_allclose(s_e, np.exp(out[:, 0]), rtol=1e-12)
    np.testing.assert_allclose(c_e, rgb, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("which", ["tiny", "full"])
def test_bf16_adjoint_emulation(orc, which):
    """The 16-bit adjoint emulation (mlp_bwd_q): with rounding off it is the
    FP64 adjoint bit for bit (the same terms in the same order, so the FD pins
    of mlp_bwd carry over); with rounding on it equals a NumPy chain that rounds
    the same operands with torch's float32 -> bfloat16 conversion."""
    import torch
    rng = np.random.default_rng(18)
    m = synth.tiny_tile().mlp if which == "tiny" else synth.MlpConfig(
        feat_real=32, n_dir=6, colour_layers=2, colour_out=4)
    w = synth.init_mlp(rng, m) * np.float32(2.0)
    n = 400
    feat = rng.normal(scale=0.5, size=(n, 32))
    view = rng.normal(size=(n, 3)).astype(np.float32)
    sun = rng.normal(size=(n, 3)).astype(np.float32) if m.n_dir == 6 else None
    rid = np.arange(n, dtype=np.int32)
    dsig = rng.normal(size=n)
    drgb = rng.normal(size=(n, 3))
    dW0, df0 = orc.mlp_bwd(m, w, feat, view, rid, dsig, drgb, sun=sun)
    dWq0, dfq0 = orc.mlp_bwd_q(m, w, feat, view, rid, dsig, drgb, sun=sun, round16=0)
    assert np.array_equal(dW0, dWq0) and np.array_equal(df0, dfq0)
    # rounding on: the same chain written with NumPy products and torch's rounding
    bf = lambda a: torch.tensor(np.asarray(a, np.float64)).float().bfloat16().double().numpy()
    shapes = synth.mlp_param_shapes(m)
    mats, o = [], 0
    for (a, b) in shapes:
        mats.append(bf(w[o:o + a * b]).reshape(a, b))
        o += a * b
    CL = m.colour_layers
    x = bf(feat)
    h1 = np.maximum(x @ mats[0].T, 0)
    h1q = bf(h1)
    out = h1q @ mats[1].T
    ci = np.concatenate([bf(out[:, 1:]), bf(view)] + ([bf(sun)] if m.n_dir == 6 else []), 1)
    gs, gq = [], []
    prev = ci
    for li in range(CL):
        gl = np.maximum(prev @ mats[2 + li].T, 0)
        gs.append(gl)
        gq.append(bf(gl))
        prev = gq[-1]
    y = prev @ mats[2 + CL].T
    sg = lambda v: 1 / (1 + np.exp(-v))
    if m.colour_out == 3:
        dout = drgb * sg(y) * (1 - sg(y))
    else:
        alb, vis = sg(y[:, :3]), sg(y[:, 3:4])
        dout = np.concatenate([drgb * vis * alb * (1 - alb), (drgb * alb).sum(1, keepdims=True) * vis * (1 - vis)], 1)
    dout = bf(dout)
    dWs = [None] * len(mats)
    dWs[2 + CL] = dout.T @ gq[-1]
    dg = bf((dout @ mats[2 + CL]) * (gs[-1] > 0))
    for li in range(CL - 1, 0, -1):
        dWs[2 + li] = dg.T @ gq[li - 1]
        dg = bf((dg @ mats[2 + li]) * (gs[li - 1] > 0))
    dWs[2] = dg.T @ ci
    dos = bf(np.concatenate([(dsig * np.exp(out[:, 0]))[:, None], dg @ mats[2][:, :m.dens_out - 1]], 1))
    dWs[1] = dos.T @ h1q
    dh = bf((dos @ mats[1]) * (h1 > 0))
    dWs[0] = dh.T @ x
    dfeat = dh @ mats[0]
    dW = np.concatenate([d.ravel() for d in dWs])
    dWq, dfq = orc.mlp_bwd_q(m, w, feat, view, rid, dsig, drgb, sun=sun, round16=1)
    np.testing.assert_allclose(dfq, dfeat, rtol=1e-10, atol=1e-12 * np.abs(dfeat).max())
    np.testing.assert_allclose(dWq, dW, rtol=1e-10, atol=1e-12 * np.abs(dW).max())
    # and the rounding is real: the 16-bit adjoint is not the FP64 one
    assert not np.allclose(dWq, dW0, rtol=1e-6)


def test_train_step_per_tile_weights_reduce_to_shared(orc):
    """Window step on 2x2 tiles with one weight set per tile: when the four
    sets are equal, the forward, the loss and the table gradient are those of
    the shared-weight step, and the per-tile weight gradients sum to the shared
    one (each sample's adjoint goes to exactly its own tile's set)."""
    import copy
    wl = synth.tiny_tile(seed=5, n_rays=300, samples=24)
    wl = copy.copy(wl)
    wl.boxes = np.array([[0, 0, 0, 0.5, 0.5, 1], [0, 0.5, 0, 0.5, 1, 1], [0.5, 0, 0, 1, 0.5, 1],
                         [0.5, 0.5, 0, 1, 1, 1]], dtype=np.float64)
    rng = np.random.default_rng(3)
    wl.table = synth.init_table(rng, wl.grid, n_tiles=4) * np.float32(1e4)
    wl.samples_per_ray = rng.integers(8, 40, size=300).astype(np.int32)
    shared = orc.train_step(wl)
    W = np.stack([wl.mlp_params] * 4)
    tiled = orc.train_step(wl, mlp_params=W)
    assert len(np.unique(shared["sample"]["tile_id"])) == 4
    assert np.array_equal(tiled["sigma"], shared["sigma"])
    assert tiled["loss"] == shared["loss"]
    assert np.allclose(tiled["dtable"], shared["dtable"], rtol=0, atol=1e-15)
    dWk = tiled["dW"].reshape(4, -1)
    assert np.allclose(dWk.sum(0), shared["dW"], rtol=1e-12, atol=1e-18)
    # every tile holds samples, so every set receives a gradient of its own
    assert np.all(np.abs(dWk).sum(1) > 0)
    assert tiled["mlp_new"].shape == (4, W.shape[1])


def test_train_step_shared_colour_net(orc):
    """Per-tile density nets with one shared colour net: equal to the per-tile
    step whose four sets carry that same colour net, with the colour gradient
    the sum of the four per-tile colour gradients."""
    import copy
    wl = synth.tiny_tile(seed=6, n_rays=200, samples=16)
    wl = copy.copy(wl)
    wl.boxes = np.array([[0, 0, 0, 0.5, 0.5, 1], [0, 0.5, 0, 0.5, 1, 1], [0.5, 0, 0, 1, 0.5, 1],
                         [0.5, 0.5, 0, 1, 1, 1]], dtype=np.float64)
    rng = np.random.default_rng(4)
    wl.table = synth.init_table(rng, wl.grid, n_tiles=4) * np.float32(1e4)
    Pd = 64 * 32 + 16 * 64
    W = np.stack([synth.init_mlp(rng, wl.mlp) for _ in range(4)])
    W[:, Pd:] = W[0, Pd:]
    per_tile = orc.train_step(wl, mlp_params=W)
    shared = orc.train_step(wl, mlp_params={"density": W[:, :Pd], "colour": W[0, Pd:]})
    assert np.array_equal(shared["sigma"], per_tile["sigma"])
    assert shared["loss"] == per_tile["loss"]
    dWt = per_tile["dW"].reshape(4, -1)
    assert np.array_equal(shared["dW"][:4 * Pd], dWt[:, :Pd].ravel())
    assert np.allclose(shared["dW"][4 * Pd:], dWt[:, Pd:].sum(0), rtol=1e-13, atol=1e-20)
    assert shared["mlp_new"].size == 4 * Pd + W.shape[1] - Pd


def test_occupancy_cells_and_culling(orc):
    """Cell lookup: every cell centre maps to its own cell; x = 1 lands in the
    last cell.  Culling with every cell occupied is the identity; with none
    occupied it removes every sample; culling keeps each ray's kept samples in
    t order and a culled ray's composite equals the composite of its kept
    intervals (empty cells add no optical depth)."""
    G = 16
    c, t = orc.occupancy_cell_centres(G, K=2)
    assert np.array_equal(orc.occupancy_cell(c[:G ** 3], G), np.arange(G ** 3))
    assert orc.occupancy_cell(np.array([[1.0, 1.0, 1.0]]), G)[0] == G ** 3 - 1
    assert orc.occupancy_cell(np.array([[0.0, 0.5, 0.999]]), G)[0] == (0 * G + 8) * G + 15
    w = synth.tiny_tile(seed=11, n_rays=200, samples=40)
    smp = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 40)
    allon = orc.cull_samples(smp, np.ones(G ** 3, dtype=bool), G)
    assert allon["n"] == smp["n"] and np.array_equal(allon["packed_info"], smp["packed_info"])
    assert orc.cull_samples(smp, np.zeros(G ** 3, dtype=bool), G)["n"] == 0
    rng = np.random.default_rng(12)
    occ = rng.random(G ** 3) < 0.4
    cu = orc.cull_samples(smp, occ, G)
    assert 0 < cu["n"] < smp["n"]
    for r in range(200):
        s, n = cu["packed_info"][r]
        assert np.all(np.diff(cu["t0"][s:s + n]) > 0) and np.all(cu["ray_id"][s:s + n] == r)
    # density zero where culled: compositing all samples with sigma = 0 in
    # empty cells equals compositing the kept samples alone
    sig = rng.uniform(0.0, 5.0, size=smp["n"])
    rgb = rng.uniform(0.0, 1.0, size=(smp["n"], 3))
    keep = cu["keep"]
    full = orc.composite_fwd(smp["packed_info"], np.where(keep, sig, 0.0), rgb, smp["t0"], smp["t1"])
    kept = orc.composite_fwd(cu["packed_info"], sig[keep], rgb[keep], cu["t0"], cu["t1"])
    assert np.allclose(full["rgb"], kept["rgb"], rtol=1e-13, atol=1e-15)
    assert np.allclose(full["opacity"], kept["opacity"], rtol=1e-13, atol=1e-15)
    d, o = orc.occupancy_update(np.full(4, 1.0), np.array([0.0, 0.5, 2.0, 0.96]), 0.95, 0.96)
    assert np.allclose(d, [0.95, 0.95, 2.0, 0.96]) and o.tolist() == [False, False, True, False]
    # the step scale multiplies sigma, not the decayed estimate
    d, o = orc.occupancy_update(np.zeros(3), np.array([1.0, 3.0, 10.0]), 0.5, 0.02, scale=0.01)
    assert np.allclose(d, [0.01, 0.03, 0.1]) and o.tolist() == [False, True, True]


def test_refine_samples(orc):
    """Density-driven sampling after culling.  With every cell occupied the
    refinement is the uniform sampler itself, bit for bit (each kept interval
    gets exactly one sample at its own midpoint), which pins its position
    mapping to the sampler's.  With a partial grid every ray that keeps
    anything spends exactly its budget, each kept interval gets floor(B/c) or
    ceil(B/c) sub-intervals that tile it exactly (first starts at ta, last
    ends at tb, no gaps), every sample lies in its interval, and a ray that
    keeps nothing gets none.  Worked split: budget 5 over 2 intervals gives
    3 and 2; budget 7 over 3 gives 2, 3, 2."""
    G = 16
    w = synth.tiny_tile(seed=11, n_rays=120, samples=40)
    smp = orc.sample_segmented(w.rays_o, w.rays_d, w.boxes, 40)
    budget = smp["packed_info"][:, 1]
    allon = orc.cull_samples(smp, np.ones(G ** 3, dtype=bool), G)
    ref = orc.refine_samples(w.rays_o, w.rays_d, w.boxes, budget, allon)
    assert ref["n"] == smp["n"] and np.array_equal(ref["packed_info"], smp["packed_info"])
    for k in ("t0", "t1", "pos", "ray_id", "tile_id"):
        assert np.array_equal(ref[k], smp[k]), k
    rng = np.random.default_rng(13)
    occ = rng.random(G ** 3) < 0.3
    cu = orc.cull_samples(smp, occ, G)
    ref = orc.refine_samples(w.rays_o, w.rays_d, w.boxes, budget, cu)
    kept_any = cu["packed_info"][:, 1] > 0
    assert kept_any.any() and np.any(cu["packed_info"][:, 1] < budget)
    assert np.array_equal(ref["packed_info"][:, 1], np.where(kept_any, budget, 0))
    for r in range(120):
        s, c = cu["packed_info"][r]
        s2, n2 = ref["packed_info"][r]
        if c == 0:
            assert n2 == 0
            continue
        t0, t1 = ref["t0"][s2:s2 + n2], ref["t1"][s2:s2 + n2]
        assert np.all(ref["ray_id"][s2:s2 + n2] == r)
        # walk the kept intervals: each is tiled by floor/ceil(B/c) sub-intervals
        j = 0
        for i in range(c):
            ta, tb = cu["t0"][s + i], cu["t1"][s + i]
            q = 0
            while j + q < n2 and t0[j + q] >= ta and t1[j + q] <= tb:
                q += 1
            assert q in (n2 // c, -(-n2 // c)), (r, i, q)
            assert t0[j] == ta and t1[j + q - 1] == tb
            assert np.all(t1[j:j + q - 1] == t0[j + 1:j + q])
            assert np.all(t0[j:j + q] < t1[j:j + q])
            j += q
        assert j == n2
    assert np.all((ref["pos"] >= 0.0) & (ref["pos"] <= 1.0))
    # worked splits on a single ray with hand-made intervals
    ray_o, ray_d = np.array([[0.5, 0.5, 2.0]]), np.array([[0.0, 0.0, -1.0]])
    box = np.array([[0.0, 0.0, 0.0, 1.0, 1.0, 1.0]])
    for B, ivals, want in ((5, [(1.0, 1.2), (1.5, 1.6)], [3, 2]), (7, [(1.0, 1.1), (1.2, 1.3), (1.4, 1.5)], [2, 3, 2])):
        c = len(ivals)
        kept = dict(packed_info=np.array([[0, c]], dtype=np.int32),
                    t0=np.array([a for a, _ in ivals], dtype=np.float32),
                    t1=np.array([b for _, b in ivals], dtype=np.float32), tile_id=np.zeros(c, dtype=np.uint8))
        out = orc.refine_samples(ray_o, ray_d, box, np.array([B]), kept)
        got = [int(np.sum((out["t0"] >= np.float32(a)) & (out["t1"] <= np.float32(b)))) for a, b in ivals]
        assert got == want
        # the ray falls straight down through the box centre: z = 2 - t, clamped
        assert np.allclose(out["pos"][:, :2], 0.5) and np.allclose(out["pos"][:, 2], np.clip(2.0 - 0.5 * (out["t0"] + out["t1"]), 0, 1), atol=1e-6)


def test_occupancy_mean_cap(orc):
    """Mean cap: with every cell below the threshold, exactly the cells above
    the mean stay occupied; with the mean above the threshold the cap is
    inactive; a uniform field below the threshold is all empty (strict >)."""
    sig = np.array([0.001, 0.002, 0.003, 0.010])             # mean 0.004
    d, o = orc.occupancy_update(np.zeros(4), sig, 0.95, 0.01, mean_cap=True)
    assert o.tolist() == [False, False, False, True]
    d, o = orc.occupancy_update(np.zeros(4), sig, 0.95, 0.0025, mean_cap=True)
    assert o.tolist() == [False, False, True, True]
    big = np.array([0.5, 0.005, 0.02, 1.0])                  # mean 0.38 > 0.01
    _, o1 = orc.occupancy_update(np.zeros(4), big, 0.95, 0.01, mean_cap=True)
    _, o2 = orc.occupancy_update(np.zeros(4), big, 0.95, 0.01, mean_cap=False)
    assert o1.tolist() == o2.tolist() == [True, False, True, True]
    _, o = orc.occupancy_update(np.zeros(5), np.full(5, 0.001), 0.95, 0.01, mean_cap=True)
    assert not o.any()
