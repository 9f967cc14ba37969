"""Host-side logic that needs no GPU: the snake path (with the per-tile window
count of Sec. 4.4 as a fixture) and the swap plan of the sweep, the
coordinate-descent autotuner (with a synthetic cost), the bench's roofline
bookkeeping and its refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("nx,ny", [(2, 2), (3, 3), (4, 3), (8, 8)])
def test_snake_path_visits_every_window_by_single_moves(nx, ny):
    from paper_2507_01631_amd.sweep import snake_path
    path = snake_path(nx, ny)
    assert len(path) == (nx - 1) * (ny - 1)
    assert sorted(path) == sorted((x, y) for x in range(nx - 1) for y in range(ny - 1))
    for a, b in zip(path, path[1:]):
        assert abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1        # neighbouring windows


def _golden_multiplicity():
    grids, cur = [], None
    with open(os.path.join(ROOT, "tests", "golden", "snake_window_multiplicity.txt")) as f:
        for line in f:
            words = line.split("#", 1)[0].split()
            if not words:
                continue
            if words[0] == "grid":
                cur = (int(words[1]), int(words[2]), [])
                grids.append(cur)
            else:
                cur[2].append([int(w) for w in words])
    return grids


def test_snake_path_trains_corners_once_edges_twice_interior_four_times():
    """Sec. 4.4: over one sweep a corner tile sits in 1 window, an edge tile in 2,
    an interior tile in 4 (fixture written from that rule, north row first)."""
    from paper_2507_01631_amd.sweep import snake_path
    grids = _golden_multiplicity()
    assert {(3, 3), (4, 4), (8, 8)} <= {(nx, ny) for nx, ny, _ in grids}
    for nx, ny, rows in grids:
        assert len(rows) == ny and all(len(r) == nx for r in rows)
        want = np.array(rows[::-1]).T                 # indexed [x][y]
        got = np.zeros((nx, ny), dtype=np.int64)
        for wx, wy in snake_path(nx, ny):
            got[wx:wx + 2, wy:wy + 2] += 1
        np.testing.assert_array_equal(got, want, err_msg=f"{nx}x{ny}")
        assert got.sum() == 4 * (nx - 1) * (ny - 1)


@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (8, 8)])
def test_move_plan_swaps_two_tiles_and_frees_the_slots_it_fills(nx, ny):
    from paper_2507_01631_amd.sweep import SnakeSweep, snake_path

    class Grid:                         # the plan needs only the tile numbering
        def __init__(self):
            self.ny = ny

        def tile_index(self, x, y):
            return x * ny + y
    g = Grid()
    path = snake_path(nx, ny)
    for a, b in zip(path, path[1:]):
        leave, stay, enter = SnakeSweep._move_plan(g, a, b)
        assert len(leave) == 2 and len(stay) == 2 and len(enter) == 2
        vacated = {s for _, s in leave}
        filled = {s_new for s_old, s_new in stay if s_new != s_old} | {s for _, s in enter}
        # every slot is filled exactly once, and only slots that were vacated
        # or left by a staying tile are written
        moved_from = {s_old for s_old, s_new in stay if s_new != s_old}
        assert filled <= vacated | moved_from
        assert len({s for _, s in enter} | {s_new for _, s_new in stay}) == 4
        for s_old, s_new in stay:
            if s_old != s_new:
                assert s_new in vacated          # never onto another staying tile
        # the tiles of window b are exactly the staying and entering ones
        bx, by = b
        want = {g.tile_index(bx + i, by + j) for i in range(2) for j in range(2)}
        ax, ay = a
        cur = {2 * i + j: g.tile_index(ax + i, ay + j) for i in range(2) for j in range(2)}
        got = {cur[s_old] for s_old, _ in stay} | {t for t, _ in enter}
        assert got == want


def test_autotune_coordinate_descent_finds_the_separable_optimum(monkeypatch):
    from paper_2507_01631_amd import _lib as L
    from paper_2507_01631_amd import autotune
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libsnake.so is not built")
    saved = autotune.current()
    best = {"hash_fwd_blocks_per_cu": 8, "bin_blocks": 512, "sampler_blocks_per_cu": 32}

    def cost():                         # separable: each tunable's own distance
        c = 1.0
        for k, v in best.items():
            c += abs(np.log2(L.snake_tune_get(k)) - np.log2(v))
        return c
    monkeypatch.setattr(autotune, "time_step", lambda step, reps=5, warmup=2: cost())
    cand = {k: autotune.CANDIDATES[k] for k in best}
    try:
        table, ms, trace = autotune.tune(lambda: None, candidates=cand)
        for k, v in best.items():
            assert table[k] == v and L.snake_tune_get(k) == v
        assert ms == 1.0 and len(trace) > 1
    finally:
        autotune.apply(saved)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "--gpus 2 is not supported" in r.stderr


def test_bench_roofline_bookkeeping():
    sys.path.insert(0, ROOT)
    import bench
    import synth
    wl = synth.tiny_tile(seed=0, n_rays=64)
    stages = {k: 1.0 for k in bench.STAGES}
    form = dict(L=16, F=2, samples_total=1e6, samples_alive=1e6, stage_ms=stages, params=1000, table_params=800,
                table_bf16=True)
    rl = bench.roofline(form, wl, "bf16", 1024)
    # algorithmic table-adjoint bytes: 16 + L F 4 + L 8 F 4 2 per kept sample, in 1 ms
    assert rl["hash_bwd"]["per_launch"] == pytest.approx(1e6 * (16 + 16 * 2 * 4 + 16 * 8 * 2 * 4 * 2))
    assert rl["hash_bwd"]["achieved"] == pytest.approx(rl["hash_bwd"]["per_launch"] / 1e-3)
    # the BF16 mirror halves the forward's gathered bytes and adds its refresh
    assert rl["hash_fwd"]["per_launch"] == pytest.approx(1e6 * (12 + 16 * 8 * 2 * 2 + 16 * 2 * 2) + 800 * 6)
    assert rl["adam"]["per_launch"] == pytest.approx(1000 * 28)
    # counter-measured traffic only for the sources and workload it was taken on
    assert bench.adjoint_traffic("fp32", 1 << 18) is None
    assert bench.adjoint_traffic("bf16", 1 << 17) is None
