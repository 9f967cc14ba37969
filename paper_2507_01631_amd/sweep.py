"""The snake sweep of Snake-NeRF (Sec. 4.4): a 2x2 window slides over an
nx x ny grid of NeRF tiles along a snake path (left to right on even window
rows, right to left on odd ones), so that each move replaces two tiles and
keeps two.  Every tile keeps its hash table, density/colour networks and
their Adam state (moments and step) across windows -- training continues
without resetting the optimiser.

Memory: the state of all tiles lives in pinned host memory; the device holds
the window's four tiles (a ``WindowNeRF``) plus two staging slots for the
tiles that enter next and two for the tiles that just left.  A move is

  1. compute stream: the window's last step is enqueued; event E_done;
  2. copy stream (waits E_done): the two leaving tiles are copied device to
     device into the out-staging slots, the two staying tiles move to their
     new slots, the two entering tiles (prefetched earlier) move from the
     in-staging slots into theirs; event E_ready -- the compute stream waits
     on it before the next window's first step;
  3. copy stream: the out-staging slots go back to pinned host memory, and
     the tiles that enter at the following move are prefetched from pinned
     host memory into the in-staging slots.  Both copies overlap the next
     window's training.

The window step works in window-local coordinates (tiles [0,2]^2 x band), so
one captured HIP graph serves every window position; rays are given in the
same frame.  Copies use torch's pinned tensors and side stream (memory and
stream plumbing); all compute is the library's.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib as L
from .window import WindowNeRF


def snake_path(nx: int, ny: int):
    """Window positions (lower-left tile index) of the snake over an nx x ny
    tile grid: rows of windows bottom to top, alternating direction."""
    out = []
    for wy in range(ny - 1):
        xs = range(nx - 1) if wy % 2 == 0 else range(nx - 2, -1, -1)
        out.extend((wx, wy) for wx in xs)
    return out


def _slot(i, j):
    return 2 * i + j        # WindowNeRF box order: tile (wx + i, wy + j)


_COPY_STREAMS = {}


def _copy_stream(dev):
    """The device's copy stream: one per device, on a hardware queue of its
    own, kept until the process ends.  It is never destroyed, since torch's
    pinned-memory allocator records events on every stream a host block was
    copied on when that block is freed, which may be after any sweep ends."""
    idx = torch.device(dev).index
    idx = torch.cuda.current_device() if idx is None else idx
    if idx not in _COPY_STREAMS:
        with torch.cuda.device(idx):
            h = L.snake_stream_create_dedicated()
        _COPY_STREAMS[idx] = torch.cuda.ExternalStream(h, device=torch.device("cuda", idx))
    return _COPY_STREAMS[idx]


class SnakeSweep:
    """Pinned host store of every tile's state and the device window that
    slides over it."""

    FIELDS_T = ("table", "m_t", "v_t")
    FIELDS_W = ("params", "m_w", "v_w")

    def __init__(self, nx, ny, *, res, n_features, log2_table, n_dir, colour_layers, colour_out,
                 init_tile, precision="bf16", band=(0.0, 1.0), max_rays=1 << 16, samples=128,
                 early_stop=0.0, lr=1e-2, device="cuda"):
        assert nx >= 2 and ny >= 2
        self.nx, self.ny = int(nx), int(ny)
        dev = torch.device(device)
        self.device = dev
        boxes = np.array([[i, j, band[0], i + 1.0, j + 1.0, band[1]] for i in range(2) for j in range(2)])
        self.win = WindowNeRF(boxes=boxes, zband=None, res=res, n_features=n_features, log2_table=log2_table,
                              n_dir=n_dir, colour_layers=colour_layers, colour_out=colour_out,
                              precision=precision, max_rays=max_rays, samples=samples, early_stop=early_stop,
                              lr=lr, device=dev)
        w = self.win
        assert not w.shared_colour
        self.per_t = w.Lv * (1 << w.log2T) * w.F
        self.per_w = w.P
        n = self.nx * self.ny
        # host store: one pinned buffer per tile and field (many moderate
        # pinned allocations rather than a few of several GB each); every
        # tile's table and network weights come from init_tile(t) ->
        # (table [L*T*F] float32, weights [P] float32), its Adam state from zero
        n = self.nx * self.ny
        self.h = {}
        for f in self.FIELDS_T:
            self.h[f] = [torch.zeros(self.per_t, dtype=torch.float32).pin_memory() for _ in range(n)]
        for f in self.FIELDS_W:
            self.h[f] = [torch.zeros(self.per_w, dtype=torch.float32).pin_memory() for _ in range(n)]
        self.h["step"] = [torch.zeros(1, dtype=torch.int32).pin_memory() for _ in range(n)]
        for t in range(n):
            tab, par = init_tile(t)
            tab = np.ascontiguousarray(tab, dtype=np.float32).reshape(-1)
            par = np.ascontiguousarray(par, dtype=np.float32).reshape(-1)
            if tab.size != self.per_t or par.size != self.per_w:
                raise ValueError("init_tile(%d) gave %d table and %d weight values, expected %d and %d"
                                 % (t, tab.size, par.size, self.per_t, self.per_w))
            self.h["table"][t].copy_(torch.from_numpy(tab))
            self.h["params"][t].copy_(torch.from_numpy(par))
        # device staging: two slots in, two out
        mk = lambda k: torch.empty((2, k), dtype=torch.float32, device=dev)   # noqa: E731
        self.st_in = {f: mk(self.per_t) for f in self.FIELDS_T}
        self.st_in.update({f: mk(self.per_w) for f in self.FIELDS_W})
        self.st_in["step"] = torch.empty((2, 1), dtype=torch.int32, device=dev)
        self.st_out = {f: torch.empty_like(v) for f, v in self.st_in.items()}
        # the window trains on its own stream and the swaps run on a stream
        # with a hardware queue of its own: streams otherwise share a small
        # pool of queues, and a copy stream on the compute stream's queue
        # would run the host transfers after the training instead of beside it
        self.compute = torch.cuda.Stream(device=dev)
        self.copy = _copy_stream(dev)
        self.pos = None
        self.in_tiles = None       # tiles held in the in-staging slots
        self.out_tiles = None      # tiles held in the out-staging slots (pending copy-back)

    # -- device views of the window state per slot ---------------------------
    def _wview(self, f):
        w = self.win
        if f == "step":
            return w.step_dev[:4].view(4, 1)
        t = getattr(w, f)
        return t.view(4, -1)

    def tile_index(self, x, y):
        return x * self.ny + y

    def _load_window(self, pos):
        """Synchronous load of a whole window (the first position)."""
        wx, wy = pos
        for i in range(2):
            for j in range(2):
                t, s = self.tile_index(wx + i, wy + j), _slot(i, j)
                for f in self.FIELDS_T + self.FIELDS_W + ("step",):
                    self._wview(f)[s].copy_(self.h[f][t])
        for f in ("g_t", "g_w"):
            getattr(self.win, f).zero_()
        torch.cuda.synchronize()
        self.pos = pos

    def _move_plan(self, a, b):
        """(leaving, staying, entering) for a move between adjacent positions:
        lists of (tile, old slot), (old slot, new slot), (tile, new slot)."""
        (ax, ay), (bx, by) = a, b
        leave, stay, enter = [], [], []
        cur = {(ax + i, ay + j): _slot(i, j) for i in range(2) for j in range(2)}
        new = {(bx + i, by + j): _slot(i, j) for i in range(2) for j in range(2)}
        for t, s in cur.items():
            if t in new:
                stay.append((s, new[t]))
            else:
                leave.append((self.tile_index(*t), s))
        for t, s in new.items():
            if t not in cur:
                enter.append((self.tile_index(*t), s))
        return leave, stay, enter

    def _prefetch(self, tiles):
        """Copy-stream H2D of up to two tiles into the in-staging slots."""
        with torch.cuda.stream(self.copy):
            for k, t in enumerate(tiles):
                for f in self.FIELDS_T + self.FIELDS_W + ("step",):
                    self.st_in[f][k].copy_(self.h[f][t], non_blocking=True)
        self.in_tiles = list(tiles)

    def _writeback(self):
        """Copy-stream D2H of the out-staging slots to the host store."""
        if not self.out_tiles:
            return
        with torch.cuda.stream(self.copy):
            for k, t in enumerate(self.out_tiles):
                for f in self.FIELDS_T + self.FIELDS_W + ("step",):
                    self.h[f][t].copy_(self.st_out[f][k], non_blocking=True)
        self.out_tiles = None

    def _move(self, b, next_b):
        leave, stay, enter = self._move_plan(self.pos, b)
        assert [t for t, _ in enter] == self.in_tiles, "prefetch did not hold the entering tiles"
        done = torch.cuda.Event()
        done.record(torch.cuda.current_stream())
        ready = torch.cuda.Event()
        with torch.cuda.stream(self.copy):
            self.copy.wait_event(done)
            fields = self.FIELDS_T + self.FIELDS_W + ("step",)
            for k, (t, s) in enumerate(leave):
                for f in fields:
                    self.st_out[f][k].copy_(self._wview(f)[s])
            # a staying tile always moves into a slot just vacated by a leaving
            # tile (whose state is already in out-staging), never onto another
            # staying tile, so the moves can run in any order
            free = {s for _, s in leave}
            for s_old, s_new in stay:
                if s_old != s_new:
                    assert s_new in free
                    for f in fields:
                        self._wview(f)[s_new].copy_(self._wview(f)[s_old])
            for k, (t, s) in enumerate(enter):
                for f in fields:
                    self._wview(f)[s].copy_(self.st_in[f][k])
            ready.record(self.copy)
        torch.cuda.current_stream().wait_event(ready)
        self.out_tiles = [t for t, _ in leave]
        self.pos = b
        # overlap with the next window: write the leavers back, prefetch the next entering pair
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(self.copy)
        self._writeback()
        if next_b is not None:
            self._prefetch([t for t, _ in self._move_plan(b, next_b)[2]])
        else:
            self.in_tiles = None
        c1.record(self.copy)
        self._copy_events.append((c0, c1))

    # -- the sweep -----------------------------------------------------------
    def run(self, steps_per_window, batches, graph=True, log=None):
        """Train every window of the snake path for steps_per_window steps.
        batches(pos, k) returns (rays_o, rays_d, target, samples_per_ray) of
        window-local rays for step k at window position pos (device tensors
        of one fixed shape).  Returns per-window times (s)."""
        with torch.cuda.stream(self.compute):
            return self._run(steps_per_window, batches, graph, log)

    def _run(self, steps_per_window, batches, graph, log):
        path = snake_path(self.nx, self.ny)
        self._copy_events = []
        self._load_window(path[0])
        if len(path) > 1:
            self._prefetch([t for t, _ in self._move_plan(path[0], path[1])[2]])
        ro, rd, tg, spr = (x.clone() for x in batches(path[0], 0))
        static = (ro, rd, tg, spr)
        if graph:
            self.win.capture(*static, warmup=1)
        times = []
        self._compute_events, self._issue_s = [], []
        for wi, pos in enumerate(path):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if wi > 0:
                self._move(pos, path[wi + 1] if wi + 1 < len(path) else None)
            self._issue_s.append(time.perf_counter() - t0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for k in range(steps_per_window):
                b = batches(pos, k)
                for dst, src in zip(static, b):
                    dst.copy_(src, non_blocking=True)
                if graph:
                    self.win.replay()
                else:
                    self.win.step(*static)
            e1.record()
            self._compute_events.append((e0, e1))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if log:
                log("  window %d at %s: %.1f ms" % (wi, pos, 1e3 * times[-1]))
        # final write-back of the window's four tiles
        torch.cuda.synchronize()
        self.copy.synchronize()
        wx, wy = self.pos
        for i in range(2):
            for j in range(2):
                t, s = self.tile_index(wx + i, wy + j), _slot(i, j)
                for f in self.FIELDS_T + self.FIELDS_W + ("step",):
                    self.h[f][t].copy_(self._wview(f)[s])
        torch.cuda.synchronize()
        return times

    def compute_ms(self):
        """Compute-stream time of each window's training steps (from after its
        move to its last step), in ms, after run()."""
        return [a.elapsed_time(b) for a, b in self._compute_events]

    def move_issue_ms(self):
        """Host time to issue each window's move (copies and events), in ms."""
        return [1e3 * x for x in self._issue_s]

    def copy_ms(self):
        """Copy-stream time of each move's host transfers (write-back of the two
        leaving tiles, prefetch of the next two), in ms, after run()."""
        return [a.elapsed_time(b) for a, b in self._copy_events]

    def trained_steps(self):
        """Adam steps each tile has taken (1, 2 or 4 windows' worth)."""
        return torch.cat(self.h["step"]).view(self.nx, self.ny).clone()
