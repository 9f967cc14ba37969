"""The 2x2 window of Snake-NeRF (Sec. 4.4): four NeRF tiles, each with its own
hash table and density/colour networks, trained together on the rays of the
loaded window.

One window step, every stage a libsnake kernel launched once for all tiles:

    snake_sample_grouped (K boxes, per-ray budgets; rays cut at tile faces;
       samples written grouped by tile, with the map from packed order)
    -> snake_hashgrid_fwd (K tables, tile id per sample)
    -> snake_mlp_fwd (K weight sets, one per 64-sample unit)
    -> snake_composite_fwd / _bwd (per ray across tiles, sample map = inverse
       grouping, so the quadrature runs over the whole ray)
    -> snake_mlp_bwd (K weight sets) -> snake_hashgrid_bwd (K tables)
    -> snake_counter_add + snake_adam_step (all tables, all networks)

Nothing in the step reads a device value on the host, so after a warm-up the
whole step is captured in one HIP graph (``capture``) and replayed
(``replay``) on fresh rays copied into the captured input buffers.

``accept`` applies the window's ray acceptance (rays that cross only the
loaded tiles), the filter from which training batches are drawn.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


class WindowNeRF:
    """K (normally 4) tile NeRFs with separate tables and networks."""

    def __init__(self, *, boxes, zband, res, n_features, log2_table, n_dir, colour_layers, colour_out,
                 precision="bf16", tables=None, mlp_params=None, max_rays=1 << 16, max_samples=None,
                 samples=128, early_stop=0.0, lr=1e-2, betas=(0.9, 0.99), eps=1e-15, hash_ws_gib=16.0,
                 shared_colour=False, lr_colour=None, table_bf16=None, device="cuda"):
        self.device = torch.device(device)
        self.boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 6)
        self.K = self.boxes.shape[0]
        assert 1 <= self.K <= 16
        self.zband = None if zband is None else np.asarray(zband, dtype=np.float64)
        self.res = [int(r) for r in res]
        self.Lv, self.F, self.log2T = len(self.res), int(n_features), int(log2_table)
        self.S = int(samples)
        self.early_stop = float(early_stop)
        bf = precision == "bf16"
        self.precision = precision
        self.feat_dtype = L.SNAKE_BF16 if bf else L.SNAKE_F32
        self.grid = L.grid_desc(self.res, self.F, self.log2T, self.feat_dtype)
        # table_bf16 (default: the BF16 form): the forward gathers from a BF16
        # copy of the tables, refreshed from the FP32 masters at each step
        self.table_bf16 = bf if table_bf16 is None else bool(table_bf16)
        self.grid_fwd = (L.grid_desc(self.res, self.F, self.log2T, self.feat_dtype, L.SNAKE_GRID_TABLE_BF16)
                         if self.table_bf16 else self.grid)
        # shared_colour: density nets per tile, one global colour net (Sec. 4.1)
        # with its own optimiser; weights are [K][Pd] then the colour set
        self.shared_colour = bool(shared_colour)
        self.mlp = L.mlp_desc(self.Lv, self.F, n_dir, colour_layers, colour_out,
                              L.SNAKE_BF16 if bf else L.SNAKE_F32, self.feat_dtype, int(self.shared_colour))
        self.n_dir = int(n_dir)
        self.P = L.snake_mlp_param_count(self.mlp)
        self.Pd = 64 * 32 + 16 * 64
        self.n_w = L.snake_mlp_weight_count(self.mlp, self.K)
        dev = self.device
        tshape = (self.K, self.Lv, 1 << self.log2T, self.F)
        self.table = (torch.zeros(tshape, device=dev) if tables is None else
                      torch.as_tensor(np.ascontiguousarray(tables, dtype=np.float32)).to(dev).reshape(tshape))
        self.params = (torch.zeros(self.n_w, device=dev) if mlp_params is None else
                       torch.as_tensor(np.ascontiguousarray(mlp_params, dtype=np.float32)).to(dev)
                       .reshape(self.n_w))
        self.m_t, self.v_t, self.g_t = (torch.zeros_like(self.table) for _ in range(3))
        self.table_h = torch.empty(tshape, dtype=torch.bfloat16, device=dev) if self.table_bf16 else None
        self.m_w, self.v_w, self.g_w = (torch.zeros_like(self.params) for _ in range(3))
        self.lr, (self.b1, self.b2), self.eps = float(lr), betas, float(eps)
        self.lr_colour = self.lr if lr_colour is None else float(lr_colour)
        # Adam step of each tile (its own optimiser state travels with it when
        # the window slides), and of the shared colour net at index K
        self.step_dev = torch.zeros(self.K + 1, dtype=torch.int32, device=dev)
        self.hash_ws_gib = float(hash_ws_gib)
        self.graph = None
        self._alloc(int(max_rays), int(max_samples) if max_samples else int(max_rays) * self.S)

    # -- buffers -----------------------------------------------------------
    def _alloc(self, R, cap):
        dev, i32, f32, i64 = self.device, torch.int32, torch.float32, torch.int64
        self.R, self.cap = R, cap
        self.packed_info = torch.zeros((R, 2), dtype=i32, device=dev)
        self.t0 = torch.empty(cap, dtype=f32, device=dev)
        self.t1 = torch.empty(cap, dtype=f32, device=dev)
        self.view = torch.empty((R, 3), dtype=f32, device=dev)
        self.n_out = torch.zeros(1, dtype=i64, device=dev)
        # samples grouped by tile; inv maps a packed (ray-major) index to its grouped one
        self.inv = torch.empty(cap, dtype=i32, device=dev)
        self.tile_start = torch.zeros(self.K + 2, dtype=i64, device=dev)
        self.pos_s = torch.empty((cap, 3), dtype=f32, device=dev)
        self.tile_s = torch.empty(cap, dtype=torch.uint8, device=dev)
        self.ray_s = torch.empty(cap, dtype=i32, device=dev)
        fdt = torch.bfloat16 if self.feat_dtype == L.SNAKE_BF16 else f32
        self.feat = torch.empty((self.Lv, cap, self.F), dtype=fdt, device=dev)
        self.sigma = torch.empty(cap, dtype=f32, device=dev)
        self.rgb = torch.empty((cap, 3), dtype=f32, device=dev)
        self.rgb_out = torch.empty((R, 3), dtype=f32, device=dev)
        self.opacity = torch.empty(R, dtype=f32, device=dev)
        self.depth = torch.empty(R, dtype=f32, device=dev)
        self.n_alive = torch.empty(R, dtype=i32, device=dev)
        self.loss = torch.zeros(1, dtype=f32, device=dev)
        self.dsigma = torch.empty(cap, dtype=f32, device=dev)
        self.drgb = torch.empty((cap, 3), dtype=f32, device=dev)
        self.dfeat = torch.empty((self.Lv, cap, self.F), dtype=f32, device=dev)
        self.ws_sample = torch.empty(L.snake_sample_grouped_workspace_bytes(R, self.K), dtype=torch.uint8,
                                     device=dev)
        self.ws_mlp = torch.empty(L.snake_mlp_bwd_workspace_bytes(self.mlp, self.K), dtype=torch.uint8,
                                  device=dev)
        budget = int(self.hash_ws_gib * (1 << 30))
        lg = 1
        for c in range(self.Lv, 0, -1):
            nb = L.snake_hashgrid_bwd_workspace_bytes(self.grid, self.K, cap, c)
            if cap * c * 8 <= 2**31 - 1 and 0 < nb <= budget:
                lg = c
                break
        self.ws_hash = torch.empty(L.snake_hashgrid_bwd_workspace_bytes(self.grid, self.K, cap, lg),
                                   dtype=torch.uint8, device=dev)

    # -- ray acceptance ----------------------------------------------------
    def window_rect(self):
        b = self.boxes
        return (b[:, 0].min(), b[:, 1].min(), b[:, 3].max(), b[:, 4].max())

    def band(self):
        if self.zband is not None:
            return tuple(self.zband)
        return (self.boxes[:, 2].min(), self.boxes[:, 5].max())

    def accept(self, rays_o, rays_d, stream=None):
        """Indices of the rays (device FP64 [R][3] each) this window may train on,
        and their device count."""
        R = int(rays_o.shape[0])
        idx = torch.empty(max(R, 1), dtype=torch.int32, device=self.device)
        n = torch.zeros(1, dtype=torch.int64, device=self.device)
        ws = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=self.device)
        L.snake_window_accept(rays_o, rays_d, R, self.window_rect(), self.band(), None, idx, n, ws,
                              stream=stream)
        return idx, n

    # -- the step ----------------------------------------------------------
    def step(self, rays_o, rays_d, target, samples_per_ray=None, sun=None, stream=None, update=True):
        """One training step of the window on R rays (device tensors; R fixed
        by the buffers given at capture time when replayed).  update=False
        stops before Adam and leaves the gradients in g_t / g_w."""
        R = int(rays_o.shape[0])
        assert R <= self.R
        cap, K = self.cap, self.K
        self.loss.zero_()
        scale = 1.0 / (3.0 * R)
        L.snake_sample_grouped(rays_o, rays_d, R, self.boxes, self.zband, samples_per_ray, self.S, None,
                               self.packed_info, self.t0, self.t1, self.view, self.pos_s, self.ray_s, self.tile_s,
                               self.inv, self.tile_start, cap, self.n_out, self.ws_sample, stream)
        if self.table_bf16:
            L.snake_convert_bf16(self.table, self.table.numel(), self.table_h, stream)
        L.snake_hashgrid_fwd(self.grid_fwd, K, self.table_h if self.table_bf16 else self.table, self.pos_s,
                             self.tile_s, None, cap, self.n_out, self.feat, None, stream)
        L.snake_mlp_fwd(self.mlp, self.params, self.feat, self.view, sun, self.ray_s, R, None, cap, self.n_out,
                        self.sigma, self.rgb, K=K, tile_start=self.tile_start, stream=stream)
        L.snake_composite_fwd(self.sigma, self.rgb, self.t0, self.t1, self.packed_info, R, self.early_stop,
                              target, scale, self.rgb_out, self.opacity, self.depth, self.n_alive, self.loss,
                              sample_map=self.inv, stream=stream)
        # samples past a ray's early stop get zero adjoints, so the networks and
        # the table see them without changing any gradient
        L.snake_composite_bwd(self.sigma, self.rgb, self.t0, self.t1, self.packed_info, R,
                              self.n_alive if self.early_stop > 0 else None, target, scale, self.dsigma,
                              self.drgb, sample_map=self.inv, stream=stream)
        L.snake_mlp_bwd(self.mlp, self.params, self.feat, cap, self.view, sun, self.ray_s, R, None, cap,
                        self.n_out, self.dsigma, self.drgb, self.g_w, self.dfeat, self.ws_mlp, K=K,
                        tile_start=self.tile_start, stream=stream)
        L.snake_hashgrid_bwd(self.grid, K, self.pos_s, self.tile_s, None, cap, self.n_out, self.dfeat, self.g_t,
                             self.ws_hash, stream)
        if not update:
            return
        L.snake_counter_add(self.step_dev, 1, stream=stream)
        self.adam(stream)

    def adam(self, stream=None):
        """Adam per tile (table and networks of tile k use step counter k) and,
        with a shared colour net, for the colour net (counter K)."""
        per_t = self.Lv * (1 << self.log2T) * self.F
        per_w = self.Pd if self.shared_colour else self.P
        flags = L.SNAKE_ADAM_ZERO_GRAD
        # every tile's table, then every tile's networks: one launch each
        L.snake_adam_step_tiles(self.table, self.g_t, self.m_t, self.v_t, per_t, self.K, self.lr, self.b1, self.b2,
                                self.eps, self.step_dev, 0.0, flags, stream=stream)
        L.snake_adam_step_tiles(self.params, self.g_w, self.m_w, self.v_w, per_w, self.K, self.lr, self.b1, self.b2,
                                self.eps, self.step_dev, 0.0, flags, stream=stream)
        if self.shared_colour:
            c = self.K * self.Pd
            L.snake_adam_step(self.params[c:], self.g_w[c:], self.m_w[c:], self.v_w[c:], self.n_w - c,
                              self.lr_colour, self.b1, self.b2, self.eps, 0, 0.0, flags,
                              step_dev=self.step_dev[self.K:], stream=stream)

    # -- rendering ---------------------------------------------------------
    def render_depth(self, rays_o, rays_d, samples_per_ray=None, sun=None, stream=None):
        """Forward-only pass (grouped sampler, encoding, networks,
        quadrature) over any number of rays, in batches of the buffer size;
        returns the expected depth t of each ray (device FP32)."""
        N = int(rays_o.shape[0])
        depth = torch.empty(N, dtype=torch.float32, device=self.device)
        cap, K = self.cap, self.K
        for b0 in range(0, N, self.R):
            b1 = min(N, b0 + self.R)
            R = b1 - b0
            spr = None if samples_per_ray is None else samples_per_ray[b0:b1]
            L.snake_sample_grouped(rays_o[b0:b1], rays_d[b0:b1], R, self.boxes, self.zband, spr, self.S, None,
                                   self.packed_info, self.t0, self.t1, self.view, self.pos_s, self.ray_s,
                                   self.tile_s, self.inv, self.tile_start, cap, self.n_out, self.ws_sample, stream)
            L.snake_hashgrid_fwd(self.grid, K, self.table, self.pos_s, self.tile_s, None, cap, self.n_out,
                                 self.feat, None, stream)
            L.snake_mlp_fwd(self.mlp, self.params, self.feat, self.view, None if sun is None else sun[b0:b1],
                            self.ray_s, R, None, cap, self.n_out, self.sigma, self.rgb, K=K,
                            tile_start=self.tile_start, stream=stream)
            L.snake_composite_fwd(self.sigma, self.rgb, self.t0, self.t1, self.packed_info, R, self.early_stop,
                                  None, 0.0, self.rgb_out, self.opacity, self.depth, self.n_alive, None,
                                  sample_map=self.inv, stream=stream)
            depth[b0:b1].copy_(self.depth[:R])
        return depth

    # -- HIP graph ---------------------------------------------------------
    def capture(self, rays_o, rays_d, target, samples_per_ray=None, sun=None, warmup=1):
        """Capture one step on these (static) input buffers into a HIP graph.
        The warm-up steps run eagerly first (they are training steps)."""
        self._static = (rays_o, rays_d, target, samples_per_ray, sun)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.step(*self._static)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(*self._static)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
