"""One training step of a tile NeRF on the HIP library.

Stage order (Snake-NeRF: segmented sampling Sec. 4.5 -> hash encoding and
density/colour nets Sec. 4.1 -> volume rendering and colour-consistency loss
Sec. 4.4 -> adjoints -> Adam, the I-NGP strategy of Sec. 4.6):

    snake_sample_segmented -> snake_hashgrid_fwd -> snake_mlp_fwd
    -> snake_composite_fwd (early stop -> n_alive)
    -> snake_composite_bwd -> snake_pack_alive
    -> snake_mlp_bwd (recompute, or stored activations)
    -> snake_hashgrid_bwd (binned exact integer sums, or FP32 atomics)
    -> snake_adam_step (table) + snake_adam_step (MLP)

PyTorch only owns device memory and the stream; every step runs in libsnake.
No call synchronises the host, so a step can be captured in a HIP graph.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as L


def level_resolutions(n_levels: int, res_min: int, res_max: int) -> list:
    """Geometric level resolutions of the multiresolution encoding:
    N_l = floor(N_min b^l + 1e-6), b = exp(ln(N_max/N_min) / (L-1))."""
    if n_levels == 1:
        return [int(res_min)]
    b = math.exp(math.log(res_max / res_min) / (n_levels - 1))
    return [int(math.floor(res_min * math.pow(b, l) + 1e-6)) for l in range(n_levels)]


def _as_dev(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


class TileNeRF:
    """Parameters, Adam state and step buffers of one (or K) tile NeRF(s).

    The K tiles share one MLP; each has its own hash table slice
    [K][L][T][F].  ``precision`` is "fp32" (FP32 MFMA) or "bf16" (BF16 MFMA
    with FP32 accumulation; features stored in bf16)."""

    def __init__(self, *, res, n_features, log2_table, n_dir, colour_layers, colour_out,
                 boxes, zband=None, samples=64, early_stop=0.0, precision="fp32",
                 table=None, mlp_params=None, max_rays=4096, lr=1e-2, betas=(0.9, 0.99),
                 eps=1e-15, hash_bwd="binned", hash_ws_gib=24.0, recompute=True, occ_grid=0,
                 occ_decay=0.95, occ_threshold=0.01, occ_mean_cap=True, occ_refine=False, table_bf16=None,
                 device="cuda"):
        self.device = torch.device(device)
        self.res = [int(r) for r in res]
        self.F = int(n_features)
        self.log2T = int(log2_table)
        self.boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 6)
        self.K = self.boxes.shape[0]
        self.zband = None if zband is None else np.asarray(zband, dtype=np.float64)
        self.S = int(samples)
        self.early_stop = float(early_stop)
        self.precision = precision
        bf = precision == "bf16"
        self.feat_dtype = L.SNAKE_BF16 if bf else L.SNAKE_F32
        self.grid = L.grid_desc(self.res, self.F, self.log2T, self.feat_dtype)
        self.mlp = L.mlp_desc(len(self.res), self.F, n_dir, colour_layers, colour_out,
                              L.SNAKE_BF16 if bf else L.SNAKE_F32, self.feat_dtype)
        self.n_dir = int(n_dir)
        self.P = L.snake_mlp_param_count(self.mlp)
        T = 1 << self.log2T
        shape = (self.K, len(self.res), T, self.F)
        dev = self.device
        self.table = (torch.zeros(shape, dtype=torch.float32, device=dev) if table is None
                      else _as_dev(table, torch.float32, dev).reshape(shape))
        self.params = (torch.zeros(self.P, dtype=torch.float32, device=dev) if mlp_params is None
                       else _as_dev(mlp_params, torch.float32, dev).reshape(self.P))
        self.m_t = torch.zeros_like(self.table)
        self.v_t = torch.zeros_like(self.table)
        self.g_t = torch.zeros_like(self.table)
        # table_bf16 (default: the BF16 form): the forward gathers from a BF16
        # copy of the table, refreshed from the FP32 master before each forward
        # (mixed-precision NGP parameters); adjoint and Adam stay FP32
        self.table_bf16 = bf if table_bf16 is None else bool(table_bf16)
        self.grid_fwd = self.grid
        if self.table_bf16:
            self.table_h = torch.empty(shape, dtype=torch.bfloat16, device=dev)
            self.grid_fwd = L.grid_desc(self.res, self.F, self.log2T, self.feat_dtype, L.SNAKE_GRID_TABLE_BF16)
        self.m_w = torch.zeros_like(self.params)
        self.v_w = torch.zeros_like(self.params)
        self.g_w = torch.zeros_like(self.params)
        self.lr, (self.b1, self.b2), self.eps = float(lr), betas, float(eps)
        # "binned": sort corner gradients by table slot and sum them in LDS;
        # "atomic": one FP32 atomic add per corner contribution
        assert hash_bwd in ("binned", "atomic")
        self.hash_bwd, self.hash_ws_gib = hash_bwd, float(hash_ws_gib)
        # recompute=False: the forward stores every sample's activations and the
        # adjoint reads them back instead of recomputing them
        self.recompute = bool(recompute)
        self.act = None
        # occ_grid = G > 0: coarse occupancy grid of G^3 cells per tile; samples in
        # unoccupied cells are culled after sampling (SAT-NGP procedure, Sec. 4.1).
        # The grid holds a decaying maximum of the optical thickness sigma * step
        # of one nominal sample step (band height / samples, unit-length rays) at
        # the cell centres; a cell is occupied while that exceeds occ_threshold,
        # capped at the grid's mean when occ_mean_cap is set.
        # occ_refine: after culling, each ray spends its whole sample budget on
        # the intervals it kept (the grid sets each segment's sample density)
        self.G = int(occ_grid)
        self.occ_refine = bool(occ_refine) and self.G > 0
        self.occ_decay, self.occ_threshold = float(occ_decay), float(occ_threshold)
        self.occ_flags = L.SNAKE_OCC_MEAN_CAP if occ_mean_cap else 0
        b = self.boxes
        zlo, zhi = float(b[:, 2].min()), float(b[:, 5].max())
        if self.zband is not None:
            zlo, zhi = max(zlo, float(self.zband[0])), min(zhi, float(self.zband[1]))
        self.occ_step = (zhi - zlo) / self.S
        if self.G:
            nc = self.K * self.G ** 3
            # every cell occupied until the first update; the estimate then
            # starts from what the networks report at the cell centres
            self.occ_density = torch.zeros((nc,), device=self.device)
            self.occ_bits = torch.full(((nc + 31) // 32,), -1, dtype=torch.int32, device=self.device)
            self.occ_pos = torch.empty((nc, 3), device=self.device)
            self.occ_tile = torch.empty(nc, dtype=torch.uint8, device=self.device) if self.K > 1 else None
            self.ws_occ = torch.empty(L.snake_occupancy_workspace_bytes(nc), dtype=torch.uint8, device=self.device)
            L.snake_occupancy_cells(self.G, self.K, self.occ_pos, self.occ_tile)
        self.step_count = 0
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.R = 0
        self.R_cur = 0
        self.alloc(max_rays)

    # -- buffers -----------------------------------------------------------
    def alloc(self, R: int):
        R = int(R)
        if R <= self.R:
            return
        dev = self.device
        cap = R * self.S
        i32, f32, i64 = torch.int32, torch.float32, torch.int64
        self.R, self.cap = R, cap
        self.packed_info = torch.zeros((R, 2), dtype=i32, device=dev)
        self.t0 = torch.empty(cap, dtype=f32, device=dev)
        self.t1 = torch.empty(cap, dtype=f32, device=dev)
        self.pos = torch.empty((cap, 3), dtype=f32, device=dev)
        self.ray_id = torch.empty(cap, dtype=i32, device=dev)
        self.tile_id = torch.empty(cap, dtype=torch.uint8, device=dev) if self.K > 1 else None
        self.view = torch.empty((R, 3), dtype=f32, device=dev)
        self.n_out = torch.zeros(1, dtype=i64, device=dev)
        fdt = torch.bfloat16 if self.feat_dtype == L.SNAKE_BF16 else f32
        self.feat = torch.empty((len(self.res), cap, self.F), dtype=fdt, device=dev)
        self.sigma = torch.empty(cap, dtype=f32, device=dev)
        self.rgb = torch.empty((cap, 3), dtype=f32, device=dev)
        self.rgb_out = torch.empty((R, 3), dtype=f32, device=dev)
        self.opacity = torch.empty(R, dtype=f32, device=dev)
        self.depth = torch.empty(R, dtype=f32, device=dev)
        self.n_alive = torch.empty(R, dtype=i32, device=dev)
        self.loss = torch.zeros(1, dtype=f32, device=dev)
        self.dsigma = torch.empty(cap, dtype=f32, device=dev)
        self.drgb = torch.empty((cap, 3), dtype=f32, device=dev)
        self.alive_idx = torch.empty(cap, dtype=i32, device=dev)
        self.n_alive_total = torch.zeros(1, dtype=i64, device=dev)
        self.dfeat = torch.empty((len(self.res), cap, self.F), dtype=f32, device=dev)
        self.ws_sample = torch.empty(L.snake_sample_workspace_bytes(R), dtype=torch.uint8, device=dev)
        self.ws_mlp = torch.empty(L.snake_mlp_bwd_workspace_bytes(self.mlp), dtype=torch.uint8,
                                  device=dev)
        if not self.recompute:
            self.act = torch.empty((cap, L.snake_mlp_act_width(self.mlp)), dtype=f32, device=dev)
        if self.G:
            # the sampler writes here; culling packs the kept samples into the
            # arrays the rest of the step reads
            self.raw = dict(packed_info=torch.zeros((R, 2), dtype=i32, device=dev),
                            t0=torch.empty(cap, dtype=f32, device=dev), t1=torch.empty(cap, dtype=f32, device=dev),
                            pos=torch.empty((cap, 3), dtype=f32, device=dev),
                            ray_id=torch.empty(cap, dtype=i32, device=dev),
                            tile_id=torch.empty(cap, dtype=torch.uint8, device=dev) if self.K > 1 else None,
                            n=torch.zeros(1, dtype=i64, device=dev))
            self.ws_cull = torch.empty(L.snake_cull_workspace_bytes(R), dtype=torch.uint8, device=dev)
            if self.occ_refine:
                # culling packs the kept intervals here; the refinement writes
                # the arrays the rest of the step reads
                self.kept = {k: torch.empty_like(v) if v is not None else None for k, v in self.raw.items()}
        self.ws_hash = None
        if self.hash_bwd == "binned":
            # as many levels per pass as fit in the budget (at least one)
            budget = int(self.hash_ws_gib * (1 << 30))
            nlev = len(self.res)
            lg = 1
            for c in range(nlev, 0, -1):
                if cap * c * 8 <= 2**31 - 1 and \
                        L.snake_hashgrid_bwd_workspace_bytes(self.grid, self.K, cap, c) <= budget:
                    lg = c
                    break
            nbytes = L.snake_hashgrid_bwd_workspace_bytes(self.grid, self.K, cap, lg)
            self.ws_hash = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    # -- stages ------------------------------------------------------------
    def sample(self, rays_o, rays_d, R, samples_per_ray=None, stream=None):
        self.R_cur = int(R)
        if not self.G:
            L.snake_sample_segmented(rays_o, rays_d, R, self.boxes, self.zband, samples_per_ray, self.S,
                                     None, self.packed_info, self.t0, self.t1, self.pos, self.ray_id,
                                     self.tile_id, self.view, self.cap, self.n_out, self.ws_sample,
                                     stream)
            return
        r = self.raw
        L.snake_sample_segmented(rays_o, rays_d, R, self.boxes, self.zband, samples_per_ray, self.S, None,
                                 r["packed_info"], r["t0"], r["t1"], r["pos"], r["ray_id"], r["tile_id"], self.view,
                                 self.cap, r["n"], self.ws_sample, stream)
        if not self.occ_refine:
            L.snake_cull_samples(self.G, self.occ_bits, self.K, R, r["packed_info"], r["t0"], r["t1"], r["pos"],
                                 r["ray_id"], r["tile_id"], self.packed_info, self.t0, self.t1, self.pos, self.ray_id,
                                 self.tile_id, self.cap, self.n_out, self.ws_cull, stream)
            return
        k = self.kept
        L.snake_cull_samples(self.G, self.occ_bits, self.K, R, r["packed_info"], r["t0"], r["t1"], r["pos"],
                             r["ray_id"], r["tile_id"], k["packed_info"], k["t0"], k["t1"], k["pos"], k["ray_id"],
                             k["tile_id"], self.cap, k["n"], self.ws_cull, stream)
        L.snake_sample_refine(rays_o, rays_d, R, self.boxes, r["packed_info"], k["packed_info"], k["t0"], k["t1"],
                              k["tile_id"], self.packed_info, self.t0, self.t1, self.pos, self.ray_id, self.tile_id,
                              self.cap, self.n_out, self.ws_sample, stream)

    def update_occupancy(self, stream=None):
        """Evaluate the density at every cell centre with the current table and
        networks, fold sigma * step into the grid's decaying maximum and
        recompute the occupancy bits."""
        nc = self.K * self.G ** 3
        if not hasattr(self, "occ_feat"):
            fdt = torch.bfloat16 if self.feat_dtype == L.SNAKE_BF16 else torch.float32
            self.occ_feat = torch.empty((len(self.res), nc, self.F), dtype=fdt, device=self.device)
            self.occ_sigma = torch.empty(nc, device=self.device)
            self.occ_rgb = torch.empty((nc, 3), device=self.device)
            self.occ_view = torch.tensor([[0.0, 0.0, -1.0]], device=self.device)
            self.occ_sun = torch.tensor([[0.0, 0.0, 1.0]], device=self.device)
            self.occ_ray = torch.zeros(nc, dtype=torch.int32, device=self.device)
        L.snake_hashgrid_fwd(self.grid, self.K, self.table, self.occ_pos, self.occ_tile, None, nc, None,
                             self.occ_feat, None, stream)
        L.snake_mlp_fwd(self.mlp, self.params, self.occ_feat, self.occ_view, self.occ_sun, self.occ_ray, 1, None,
                        nc, None, self.occ_sigma, self.occ_rgb, stream=stream)
        L.snake_occupancy_update(self.occ_sigma, nc, self.occ_decay, self.occ_step, self.occ_threshold,
                                 self.occ_flags, self.occ_density, self.occ_bits, self.ws_occ, stream)

    def occupied_fraction(self):
        """Fraction of the grid's cells marked occupied (reads the bits back)."""
        nc = self.K * self.G ** 3
        w = self.occ_bits.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        bits = (w.unsqueeze(1) >> torch.arange(32, device=w.device)) & 1
        return float(bits.reshape(-1)[:nc].sum().item()) / nc

    def field_fwd(self, sun=None, stream=None):
        if self.table_bf16:
            L.snake_convert_bf16(self.table, self.table.numel(), self.table_h, stream)
            L.snake_hashgrid_fwd(self.grid_fwd, self.K, self.table_h, self.pos, self.tile_id, None, self.cap,
                                 self.n_out, self.feat, None, stream)
        else:
            L.snake_hashgrid_fwd(self.grid, self.K, self.table, self.pos, self.tile_id, None, self.cap,
                                 self.n_out, self.feat, None, stream)
        L.snake_mlp_fwd(self.mlp, self.params, self.feat, self.view, sun, self.ray_id, self.R_cur, None,
                        self.cap, self.n_out, self.sigma, self.rgb, act=self.act, stream=stream)

    def render(self, R, target=None, loss_scale=0.0, stream=None):
        L.snake_composite_fwd(self.sigma, self.rgb, self.t0, self.t1, self.packed_info, R,
                              self.early_stop, target, loss_scale, self.rgb_out, self.opacity,
                              self.depth, self.n_alive, self.loss if target is not None else None,
                              stream=stream)

    def field_bwd(self, R, target, loss_scale, sun=None, stream=None):
        """Adjoint chain; gradients accumulate into g_t / g_w."""
        L.snake_composite_bwd(self.sigma, self.rgb, self.t0, self.t1, self.packed_info, R,
                              self.n_alive, target, loss_scale, self.dsigma, self.drgb, stream=stream)
        if self.early_stop > 0.0:
            L.snake_pack_alive(self.packed_info, self.n_alive, R, self.alive_idx, self.cap,
                               self.n_alive_total, self.ws_sample, stream)
            idx, n_dev = self.alive_idx, self.n_alive_total
        else:
            idx, n_dev = None, self.n_out
        L.snake_mlp_bwd(self.mlp, self.params, self.feat, self.cap, self.view, sun, self.ray_id, R, idx,
                        self.cap, n_dev, self.dsigma, self.drgb, self.g_w, self.dfeat, self.ws_mlp,
                        act=self.act, stream=stream)
        L.snake_hashgrid_bwd(self.grid, self.K, self.pos, self.tile_id, idx, self.cap, n_dev, self.dfeat,
                             self.g_t, self.ws_hash, stream)
        return n_dev

    def adam(self, stream=None):
        """Adam on the table and the MLP; the step counter lives on the device
        so that a captured step replays with the right bias corrections."""
        self.step_count += 1
        L.snake_counter_add(self.step_dev, 1, stream=stream)
        L.snake_adam_step(self.table, self.g_t, self.m_t, self.v_t, self.table.numel(), self.lr,
                          self.b1, self.b2, self.eps, 0, 0.0, L.SNAKE_ADAM_ZERO_GRAD,
                          step_dev=self.step_dev, stream=stream)
        L.snake_adam_step(self.params, self.g_w, self.m_w, self.v_w, self.P, self.lr, self.b1,
                          self.b2, self.eps, 0, 0.0, L.SNAKE_ADAM_ZERO_GRAD, step_dev=self.step_dev,
                          stream=stream)

    def train_step(self, rays_o, rays_d, target, sun=None, stream=None):
        """One full step on R rays (device tensors).  Returns the device count of
        samples that entered the adjoint (after early stop)."""
        R = int(rays_o.shape[0])
        self.alloc(R)
        self.loss.zero_()
        scale = 1.0 / (3.0 * R)
        self.sample(rays_o, rays_d, R, stream=stream)
        self.field_fwd(sun, stream)
        self.render(R, target, scale, stream)
        n_dev = self.field_bwd(R, target, scale, sun, stream)
        self.adam(stream)
        return n_dev


class SnakeTileStep(torch.autograd.Function):
    """loss = colour-consistency loss of the rendered rays, differentiable with
    respect to the hash table and the MLP weights through the hand-written
    adjoint kernels (composite -> MLP with recomputation -> hash scatter)."""

    @staticmethod
    def forward(ctx, table, params, nerf: TileNeRF, rays_o, rays_d, target, sun):
        R = int(rays_o.shape[0])
        nerf.alloc(R)
        assert table.data_ptr() == nerf.table.data_ptr() and params.data_ptr() == nerf.params.data_ptr()
        nerf.loss.zero_()
        scale = 1.0 / (3.0 * R)
        nerf.sample(rays_o, rays_d, R)
        nerf.field_fwd(sun)
        nerf.render(R, target, scale)
        ctx.nerf, ctx.R, ctx.scale, ctx.target, ctx.sun = nerf, R, scale, target, sun
        return nerf.loss.clone().reshape(())

    @staticmethod
    def backward(ctx, grad_loss):
        nerf = ctx.nerf
        g = float(grad_loss)
        nerf.g_t.zero_()
        nerf.g_w.zero_()
        nerf.field_bwd(ctx.R, ctx.target, ctx.scale * g, ctx.sun)
        return nerf.g_t.clone(), nerf.g_w.clone(), None, None, None, None, None
