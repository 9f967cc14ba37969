"""ctypes binding of libsnake (include/snake.h): argument marshalling only.

Every function here has the name of the C entry point it calls, takes torch
tensors for device arrays (``None`` for NULL), host scalars / NumPy arrays for
host arguments, and raises ``SnakeError`` on a non-zero status.  All compute
runs in the HIP library; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnake.so")

SNAKE_F32, SNAKE_BF16 = 0, 1
SNAKE_GRID_ALWAYS_HASH = 1
SNAKE_GRID_TABLE_BF16 = 2
SNAKE_ADAM_ZERO_GRAD = 1
SNAKE_OCC_MEAN_CAP = 1
SNAKE_DEVERR_CAPACITY = 1
SNAKE_DEVERR_TILE_ID = 2
SNAKE_DEVERR_RAY_ID = 4
SNAKE_DEVERR_INTERNAL = 8
SNAKE_DEVERR_NONFINITE = 16
MAX_LEVELS = 32
TUNABLES = {
    "hash_fwd_blocks_per_cu": 0, "mlp_fwd_blocks_per_cu": 1, "mlp_bwd_blocks_per_cu": 2,
    "composite_blocks_per_cu": 3, "bin_blocks": 4, "bin_levels_per_pass": 5, "sampler_blocks_per_cu": 6,
    "hash_fwd_superchunk": 7, "hash_fwd_lds": 8,
}

EXPORTS = (
    "snake_abi_version", "snake_last_error", "snake_check_device_error", "snake_tune_set", "snake_tune_get",
    "snake_stream_create_dedicated", "snake_stream_destroy",
    "snake_sample_workspace_bytes", "snake_sample_segmented", "snake_sample_segmented_static_max_rays",
    "snake_sample_grouped_workspace_bytes", "snake_sample_grouped",
    "snake_sample_segmented_static", "snake_pack_alive",
    "snake_window_accept", "snake_tile_partition_workspace_bytes", "snake_tile_partition",
    "snake_occupancy_cells", "snake_occupancy_workspace_bytes", "snake_occupancy_update",
    "snake_cull_workspace_bytes", "snake_cull_samples", "snake_sample_refine",
    "snake_convert_bf16", "snake_hashgrid_fwd", "snake_hashgrid_bwd", "snake_hashgrid_bwd_workspace_bytes",
    "snake_mlp_param_count", "snake_mlp_weight_count", "snake_mlp_act_width", "snake_mlp_bwd_workspace_bytes", "snake_mlp_fwd",
    "snake_mlp_bwd",
    "snake_composite_fwd", "snake_composite_bwd", "snake_adam_step", "snake_adam_step_tiles", "snake_counter_add",
)


class SnakeError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__("%s failed (%d): %s" % (fn, code, msg))
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("log2_table", ctypes.c_int32), ("feat_dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("resolution", ctypes.c_int32 * MAX_LEVELS)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("n_dir", ctypes.c_int32), ("colour_layers", ctypes.c_int32),
                ("colour_out", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("feat_dtype", ctypes.c_int32), ("shared_colour", ctypes.c_int32)]


def grid_desc(resolution, n_features, log2_table, feat_dtype=SNAKE_F32, flags=0) -> GridDesc:
    res = [int(r) for r in resolution]
    d = GridDesc()
    d.n_levels = len(res)
    d.n_features = int(n_features)
    d.log2_table = int(log2_table)
    d.feat_dtype = int(feat_dtype)
    d.flags = int(flags)
    for i, r in enumerate(res):
        d.resolution[i] = r
    return d


def mlp_desc(n_levels, n_features, n_dir, colour_layers, colour_out, precision=SNAKE_F32,
             feat_dtype=SNAKE_F32, shared_colour=0) -> MlpDesc:
    return MlpDesc(int(n_levels), int(n_features), int(n_dir), int(colour_layers),
                   int(colour_out), int(precision), int(feat_dtype), int(shared_colour))


_P, _I32, _I64, _U32, _F, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_float, ctypes.c_size_t)
_SIGS = {
    "snake_tune_set": ([_I32, _I32], ctypes.c_int),
    "snake_tune_get": ([_I32], _I32),
    "snake_abi_version": ([], ctypes.c_int),
    "snake_last_error": ([], ctypes.c_char_p),
    "snake_check_device_error": ([_P, _P], ctypes.c_int),
    "snake_stream_create_dedicated": ([_P], ctypes.c_int),
    "snake_stream_destroy": ([_P], ctypes.c_int),
    "snake_sample_workspace_bytes": ([_I32], _SZ),
    "snake_sample_segmented": ([_P, _P, _I32, _P, _I32, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P,
                                _I64, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_sample_segmented_static_max_rays": ([], _I32),
    "snake_sample_grouped_workspace_bytes": ([_I32, _I32], _SZ),
    "snake_sample_grouped": ([_P, _P, _I32, _P, _I32, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                              _I64, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_sample_segmented_static": ([_P, _P, _I32, _P, _I32, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P,
                                       _I64, _P, _P], ctypes.c_int),
    "snake_pack_alive": ([_P, _P, _I32, _P, _I64, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_window_accept": ([_P, _P, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_tile_partition_workspace_bytes": ([_I32], _SZ),
    "snake_occupancy_cells": ([_I32, _I32, _P, _P, _P], ctypes.c_int),
    "snake_occupancy_workspace_bytes": ([_I64], _SZ),
    "snake_occupancy_update": ([_P, _I64, _F, _F, _F, ctypes.c_uint32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_cull_workspace_bytes": ([_I32], _SZ),
    "snake_cull_samples": ([_I32, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P, _P,
                            _SZ, _P], ctypes.c_int),
    "snake_sample_refine": ([_P, _P, _I32, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _SZ,
                             _P], ctypes.c_int),
    "snake_tile_partition": ([_P, _P, _P, _I64, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_convert_bf16": ([_P, _I64, _P, _P], ctypes.c_int),
    "snake_hashgrid_fwd": ([_P, _I32, _P, _P, _P, _P, _I64, _P, _P, _P, _P], ctypes.c_int),
    "snake_hashgrid_bwd": ([_P, _I32, _P, _P, _P, _I64, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "snake_hashgrid_bwd_workspace_bytes": ([_P, _I32, _I64, _I32], _SZ),
    "snake_mlp_param_count": ([_P], _I64),
    "snake_mlp_weight_count": ([_P, _I32], _I64),
    "snake_mlp_bwd_workspace_bytes": ([_P, _I32], _SZ),
    "snake_mlp_act_width": ([_P], _I32),
    "snake_mlp_fwd": ([_P, _I32, _P, _P, _P, _P, _P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P], ctypes.c_int),
    "snake_mlp_bwd": ([_P, _I32, _P, _P, _P, _I64, _P, _P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P, _P, _P,
                       _SZ, _P],
                      ctypes.c_int),
    "snake_composite_fwd": ([_P, _P, _P, _P, _P, _I32, _P, _F, _P, _F, _P, _P, _P, _P, _P, _P],
                            ctypes.c_int),
    "snake_composite_bwd": ([_P, _P, _P, _P, _P, _I32, _P, _P, _P, _F, _P, _P, _P], ctypes.c_int),
    "snake_adam_step": ([_P, _P, _P, _P, _I64, _F, _F, _F, _F, _I32, _P, _F, _U32, _P], ctypes.c_int),
    "snake_adam_step_tiles": ([_P, _P, _P, _P, _I64, _I32, _F, _F, _F, _F, _P, _F, _U32, _P], ctypes.c_int),
    "snake_counter_add": ([_P, _I32, _I32, _P], ctypes.c_int),
}

_lib = None


def lib():
    """Load libsnake.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsnake.so is not built: run `python -m paper_2507_01631_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _check(fn, rc):
    if rc != 0:
        raise SnakeError(fn, rc, lib().snake_last_error().decode())


def _host_f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
def snake_abi_version() -> int:
    return lib().snake_abi_version()


def snake_last_error() -> str:
    return lib().snake_last_error().decode()


def snake_tune_set(which, value):
    which = TUNABLES[which] if isinstance(which, str) else int(which)
    _check("snake_tune_set", lib().snake_tune_set(which, int(value)))


def snake_tune_get(which) -> int:
    which = TUNABLES[which] if isinstance(which, str) else int(which)
    return int(lib().snake_tune_get(which))


def snake_check_device_error(stream=None) -> int:
    bits = ctypes.c_uint32(0)
    rc = lib().snake_check_device_error(_stream(stream), ctypes.byref(bits))
    if rc not in (0, -7):
        _check("snake_check_device_error", rc)
    return int(bits.value)


def snake_sample_workspace_bytes(R: int) -> int:
    return int(lib().snake_sample_workspace_bytes(int(R)))


def snake_sample_segmented(rays_o, rays_d, R, boxes, zband, samples_per_ray, S, max_count,
                           packed_info, t0, t1, pos, ray_id, tile_id, view, cap, n_out,
                           workspace, stream=None):
    boxes = _host_f64(boxes).reshape(-1, 6)
    zb = _host_f64(zband)
    rc = lib().snake_sample_segmented(
        _ptr(rays_o), _ptr(rays_d), int(R), boxes.ctypes.data, int(boxes.shape[0]),
        None if zb is None else zb.ctypes.data, _ptr(samples_per_ray), int(S), _ptr(max_count),
        _ptr(packed_info), _ptr(t0), _ptr(t1), _ptr(pos), _ptr(ray_id), _ptr(tile_id), _ptr(view),
        int(cap), _ptr(n_out), _ptr(workspace), workspace.numel() * workspace.element_size(),
        _stream(stream))
    _check("snake_sample_segmented", rc)


def snake_sample_grouped_workspace_bytes(R, K):
    return int(lib().snake_sample_grouped_workspace_bytes(int(R), int(K)))


def snake_sample_grouped(rays_o, rays_d, R, boxes, zband, samples_per_ray, S, max_count, packed_info, t0, t1,
                         view, pos, ray_id, tile_id, sample_map, tile_start, cap, n_out, workspace, stream=None):
    boxes = _host_f64(boxes).reshape(-1, 6)
    zb = _host_f64(zband)
    rc = lib().snake_sample_grouped(
        _ptr(rays_o), _ptr(rays_d), int(R), boxes.ctypes.data, int(boxes.shape[0]),
        None if zb is None else zb.ctypes.data, _ptr(samples_per_ray), int(S), _ptr(max_count),
        _ptr(packed_info), _ptr(t0), _ptr(t1), _ptr(view), _ptr(pos), _ptr(ray_id), _ptr(tile_id),
        _ptr(sample_map), _ptr(tile_start), int(cap), _ptr(n_out), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream))
    _check("snake_sample_grouped", rc)


def snake_sample_segmented_static_max_rays():
    return int(lib().snake_sample_segmented_static_max_rays())


def snake_sample_segmented_static(rays_o, rays_d, R, boxes, zband, samples_per_ray, S, max_count,
                                  packed_info, t0, t1, pos, ray_id, tile_id, view, cap, n_out, stream=None):
    boxes = _host_f64(boxes).reshape(-1, 6)
    zb = _host_f64(zband)
    rc = lib().snake_sample_segmented_static(
        _ptr(rays_o), _ptr(rays_d), int(R), boxes.ctypes.data, int(boxes.shape[0]),
        None if zb is None else zb.ctypes.data, _ptr(samples_per_ray), int(S), _ptr(max_count),
        _ptr(packed_info), _ptr(t0), _ptr(t1), _ptr(pos), _ptr(ray_id), _ptr(tile_id), _ptr(view),
        int(cap), _ptr(n_out), _stream(stream))
    _check("snake_sample_segmented_static", rc)


def snake_pack_alive(packed_info, n_alive, R, idx_out, cap, n_out, workspace, stream=None):
    rc = lib().snake_pack_alive(_ptr(packed_info), _ptr(n_alive), int(R), _ptr(idx_out), int(cap),
                                _ptr(n_out), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream))
    _check("snake_pack_alive", rc)


def snake_window_accept(rays_o, rays_d, R, window, zband, accept, idx_out, n_out, workspace, stream=None):
    win = _host_f64(window).reshape(4)
    zb = _host_f64(zband).reshape(2)
    rc = lib().snake_window_accept(_ptr(rays_o), _ptr(rays_d), int(R), win.ctypes.data, zb.ctypes.data,
                                   _ptr(accept), _ptr(idx_out), _ptr(n_out), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream))
    _check("snake_window_accept", rc)


def snake_tile_partition_workspace_bytes(K) -> int:
    return int(lib().snake_tile_partition_workspace_bytes(int(K)))


def snake_tile_partition(tile_id, pos, ray_id, n, n_dev, K, perm, inv, tile_start, pos_out, tile_out,
                         ray_out, workspace, stream=None):
    rc = lib().snake_tile_partition(_ptr(tile_id), _ptr(pos), _ptr(ray_id), int(n), _ptr(n_dev), int(K),
                                    _ptr(perm), _ptr(inv), _ptr(tile_start), _ptr(pos_out), _ptr(tile_out),
                                    _ptr(ray_out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream(stream))
    _check("snake_tile_partition", rc)


def snake_occupancy_cells(G, K, pos, tile_id, stream=None):
    _check("snake_occupancy_cells", lib().snake_occupancy_cells(int(G), int(K), _ptr(pos), _ptr(tile_id),
                                                                _stream(stream)))


def snake_occupancy_workspace_bytes(n_cells) -> int:
    return int(lib().snake_occupancy_workspace_bytes(int(n_cells)))


def snake_occupancy_update(sigma, n_cells, decay, sigma_scale, threshold, flags, density, bits, workspace,
                           stream=None):
    _check("snake_occupancy_update", lib().snake_occupancy_update(
        _ptr(sigma), int(n_cells), float(decay), float(sigma_scale), float(threshold), int(flags), _ptr(density),
        _ptr(bits), _ptr(workspace), workspace.numel() * workspace.element_size() if workspace is not None else 0,
        _stream(stream)))


def snake_cull_workspace_bytes(R) -> int:
    return int(lib().snake_cull_workspace_bytes(int(R)))


def snake_cull_samples(G, bits, K, R, packed_info, t0, t1, pos, ray_id, tile_id, packed_info_out, t0_out, t1_out,
                       pos_out, ray_id_out, tile_id_out, cap, n_out, workspace, stream=None):
    rc = lib().snake_cull_samples(int(G), _ptr(bits), int(K), int(R), _ptr(packed_info), _ptr(t0), _ptr(t1),
                                  _ptr(pos), _ptr(ray_id), _ptr(tile_id), _ptr(packed_info_out), _ptr(t0_out),
                                  _ptr(t1_out), _ptr(pos_out), _ptr(ray_id_out), _ptr(tile_id_out), int(cap),
                                  _ptr(n_out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream(stream))
    _check("snake_cull_samples", rc)


def snake_sample_refine(rays_o, rays_d, R, boxes, packed_info_all, packed_info_kept, t0_kept, t1_kept, tile_id_kept,
                        packed_info, t0, t1, pos, ray_id, tile_id, cap, n_out, workspace, stream=None):
    boxes = _host_f64(boxes).reshape(-1, 6)
    rc = lib().snake_sample_refine(
        _ptr(rays_o), _ptr(rays_d), int(R), boxes.ctypes.data, int(boxes.shape[0]), _ptr(packed_info_all),
        _ptr(packed_info_kept), _ptr(t0_kept), _ptr(t1_kept), _ptr(tile_id_kept), _ptr(packed_info), _ptr(t0),
        _ptr(t1), _ptr(pos), _ptr(ray_id), _ptr(tile_id), int(cap), _ptr(n_out), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream))
    _check("snake_sample_refine", rc)


def snake_convert_bf16(src, n, dst, stream=None):
    _check("snake_convert_bf16", lib().snake_convert_bf16(_ptr(src), int(n), _ptr(dst), _stream(stream)))


def snake_hashgrid_fwd(g: GridDesc, K, table, pos, tile_id, sample_idx, n, n_dev, feat, idx_dbg=None,
                       stream=None):
    rc = lib().snake_hashgrid_fwd(ctypes.byref(g), int(K), _ptr(table), _ptr(pos), _ptr(tile_id),
                                  _ptr(sample_idx), int(n), _ptr(n_dev), _ptr(feat), _ptr(idx_dbg),
                                  _stream(stream))
    _check("snake_hashgrid_fwd", rc)


def snake_hashgrid_bwd_workspace_bytes(g: GridDesc, K, n, levels_per_pass) -> int:
    return int(lib().snake_hashgrid_bwd_workspace_bytes(ctypes.byref(g), int(K), int(n),
                                                        int(levels_per_pass)))


def snake_hashgrid_bwd(g: GridDesc, K, pos, tile_id, sample_idx, n, n_dev, dfeat, dtable,
                       workspace=None, stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    rc = lib().snake_hashgrid_bwd(ctypes.byref(g), int(K), _ptr(pos), _ptr(tile_id), _ptr(sample_idx),
                                  int(n), _ptr(n_dev), _ptr(dfeat), _ptr(dtable), _ptr(workspace),
                                  nbytes, _stream(stream))
    _check("snake_hashgrid_bwd", rc)


def snake_mlp_param_count(m: MlpDesc) -> int:
    return int(lib().snake_mlp_param_count(ctypes.byref(m)))


def snake_mlp_weight_count(m: MlpDesc, K=1) -> int:
    return int(lib().snake_mlp_weight_count(ctypes.byref(m), int(K)))


def snake_mlp_act_width(m: MlpDesc) -> int:
    return int(lib().snake_mlp_act_width(ctypes.byref(m)))


def snake_mlp_bwd_workspace_bytes(m: MlpDesc, K=1) -> int:
    return int(lib().snake_mlp_bwd_workspace_bytes(ctypes.byref(m), int(K)))


def snake_mlp_fwd(m: MlpDesc, weights, feat, view, sun, ray_id, R, sample_idx, n, n_dev, sigma, rgb,
                  act=None, K=1, tile_start=None, stream=None):
    rc = lib().snake_mlp_fwd(ctypes.byref(m), int(K), _ptr(weights), _ptr(tile_start), _ptr(feat), _ptr(view),
                             _ptr(sun),
                             _ptr(ray_id), int(R), _ptr(sample_idx), int(n), _ptr(n_dev), _ptr(sigma),
                             _ptr(rgb), _ptr(act), _stream(stream))
    _check("snake_mlp_fwd", rc)


def snake_mlp_bwd(m: MlpDesc, weights, feat, feat_ld, view, sun, ray_id, R, sample_idx, n, n_dev,
                  dsigma, drgb, dW, dfeat, workspace, act=None, K=1, tile_start=None, stream=None):
    rc = lib().snake_mlp_bwd(ctypes.byref(m), int(K), _ptr(weights), _ptr(tile_start), _ptr(feat), int(feat_ld),
                             _ptr(view),
                             _ptr(sun), _ptr(ray_id), int(R), _ptr(sample_idx), int(n), _ptr(n_dev),
                             _ptr(dsigma), _ptr(drgb), _ptr(act), _ptr(dW), _ptr(dfeat), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream))
    _check("snake_mlp_bwd", rc)


def snake_composite_fwd(sigma, rgb, t0, t1, packed_info, R, early_stop_T, target, loss_scale,
                        rgb_out, opacity, depth, n_alive, loss, sample_map=None, stream=None):
    rc = lib().snake_composite_fwd(_ptr(sigma), _ptr(rgb), _ptr(t0), _ptr(t1), _ptr(packed_info),
                                   int(R), _ptr(sample_map), float(early_stop_T), _ptr(target), float(loss_scale),
                                   _ptr(rgb_out), _ptr(opacity), _ptr(depth), _ptr(n_alive),
                                   _ptr(loss), _stream(stream))
    _check("snake_composite_fwd", rc)


def snake_composite_bwd(sigma, rgb, t0, t1, packed_info, R, n_alive, target, loss_scale, dsigma,
                        drgb, sample_map=None, stream=None):
    rc = lib().snake_composite_bwd(_ptr(sigma), _ptr(rgb), _ptr(t0), _ptr(t1), _ptr(packed_info),
                                   int(R), _ptr(sample_map), _ptr(n_alive), _ptr(target), float(loss_scale),
                                   _ptr(dsigma), _ptr(drgb), _stream(stream))
    _check("snake_composite_bwd", rc)


def snake_adam_step(p, g, m, v, n, lr, b1, b2, eps, step, l2=0.0, flags=0, step_dev=None, stream=None):
    rc = lib().snake_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(n), float(lr), float(b1),
                               float(b2), float(eps), int(step), _ptr(step_dev), float(l2), int(flags),
                               _stream(stream))
    _check("snake_adam_step", rc)


def snake_adam_step_tiles(p, g, m, v, tile_n, K, lr, b1, b2, eps, step_dev, l2=0.0, flags=0, stream=None):
    rc = lib().snake_adam_step_tiles(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(tile_n), int(K), float(lr), float(b1),
                                     float(b2), float(eps), _ptr(step_dev), float(l2), int(flags), _stream(stream))
    _check("snake_adam_step_tiles", rc)


def snake_stream_create_dedicated():
    """Handle (int) of a new stream on a hardware queue of its own."""
    h = ctypes.c_void_p()
    _check("snake_stream_create_dedicated", lib().snake_stream_create_dedicated(ctypes.byref(h)))
    return int(h.value)


def snake_stream_destroy(handle):
    _check("snake_stream_destroy", lib().snake_stream_destroy(ctypes.c_void_p(handle)))


def snake_counter_add(counter, delta, n=None, stream=None):
    n = counter.numel() if n is None else int(n)
    _check("snake_counter_add", lib().snake_counter_add(_ptr(counter), n, int(delta), _stream(stream)))
