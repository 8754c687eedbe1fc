"""MI355X-native CSGV brick decoder.

The decode stage of a segmentation-volume renderer: bricks of a compressed
volume resident in HBM are decompressed, in parallel and at per-brick level of
detail, into brick-cache slots.  `csgv` is the ctypes binding of the C ABI
(include/csgv.h); this module adds host-side conveniences that only move data
(brick reordering, offsets, device buffers).
"""
from __future__ import annotations

import numpy as np

from . import csgv
from .csgv import (ALL_OPS, MODE_PERSISTENT, MODE_PLAIN, TASK_CORRUPT, TASK_INVALID, TASK_OK, CsgvError,  # noqa: F401
                   csgv_check_status, csgv_decode_bricks, csgv_encode_bricks, csgv_plan, csgv_volume_parse)


def bricks_of_volume(vol: np.ndarray, log2b: int) -> np.ndarray:
    """[z,y,x] volume -> concatenated b^3 bricks (brick id = bx + nbx*(by + nby*bz)), each x fastest."""
    b = 1 << log2b
    nz, ny, nx = vol.shape
    if nx % b or ny % b or nz % b:
        raise ValueError("volume dimensions must be multiples of the brick side")
    v = vol.reshape(nz // b, b, ny // b, b, nx // b, b)
    return np.ascontiguousarray(v.transpose(0, 2, 4, 1, 3, 5)).reshape(-1)


def encode_volume(vol: np.ndarray, log2b: int = 5, **kw) -> bytes:
    """Compress a [z,y,x] u32/u64 label volume with a regular brick grid (CPU encoder of libcsgv)."""
    b = 1 << log2b
    nz, ny, nx = vol.shape
    grid = (nx // b, ny // b, nz // b)
    n = grid[0] * grid[1] * grid[2]
    return csgv_encode_bricks(bricks_of_volume(vol, log2b), [log2b] * n, vol.dtype.itemsize, dims=(nx, ny, nz),
                              default_log2b=log2b, grid=grid, **kw)


def dense_offsets(log2bs, lods):
    """Element offsets packing the task outputs back to back, and their total."""
    l2 = np.asarray(log2bs, dtype=np.int64)
    ld = np.asarray(lods, dtype=np.int64)
    sizes = (np.int64(1) << (3 * (l2 - ld))).astype(np.uint64)
    offs = np.zeros(len(sizes), dtype=np.uint64)
    if len(sizes) > 1:
        offs[1:] = np.cumsum(sizes)[:-1]
    return offs, int(sizes.sum())


def brick_log2b(container: bytes, info=None) -> np.ndarray:
    """Per-brick log2(side): from the directory when present, else the header default."""
    info = info or csgv_volume_parse(container)
    if info.dir_pos:
        d = np.frombuffer(container, dtype=np.uint32, count=4 * info.n_bricks, offset=info.dir_pos)
        return d.reshape(-1, 4)[:, 3].astype(np.int64)
    return np.full(info.n_bricks, info.log2b, dtype=np.int64)


class DeviceVolume:
    """A container resident in device memory plus its parsed header."""

    def __init__(self, container: bytes, device="cuda"):
        import torch
        self.host = container
        self.info = csgv_volume_parse(container)
        self.label_bytes = int(self.info.label_bytes)
        self.dtype = torch.int64 if self.label_bytes == 8 else torch.int32
        self.tensor = torch.frombuffer(bytearray(container), dtype=torch.uint8).to(device)
        self.log2b = brick_log2b(container, self.info)

    def tasks(self, ids, lods, device="cuda"):
        """Device task arrays and dense output offsets for (ids, lods)."""
        import torch
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        lods = np.ascontiguousarray(np.asarray(lods, dtype=np.uint8))
        offs, total = dense_offsets(self.log2b[ids.astype(np.int64)], lods)
        d_ids = torch.from_numpy(ids.view(np.int32)).to(device)
        d_lods = torch.from_numpy(lods).to(device)
        d_offs = torch.from_numpy(offs.view(np.int64)).to(device)
        return d_ids, d_lods, d_offs, offs, total

    def decode(self, ids, lods, mode=MODE_PLAIN, out=None, stream=None, **kw):
        """Decode tasks into a fresh (or given) label tensor; returns (out, status, host offsets)."""
        import torch
        d_ids, d_lods, d_offs, offs, total = self.tasks(ids, lods, self.tensor.device)
        n = len(offs)
        if out is None:
            out = torch.empty(max(total, 1), dtype=self.dtype, device=self.tensor.device)
        status = torch.full((max(n, 1),), -1, dtype=torch.int32, device=self.tensor.device)
        csgv_decode_bricks(stream, self.info, self.tensor, d_ids, d_lods, d_offs, n, out, out.numel(), status,
                           mode=mode, **kw)
        return out, status[:n], offs
