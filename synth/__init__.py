"""Seeded synthetic label volumes (inputs only; none of the codec's arithmetic).

The paper evaluates on connectomics, cell and material segmentation volumes
(Results, dataset table) that are not available here; these generators stand
in for them.  Every generator is deterministic in its seed, so the CPU oracle
and the GPU decoder always consume identical bytes.  Volumes are numpy arrays
indexed [z, y, x] (x fastest in memory).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_synth.so")
_lib = None

NEURITE_STEP = 20.5  # random-walk step (isotropic voxels); gives ~30 % background at 1024^3
NEURITE_ZSTRETCH = 4.0


def build(verbose: bool = False) -> str:
    """Compile the generator library in-tree (plain C, OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-D_DEFAULT_SOURCE",
           src, "-o", LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.synth_voronoi_u32.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int]
    lib.synth_voids_u32.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64]
    lib.synth_voids_u32.restype = ctypes.c_long
    lib.synth_neurite_u32.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int]
    lib.synth_uneven_brick_u64.argtypes = [P, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_uneven_tile_split.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_test_brick_u64.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_uneven_batch_u64.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_int]
    lib.synth_pcg32_first.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_pcg32_first.restype = ctypes.c_uint32
    _lib = lib
    return lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def pcg32_first(seed: int, stream: int) -> int:
    return int(_load().synth_pcg32_first(seed, stream))


def voronoi_u32(n: int, n_seeds: int, seed: int = 0, dims=None) -> np.ndarray:
    nx, ny, nz = dims if dims is not None else (n, n, n)
    v = np.empty((nz, ny, nx), dtype=np.uint32)
    rc = _load().synth_voronoi_u32(v.ctypes.data, nx, ny, nz, n_seeds, seed, _threads())
    if rc != 0:
        raise ValueError("bad Voronoi parameters")
    return v


def add_voids(vol: np.ndarray, frac: float, rmin: float, rmax: float, seed: int) -> int:
    assert vol.dtype == np.uint32 and vol.flags.c_contiguous
    nz, ny, nx = vol.shape
    return int(_load().synth_voids_u32(vol.ctypes.data, nx, ny, nz, frac, rmin, rmax, seed))


def neurite_u32(n: int, n_tubes: int, seed: int = 0, z0: int = 0, z1: int | None = None,
                step_len: float = NEURITE_STEP, zstretch: float = NEURITE_ZSTRETCH) -> np.ndarray:
    """Planes [z0, z1) of an n^3 neurite volume (see synth.c for the recipe)."""
    z1 = n if z1 is None else z1
    v = np.empty((z1 - z0, n, n), dtype=np.uint32)
    rc = _load().synth_neurite_u32(v.ctypes.data, n, n, n, z0, z1, n_tubes, step_len, zstretch, seed, _threads())
    if rc != 0:
        raise ValueError("bad neurite slab")
    return v


def uneven_brick_u64(b: int, seed: int, brick_id: int) -> tuple[np.ndarray, int]:
    out = np.empty((b, b, b), dtype=np.uint64)
    kind = _load().synth_uneven_brick_u64(out.ctypes.data, b, seed, brick_id)
    return out, int(kind)


def uneven_batch_u64(log2b, seed: int = 0):
    """Bricks 0..n-1 of the uneven batch concatenated (brick k = uneven_brick_u64(2^log2b[k], seed, k)).

    Returns (flat u64 labels, element offset of each brick, kinds)."""
    l2 = np.ascontiguousarray(np.asarray(log2b, dtype=np.uint8))
    sizes = np.left_shift(np.uint64(1), 3 * l2.astype(np.uint64))
    offs = np.zeros(len(l2), dtype=np.uint64)
    if len(l2) > 1:
        offs[1:] = np.cumsum(sizes)[:-1]
    flat = np.empty(int(sizes.sum()), dtype=np.uint64)
    kinds = np.zeros(len(l2), dtype=np.int32)
    _load().synth_uneven_batch_u64(flat.ctypes.data, offs.ctypes.data, l2.ctypes.data, len(l2), seed,
                                   kinds.ctypes.data, _threads())
    return flat, offs, kinds


def uneven_tile_split(seed: int, tile: int) -> bool:
    return bool(_load().synth_uneven_tile_split(seed, tile))


def test_brick_u64(b: int, kind: int, nlab: int, base: int = 1, seed: int = 0) -> np.ndarray:
    out = np.empty((b, b, b), dtype=np.uint64)
    _load().synth_test_brick_u64(out.ctypes.data, b, kind, nlab, base, seed)
    return out


# ------------------------------------------------------------------ workloads
# The five workloads of the evaluation (sizes as named in each docstring).

def voronoi_small(seed: int = 0) -> np.ndarray:
    """128^3 u32 Voronoi, 500 seeds, labels 1..500 (64 bricks of 32^3)."""
    return voronoi_u32(128, 500, seed)


def voronoi_voids(n: int = 512, n_seeds: int = 20000, seed: int = 0, frac: float = 0.10) -> np.ndarray:
    """512^3 u32 Voronoi with 20,000 seeds plus >= 10 % label-0 spherical voids (radius U[8,32))."""
    v = voronoi_u32(n, n_seeds, seed)
    add_voids(v, frac, 8.0, 32.0, seed)
    return v


def neurite_volume(n: int = 1024, n_tubes: int = 100000, seed: int = 0) -> np.ndarray:
    """1024^3 u32 neurite volume: 100,000 spline tubes, radius U[3,20), z stretched 4x."""
    return neurite_u32(n, n_tubes, seed)


def uneven_layout(n_tiles_side: int = 16, seed: int = 0):
    """Brick directory of the uneven u64 batch: list of (origin_xyz, log2b) in brick-id order.

    Tiles of 64^3 in x-fastest order; a split tile contributes its eight 32^3
    octants in Morton order (x, then y, then z bit).
    """
    bricks = []
    T = n_tiles_side
    for tz in range(T):
        for ty in range(T):
            for tx in range(T):
                t = (tz * T + ty) * T + tx
                o = (64 * tx, 64 * ty, 64 * tz)
                if uneven_tile_split(seed, t):
                    for j in range(8):
                        bricks.append(((o[0] + 32 * (j & 1), o[1] + 32 * ((j >> 1) & 1), o[2] + 32 * (j >> 2)), 5))
                else:
                    bricks.append((o, 6))
    return bricks
