"""The five evaluation workloads as seeded raw inputs.

Only raw label volumes, brick directories and task lists come from here;
encoding and decoding are the caller's (the product encoder, or the oracle's
in the tests).  Sizes follow the workload definitions:

  voronoi128   128^3 u32 Voronoi, 500 seeds (labels 1..500), seed 0; 32^3
               bricks (64), LOD 0.
  voronoi512   512^3 u32 Voronoi, 20,000 seeds, then label-0 spherical voids
               (radius U[8,32)) until >= 10 % of voxels are 0; 32^3 bricks
               (4096), LOD 0.
  neurite1024  1024^3 u32 neurite volume, 100,000 spline tubes, radius
               U[3,20), z stretched 4x, ~30 % background, random 32-bit labels;
               32^3 bricks (32,768), per-brick LOD uniform in {0..3}.
  neurite2048  2048^3 u32, the same generator with 800,000 tubes, produced in
               z-slabs (served workload).
  uneven1024   1024^3 u64: 4096 tiles of 64^3, each one 64^3 brick or eight
               32^3 bricks (fair coin); per brick 40 % constant, 40 % Voronoi
               with 2..64 random u64 labels, 20 % i.i.d. noise; LOD 0.
"""
from __future__ import annotations

import numpy as np

from . import neurite_u32, neurite_volume, uneven_batch_u64, uneven_layout, voronoi_small, voronoi_voids


def voronoi128() -> np.ndarray:
    return voronoi_small(0)


def voronoi512() -> np.ndarray:
    return voronoi_voids(512, 20000, seed=0, frac=0.10)


def neurite1024() -> np.ndarray:
    return neurite_volume(1024, 100000, seed=0)


def neurite1024_lods(n_bricks: int = 32768, seed: int = 0) -> np.ndarray:
    """Per-brick LOD, uniform in {0, 1, 2, 3}."""
    return np.random.default_rng(seed + 1000).integers(0, 4, size=n_bricks).astype(np.uint8)


NEURITE2048_TUBES = 800000


def neurite2048_slab(z0: int, z1: int, n: int = 2048, n_tubes: int = NEURITE2048_TUBES, seed: int = 0):
    """Planes [z0, z1) of the served 2048^3 volume (generated slab by slab)."""
    return neurite_u32(n, n_tubes, seed=seed, z0=z0, z1=z1)


def uneven1024(seed: int = 0, tiles_side: int = 16):
    """Bricks of the uneven u64 batch: (flat labels, log2b per brick, origins [n,3], kinds)."""
    lay = uneven_layout(tiles_side, seed)
    l2 = np.array([l for _, l in lay], dtype=np.uint8)
    origins = np.array([o for o, _ in lay], dtype=np.uint32)
    flat, _, kinds = uneven_batch_u64(l2, seed)
    return flat, l2, origins, kinds
