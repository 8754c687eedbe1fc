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


def frustum_requests(n_requests: int, grid, rate_hz: float, brick: int = 32, seed: int = 0, fov_deg: float = 60.0,
                     screen_h: int = 1080, max_lod: int = 4, orbit=(0.75, 8.0), n_max: int = 4096):
    """A Poisson stream of brick-set requests from random orbiting camera frusta.

    Request i arrives at the i-th event of a Poisson process of rate rate_hz.
    Its camera sits at distance U[orbit] x (volume extent) from the volume
    centre in a uniformly random direction and looks at the centre; the
    visible bricks are those whose centre lies within half the field of view
    of the view direction.  A brick at distance d gets LOD
    clamp(floor(log2(2 d tan(fov/2) / screen_h)), 0, max_lod), i.e. about one
    voxel per pixel.  The request is n ~ log-uniform[1, n_max] bricks drawn
    without replacement from the visible ones.

    Grids of more than 2^16 bricks test visibility on random candidates
    (doubling their number until n visible ones are found, or every brick has
    been tested), which draws from the same distribution without evaluating
    every brick for every request.  The arrival times scale with 1 / rate_hz
    and the requests themselves do not depend on it.

    Returns (ids u32, lods u8, starts u64[n+1], arrivals f64[n] in seconds).
    """
    rng = np.random.default_rng(seed + 7001)
    nbx, nby, nbz = grid
    nb = nbx * nby * nbz
    extent = float(brick * max(grid))
    vol_c = np.array([nbx, nby, nbz], np.float64) * brick * 0.5
    half = np.deg2rad(fov_deg) / 2
    cos_half = np.cos(half)
    arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))

    def geometry(b, v, cam):
        """distance and visibility of bricks b (flat ids, x fastest) from camera cam looking along -v"""
        b = np.asarray(b, dtype=np.int64)
        c = np.stack([b % nbx, (b // nbx) % nby, b // (nbx * nby)], 1).astype(np.float32)
        c = (c + np.float32(0.5)) * np.float32(brick)
        cc = (c.astype(np.float64) ** 2).sum(1)
        # centre . (-v) and centre . cam in one product
        dots = c @ np.stack([-v, cam], 1).astype(np.float32)
        dist = np.sqrt(np.maximum(cc - 2.0 * dots[:, 1] + cam @ cam, 0.0))
        along = dots[:, 0] + cam @ v  # (centre - cam) . (-v)
        return dist, along >= cos_half * dist

    every = np.arange(nb, dtype=np.int64) if nb <= (1 << 16) else None
    ids, lods, starts = [], [], [0]
    for _ in range(n_requests):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        cam = vol_c + v * (extent * rng.uniform(*orbit))
        n = int(round(np.exp(rng.uniform(0.0, np.log(n_max)))))
        pick = None
        if every is None:
            m = max(4 * n, 4096)
            while m < nb:
                cand = np.unique(rng.integers(0, nb, size=m))
                rng.shuffle(cand)
                dist, vis = geometry(cand, v, cam)
                if vis.sum() >= n:
                    sel = np.nonzero(vis)[0][:n]
                    pick, pdist = cand[sel], dist[sel]
                    break
                m *= 2
        if pick is None:
            allb = every if every is not None else np.arange(nb, dtype=np.int64)
            dist, vis = geometry(allb, v, cam)
            vis = np.nonzero(vis)[0]
            if len(vis) == 0:
                vis = np.array([int(np.argmin(dist))])
            n = max(1, min(n, len(vis)))
            sel = rng.choice(vis, size=n, replace=False)
            pick, pdist = allb[sel], dist[sel]
        lod = np.floor(np.log2(np.maximum(2 * pdist * np.tan(half) / screen_h, 1e-9)))
        ids.append(pick.astype(np.uint32))
        lods.append(np.clip(lod, 0, max_lod).astype(np.uint8))
        starts.append(starts[-1] + len(pick))
    return (np.concatenate(ids).astype(np.uint32), np.concatenate(lods).astype(np.uint8),
            np.array(starts, dtype=np.uint64), arrivals)
