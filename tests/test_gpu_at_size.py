"""GPU parity at the evaluation workloads' full sizes.

Every task of each workload is decoded on the GPU through the C ABI (batched
plan, and for the uneven batch the plain form too) and compared element by
element with the CPU oracle decoding the same container, which the oracle's
own encoder wrote from the seeded raw input.  Workload sizes:
  voronoi512   4096 tasks of 32^3, LOD 0
  neurite1024  32,768 tasks of 32^3, per-brick LOD uniform in {0..3}
  uneven1024   18,600 tasks (32^3 and 64^3 bricks interleaved), u64, LOD 0
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from synth import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = max(1, min(16, os.cpu_count() or 1))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_36898_amd
    return paper_2609_36898_amd


def _gpu_equal(got, want_np, offs, ids, lods, what):
    """Compare a device label tensor with the oracle's host array, chunk by chunk on the GPU."""
    import torch
    lb = want_np.dtype.itemsize
    tdt = torch.int64 if lb == 8 else torch.int32
    want_t = torch.from_numpy(want_np.view(np.int64 if lb == 8 else np.int32))
    n = want_np.size
    step = 1 << 27
    for a in range(0, n, step):
        b = min(n, a + step)
        w = want_t[a:b].to(got.device)
        g = got[a:b].view(tdt)
        if not torch.equal(g, w):
            bad = torch.nonzero(g != w)[0].item() + a
            task = int(np.searchsorted(offs.astype(np.int64), bad, side="right") - 1)
            raise AssertionError("%s: first mismatch at element %d (task %d, brick %d, lod %d)" %
                                 (what, bad, task, ids[task], lods[task]))


def _run_plan(P, container, ids, lods, lb, want, wst, what, plain=False):
    import torch
    dv = P.DeviceVolume(container)
    d_ids, d_lods, d_offs, offs, total = dv.tasks(ids, lods)
    n = len(ids)
    forms = [("batched plan", None)] + ([("plain", P.MODE_PLAIN)] if plain else [])
    for name, mode in forms:
        _say("%s: %s, %d tasks, %d labels" % (what, name, n, total))
        out = torch.empty(total, dtype=dv.dtype, device="cuda")
        status = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        t0 = time.time()
        if mode is None:
            plan = P.csgv_plan(dv.info, n)
            plan.launch(None, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status)
            torch.cuda.synchronize()
            # a second launch through the captured graph must give the same result
            out2 = torch.empty_like(out)
            plan.launch(None, dv.tensor, d_ids, d_lods, d_offs, n, out2, total, status)
            torch.cuda.synchronize()
            assert torch.equal(out, out2), what + ": graph replay differs"
            del out2
            plan.destroy()
        else:
            P.csgv_decode_bricks(None, dv.info, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status, mode=mode)
            torch.cuda.synchronize()
        _say("  decoded in %.2f s (wall, incl. launch)" % (time.time() - t0))
        gst = status.cpu().numpy().view(np.uint32)
        assert np.array_equal(gst, wst), (what, name, np.nonzero(gst != wst)[0][:8])
        _gpu_equal(out, want, offs, ids, lods, what + " " + name)
        del out, status
    del dv
    torch.cuda.empty_cache()


def test_voronoi512_every_brick(P):
    vol = workloads.voronoi512()
    c = oracle.encode_volume(vol, 5, nthreads=THREADS)
    n = 4096
    ids = np.arange(n, dtype=np.uint32)
    lods = np.zeros(n, dtype=np.uint8)
    offs, total = oracle.dense_offsets([5] * n, lods)
    want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 4, nthreads=THREADS)
    assert (wst == 0).all()
    # LOD 0 is the raw volume, brick by brick
    assert np.array_equal(want, oracle._bricks_of_volume(vol, 5))
    del vol
    _run_plan(P, c, ids, lods, 4, want, wst, "voronoi512")


def test_neurite1024_mixed_lods(P):
    vol = workloads.neurite1024()
    c = oracle.encode_volume(vol, 5, nthreads=THREADS)
    del vol
    n = 32768
    ids = np.random.default_rng(11).permutation(n).astype(np.uint32)
    lods = workloads.neurite1024_lods(n)[ids]
    offs, total = oracle.dense_offsets([5] * n, lods)
    want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 4, nthreads=THREADS)
    assert (wst == 0).all()
    _run_plan(P, c, ids, lods, 4, want, wst, "neurite1024")


def test_uneven1024_batched_and_plain(P):
    flat, l2, origins, kinds = workloads.uneven1024()
    c = oracle.encode_bricks(flat, l2, 8, dims=(1024, 1024, 1024), origins=origins, nthreads=THREADS)
    n = len(l2)
    ids = np.arange(n, dtype=np.uint32)
    lods = np.zeros(n, dtype=np.uint8)
    offs, total = oracle.dense_offsets(l2, lods)
    want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 8, nthreads=THREADS)
    assert (wst == 0).all()
    assert np.array_equal(want, flat)  # LOD 0 of every brick is the brick itself
    del flat
    _run_plan(P, c, ids, lods, 8, want, wst, "uneven1024", plain=True)
