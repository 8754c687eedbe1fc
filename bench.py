"""Benchmark: decoded GVoxel/s of the batched (persistent, graph-launched)
CSGV brick decoder on one MI355X, with the plain one-launch-per-brick form,
the decode kernel's HBM roofline fraction and the CPU oracle beside it.

Workload (the metric's reference configuration): a 512^3 u32 Voronoi label
volume with 20,000 seeds and >= 10 % label-0 spherical voids, 32^3 bricks
(4096 bricks), every brick decoded at full resolution in one batched launch.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("decode_kernel.hip", "decode_kernel.h", "csgv_format.h"):
        with open(os.path.join(ROOT, "paper_2609_36898_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profiled_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "decode_kernel_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != _kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def build_workload(seed: int = 0):
    import synth
    import paper_2609_36898_amd as P
    t0 = time.time()
    vol = synth.voronoi_voids(512, 20000, seed=seed, frac=0.10)
    t1 = time.time()
    container = P.encode_volume(vol, 5)
    t2 = time.time()
    _log("workload: generated %.1fs, encoded %.1fs, %d bytes (%.2f%% of raw)" %
         (t1 - t0, t2 - t1, len(container), 100.0 * len(container) / vol.nbytes))
    return vol, container


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--wg", type=int, default=0, help="work-group size (0 = plan default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the decode path has no multi-GPU form in this build "
              "(bricks are independent; sharding is by brick-id range, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_36898_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    vol, container = build_workload()
    dv = P.DeviceVolume(container, device=dev)
    n = dv.info.n_bricks
    ids = np.arange(n, dtype=np.uint32)
    lods = np.zeros(n, dtype=np.uint8)
    d_ids, d_lods, d_offs, offs, total = dv.tasks(ids, lods, dev)
    out = torch.empty(total, dtype=torch.int32, device=dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    voxels = float(total)
    offsets = np.frombuffer(container, dtype=np.uint64, count=n + 1, offset=int(dv.info.offsets_pos))
    record_bytes = float(offsets[-1] - offsets[0])
    alg_bytes = record_bytes + voxels * 4  # read every record once, write every label once

    plan = P.csgv_plan(dv.info, n, wg_size=args.wg)
    opts = plan.get_opts()
    stream = torch.cuda.current_stream(dev)

    def step():
        plan.launch(stream, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    gvox = voxels / (ms * 1e-3) / 1e9

    # bit-exactness of the timed output: LOD 0 of every brick is the raw brick
    ref = torch.from_numpy(P.bricks_of_volume(vol, 5).view(np.int32)).to(dev)
    bit_exact = bool(torch.equal(out, ref)) and bool((status == 0).all().item())
    del ref

    # dominant kernel: average decode-kernel duration from events on the launch stream
    plan.set_timing(True)
    kms = []
    for _ in range(max(3, args.steps // 2)):
        step()
        kms.append(plan.last_kernel_ms())
    plan.set_timing(False)
    kernel_ms = float(np.mean(kms))
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = _profiled_traffic("voronoi512")

    # plain form: one kernel launch per brick
    plain_out = torch.empty_like(out)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    P.csgv_decode_bricks(stream, dv.info, dv.tensor, d_ids, d_lods, d_offs, n, plain_out, total, status,
                         mode=P.MODE_PLAIN)
    torch.cuda.synchronize()
    p0.record(stream)
    for _ in range(args.plain_steps):
        P.csgv_decode_bricks(stream, dv.info, dv.tensor, d_ids, d_lods, d_offs, n, plain_out, total, status,
                             mode=P.MODE_PLAIN)
    p1.record(stream)
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1) / args.plain_steps
    plain_exact = bool(torch.equal(plain_out, out))
    del plain_out

    result = {
        "metric": "decoded GVoxel/s (bit-exact), batched",
        "value": round(gvox, 3) if bit_exact else None,
        "unit": "GVoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "voronoi512_voids_u32_b32_lod0", "volume": [512, 512, 512], "label_bytes": 4,
                   "brick": 32, "bricks": n, "tasks": n, "lod": 0, "seeds": 20000, "void_fraction_min": 0.10,
                   "form": "persistent+graph", "wg_size": int(opts.wg_size), "sort_tasks": int(opts.sort_tasks),
                   "compressed_bytes": len(container)},
        "bit_exact": bit_exact,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "decode_kernel", "kernel_ms": round(kernel_ms, 4),
                     "alg_bytes_per_launch": alg_bytes},
        "plain": {"value": round(voxels / (plain_ms * 1e-3) / 1e9, 3), "unit": "GVoxel/s",
                  "ms_per_step": round(plain_ms, 3), "launches_per_step": n, "bit_exact": plain_exact},
    }

    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        reps = 3
        sel = np.arange(n, dtype=np.uint32)
        times = []
        cpu_out = np.empty(total, dtype=np.uint32)
        for _ in range(reps):
            t0 = time.perf_counter()
            cpu_out, cpu_st = oracle.decode_tasks(container, sel, np.zeros(n, np.uint8), offs, total, 4,
                                                  nthreads=threads, out=cpu_out)
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        gpu_all = out.cpu().numpy().view(np.uint32)
        result["cpu_baseline"] = {
            "value": round(voxels / dt / 1e9, 4), "unit": "GVoxel/s", "cores": threads, "kind": "oracle",
            "sample": "the whole task list (%d bricks, LOD 0), OpenMP over bricks, median of %d runs of %.2f s "
                      "wall (%.1f thread-s each)" % (n, reps, dt, dt * threads),
            "matches_gpu": bool(np.array_equal(cpu_out, gpu_all)) and bool((cpu_st == 0).all()),
        }
    plan.destroy()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
