"""Benchmark of the CSGV brick decoder on one MI355X.

Prints ONE JSON line.  The headline is the largest workload, the served one:
a 2048^3 u32 neurite volume (800,000 spline tubes, 262,144 bricks of 32^3)
resident compressed in HBM with a 24 GiB decoded-brick cache, fed a stream of
frustum brick-set requests (1..4096 bricks, LOD 0..4).  It reports decoded
GVoxel/s at saturation (a step = one request of the measured trace) and p50 /
p99 request latency at 0.5x and 0.8x the saturation request rate.  Secondary
entries: the 1024^3 neurite volume (32,768 bricks at per-brick LOD 0..3, one
autotuned persistent launch), the 512^3 Voronoi volume with voids (4096
bricks, LOD 0), the 1024^3 u64 uneven batch (32^3 and 64^3 bricks, batched vs
plain) and the 128^3 Voronoi volume (plain).

Every entry: decoded GVoxel/s with inputs resident in HBM before the timed
region, the decode kernel's HBM roofline fraction from HIP events on the
stream it runs on, bit-exactness against the CPU oracle, and the oracle timed
on the host cores over the same tasks (or a bounded sample of them).

    python bench.py [--steps K] [--warmup W] [--workload NAME ...] [--no-cpu] [--no-plain]
    python bench.py --summarize-rocprof DIR --workload NAME   (profile summary text)
    python bench.py --summarize-traffic FETCH_DIR WRITE_DIR --workload NAME
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
HEADLINE = "neurite2048"
SECONDARY = ["neurite1024", "voronoi512", "uneven1024", "voronoi128"]
SERVE_CACHE_BYTES = 24 << 30  # decoded brick cache of the served workload
SERVE_SIDE, SERVE_SLAB = 2048, 32
DECODE_KERNEL = "decode_kernel"


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("decode_kernel.hip", "decode_kernel.h", "csgv_format.h"):
        with open(os.path.join(ROOT, "paper_2609_36898_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, key: str = "hbm_bytes_per_launch"):
    """HBM bytes per launch (or, key hbm_bytes_total, over all decode dispatches
    of the profiled process) from the committed rocprofv3 counter summary, when
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "decode_kernel_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def host_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    sha = None
    try:
        sha = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short=12", "HEAD"], capture_output=True,
                             text=True, timeout=10).stdout.strip() or None
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "git": sha}


def cpu_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------ workloads
class Workload:
    """Container + task list of one workload (built with the product encoder)."""

    def __init__(self, name, container, ids, lods, label_bytes, raw_lod0=None, config=None, plain=False):
        self.name = name
        self.container = container
        self.ids = np.ascontiguousarray(ids, dtype=np.uint32)
        self.lods = np.ascontiguousarray(lods, dtype=np.uint8)
        self.label_bytes = label_bytes
        self.raw_lod0 = raw_lod0  # expected output when every task is LOD 0 in brick order
        self.config = config or {}
        self.plain = plain
        self.served = False


def build_workload(name: str) -> Workload:
    from synth import workloads as W
    import paper_2609_36898_amd as P
    t0 = time.time()
    if name == "voronoi128":
        vol = W.voronoi128()
        c = P.encode_volume(vol, 5)
        n = 64
        wl = Workload(name, c, np.arange(n), np.zeros(n), 4, P.bricks_of_volume(vol, 5),
                      {"workload": "voronoi128_u32_b32_lod0", "volume": [128] * 3, "bricks": n, "seeds": 500,
                       "form": "plain"}, plain=True)
    elif name == "voronoi512":
        vol = W.voronoi512()
        c = P.encode_volume(vol, 5)
        n = 4096
        wl = Workload(name, c, np.arange(n), np.zeros(n), 4, P.bricks_of_volume(vol, 5),
                      {"workload": "voronoi512_voids_u32_b32_lod0", "volume": [512] * 3, "bricks": n,
                       "seeds": 20000, "void_fraction_min": 0.10, "form": "persistent+graph"})
    elif name == "neurite1024":
        vol = W.neurite1024()
        c = P.encode_volume(vol, 5)
        del vol
        n = 32768
        wl = Workload(name, c, np.arange(n), W.neurite1024_lods(n), 4, None,
                      {"workload": "neurite1024_u32_b32_lod0-3", "volume": [1024] * 3, "bricks": n,
                       "tubes": 100000, "lod": "uniform 0..3 per brick", "form": "autotuned persistent+graph"})
    elif name == "uneven1024":
        flat, l2, origins, kinds = W.uneven1024()
        c = P.csgv_encode_bricks(flat, l2, 8, dims=(1024, 1024, 1024), origins=origins)
        n = len(l2)
        wl = Workload(name, c, np.arange(n), np.zeros(n), 8, flat,
                      {"workload": "uneven1024_u64_b32+b64_lod0", "volume": [1024] * 3, "bricks": n,
                       "bricks_64": int((l2 == 6).sum()), "bricks_32": int((l2 == 5).sum()),
                       "kinds": {"constant": int((kinds == 0).sum()), "voronoi": int((kinds == 1).sum()),
                                 "noise": int((kinds == 2).sum())},
                       "form": "persistent+graph vs plain"}, plain=True)
    elif name == "neurite2048":
        # generated and encoded slab by slab (32 planes = one layer of bricks)
        n = SERVE_SIDE
        enc = P.csgv.csgv_encoder(4, dims=(n, n, n))
        for z0 in range(0, n, SERVE_SLAB):
            b = P.bricks_of_volume(W.neurite2048_slab(z0, z0 + SERVE_SLAB), 5)
            enc.add(b, np.full(len(b) >> 15, 5, np.uint8))
            del b
        c = enc.finish()
        nb = (n // 32) ** 3
        wl = Workload(name, c, np.zeros(0), np.zeros(0), 4, None,
                      {"workload": "neurite2048_u32_b32_served", "volume": [n] * 3, "bricks": nb,
                       "tubes": W.NEURITE2048_TUBES, "cache_bytes": SERVE_CACHE_BYTES,
                       "requests": "Poisson arrivals of frustum brick sets, n log-uniform in [1, 4096], LOD 0..4",
                       "form": "served: LRU brick cache + continuous batching"})
        wl.served = True
    else:
        raise ValueError("unknown workload " + name)
    wl.config["compressed_bytes"] = len(c)
    wl.config["container_sha256_16"] = hashlib.sha256(c).hexdigest()[:16]  # identifies the synthetic input
    wl.config["label_bytes"] = wl.label_bytes
    _log("%s: built in %.1f s, %d tasks, %d compressed bytes" % (name, time.time() - t0, len(wl.ids), len(c)))
    return wl


# ---------------------------------------------------------------- measurement
def measure(wl: Workload, args, dev):
    import torch
    import paper_2609_36898_amd as P
    dv = P.DeviceVolume(wl.container, device=dev)
    n = len(wl.ids)
    d_ids, d_lods, d_offs, offs, total = dv.tasks(wl.ids, wl.lods, dev)
    lb = wl.label_bytes
    out = torch.empty(total, dtype=dv.dtype, device=dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    voxels = float(total)
    recs = np.frombuffer(wl.container, dtype=np.uint64, count=dv.info.n_bricks + 1, offset=int(dv.info.offsets_pos))
    rec_bytes = float((recs[wl.ids.astype(np.int64) + 1] - recs[wl.ids.astype(np.int64)]).sum())
    alg_bytes = rec_bytes + voxels * lb  # read each task's record once, write each label once
    stream = torch.cuda.current_stream(dev)
    plan = P.csgv_plan(dv.info, n)
    tune = None
    if args.shape:
        wg, slots, per_cu = (int(v) for v in args.shape.split(","))
        plan.set_opts(wg_size=wg, lds_slots=slots, wgs_per_cu=per_cu)
        tune = {"fixed_shape": args.shape}
    elif not args.no_tune:
        rep = plan.autotune(stream, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status,
                            cache_path=args.tune_cache)
        tune = {"from_cache": bool(rep.from_cache), "tried": int(rep.tried), "best_kernel_ms": round(rep.best_ms, 4),
                "default_kernel_ms": round(rep.default_ms, 4)}
    opts = plan.get_opts()

    def step():
        plan.launch(stream, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps

    # the decode kernel alone: events on the plan's launch stream around it
    plan.set_timing(True)
    kms = []
    for _ in range(max(3, args.steps)):
        step()
        kms.append(plan.last_kernel_ms())
    plan.set_timing(False)
    kernel_ms = float(np.mean(kms))
    torch.cuda.synchronize()

    st_ok = bool((status == 0).all().item())
    bit_exact = None  # decided against the raw bricks (LOD 0) or the oracle below
    if wl.raw_lod0 is not None:
        ref = torch.from_numpy(wl.raw_lod0.view(np.int64 if lb == 8 else np.int32)).to(dev)
        bit_exact = bool(torch.equal(out, ref)) and st_ok
        del ref
    kernel_gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    res = {
        "workload": wl.config.get("workload", wl.name), "tasks": n, "voxels": int(total),
        "value": round(voxels / (ms * 1e-3) / 1e9, 3), "unit": "GVoxel/s", "ms_per_step": round(ms, 4),
        "shape": {"wg_size": int(opts.wg_size), "lds_slots": int(opts.lds_slots),
                  "wgs_per_cu": int(opts.wgs_per_cu), "sort_tasks": int(opts.sort_tasks)},
        "autotune": tune,
        "roofline": {"bound": "hbm", "achieved": round(kernel_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kernel_gbs / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(wl.name),
                     "kernel": DECODE_KERNEL, "kernel_ms": round(kernel_ms, 4), "alg_bytes_per_launch": alg_bytes,
                     "label_bytes_per_launch": voxels * lb,
                     "label_only_frac": round(voxels * lb / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "config": wl.config,
    }

    if args.calib_copy:
        calib_copy(dev)

    if wl.plain and not args.no_plain:
        plain_out = torch.empty_like(out)
        P.csgv_decode_bricks(stream, dv.info, dv.tensor, d_ids, d_lods, d_offs, n, plain_out, total, status,
                             mode=P.MODE_PLAIN)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for _ in range(args.plain_steps):
            P.csgv_decode_bricks(stream, dv.info, dv.tensor, d_ids, d_lods, d_offs, n, plain_out, total, status,
                                 mode=P.MODE_PLAIN)
        p1.record(stream)
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / args.plain_steps
        res["plain"] = {"value": round(voxels / (plain_ms * 1e-3) / 1e9, 3), "unit": "GVoxel/s",
                        "ms_per_step": round(plain_ms, 3), "launches_per_step": n,
                        "bit_exact": bool(torch.equal(plain_out, out))}
        del plain_out

    if not args.no_cpu:
        got = out.cpu().numpy().view(np.uint64 if lb == 8 else np.uint32)
        res["cpu_baseline"] = cpu_baseline(wl, offs, total, got)
        if bit_exact is None:
            bit_exact = res["cpu_baseline"]["matches_gpu"] and st_ok
        del got
    res["bit_exact"] = bit_exact
    plan.destroy()
    del out, status, dv
    torch.cuda.empty_cache()
    return res


def calib_copy(dev):
    """Device copies of CALIB_COPY_BYTES: the reference kernel for HBM counter scaling."""
    import torch
    src = torch.empty(CALIB_COPY_BYTES // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def measure_paletted(wl: Workload, args, dev, shape):
    """The same task list decoded to cache-paletted form (packed palette
    indices, I = ceil(log2 |P|max) bits, floor(32/I) per 32-bit word) with the
    plan shape the label run chose; bit-exact against the oracle's paletted
    decode of every task."""
    import torch
    import oracle
    import paper_2609_36898_amd as P
    dv = P.DeviceVolume(wl.container, device=dev)
    n = len(wl.ids)
    bits = P.csgv.palette_bits_for(dv.info.max_palette)
    log2b = P.brick_log2b(wl.container, dv.info)[wl.ids.astype(np.int64)]
    voxels = np.int64(1) << (3 * (log2b - wl.lods.astype(np.int64)))
    words = P.csgv.paletted_words(voxels, bits)
    offs = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    total = int(words.sum())
    d_ids = torch.from_numpy(wl.ids.view(np.int32)).to(dev)
    d_lods = torch.from_numpy(wl.lods).to(dev)
    d_offs = torch.from_numpy(offs.view(np.int64)).to(dev)
    out = torch.empty(total, dtype=torch.int32, device=dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    plan = P.csgv_plan(dv.info, n, wg_size=shape["wg_size"], lds_slots=shape["lds_slots"], palette_bits=bits)

    def step():
        plan.launch(stream, dv.tensor, d_ids, d_lods, d_offs, n, out, total, status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    plan.set_timing(True)
    kms = []
    for _ in range(max(3, args.steps)):
        step()
        kms.append(plan.last_kernel_ms())
    plan.destroy()
    torch.cuda.synchronize()
    kernel_ms = float(np.mean(kms))
    recs = np.frombuffer(wl.container, dtype=np.uint64, count=dv.info.n_bricks + 1, offset=int(dv.info.offsets_pos))
    rec_bytes = float((recs[wl.ids.astype(np.int64) + 1] - recs[wl.ids.astype(np.int64)]).sum())
    alg = rec_bytes + 4.0 * total
    got = out.cpu().numpy().view(np.uint32)
    st = status.cpu().numpy()
    want, wst = oracle.decode_tasks_paletted(wl.container, wl.ids, wl.lods, offs, total, bits, nthreads=cpu_threads())
    exact = bool((st == 0).all()) and bool((wst == 0).all()) and bool(np.array_equal(got, want))
    vox = float(voxels.sum())
    del out, dv
    torch.cuda.empty_cache()
    kgbs = alg / (kernel_ms * 1e-3) / 1e9
    return {"value": round(vox / (ms * 1e-3) / 1e9, 3) if exact else None, "unit": "GVoxel/s",
            "ms_per_step": round(ms, 4), "bit_exact": exact,
            "config": {"workload": wl.config["workload"] + "_paletted", "palette_bits": bits,
                       "max_palette": int(P.csgv_volume_parse(wl.container).max_palette),
                       "indices_per_word": 32 // bits, "words_per_launch": total,
                       "label_bytes_saved": round(1.0 - 4.0 * total / (vox * wl.label_bytes), 4)},
            "roofline": {"bound": "hbm", "achieved": round(kgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(kgbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": DECODE_KERNEL,
                         "kernel_ms": round(kernel_ms, 4), "alg_bytes_per_launch": alg}}


def measure_served(wl: Workload, args, dev):
    """The served workload: the compressed volume and a 24 GiB decoded-brick
    cache resident in HBM, a stream of frustum requests through the server.

    Three runs on fresh servers, each after the same warm-up requests: every
    measured request at t = 0 (saturation: the admission queue never empties),
    then Poisson arrivals at 0.5x and 0.8x the saturation request rate.  A
    request's latency runs from its arrival until all of its pairs are
    resident.  GVoxel/s counts voxels decoded (cache misses) per second of the
    run; served GVoxel/s counts every requested voxel.  Bit-exactness: pinned
    requests of the trace, served one by one, against the CPU oracle."""
    import torch
    import oracle
    import paper_2609_36898_amd as P
    from synth import workloads as W
    dv = P.DeviceVolume(wl.container, device=dev)
    if args.calib_copy:
        calib_copy(dev)
    cache_elems = SERVE_CACHE_BYTES // 4
    cache = torch.empty(cache_elems, dtype=torch.int32, device=dev)
    nw, nm = args.serve_warmup, args.serve_requests
    g = SERVE_SIDE // 32
    t0 = time.time()
    ids, lods, starts, unit_arr = W.frustum_requests(nw + nm, (g, g, g), 1.0, seed=11, n_max=4096)
    _log("%s: %d requests (%d pairs) generated in %.1f s" % (wl.name, nw + nm, len(ids), time.time() - t0))
    sw = int(starts[nw])
    m_ids, m_lods = ids[sw:], lods[sw:]
    m_starts = starts[nw:] - starts[nw]
    lod_hist = np.bincount(lods, minlength=5).tolist()

    # algorithmic bytes of every decode dispatch this process makes (all servers)
    proc = {"alg": 0.0, "dispatches": 0}

    def account(s):
        proc["alg"] += s["record_bytes"] + 4.0 * s["decoded_elements"]
        proc["dispatches"] += s["batches"]

    def run(rate):
        srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=args.serve_streams,
                                 max_batch=args.serve_batch, n_shards=args.serve_shards)
        srv.run(ids[:sw], lods[:sw], starts[:nw + 1], np.zeros(nw))
        s0 = srv.stats()
        arr = np.zeros(nm) if rate is None else (unit_arr[nw:] - unit_arr[nw]) / rate
        rec = srv.run(m_ids, m_lods, m_starts, arr)
        s1 = srv.stats()
        account(s1)
        srv.destroy()
        d = {k: s1[k] - s0[k] for k in s1 if k not in ("cache_top", "resident", "pinned", "max_batch_seen")}
        span = float(rec["t_done"].max())
        lat = (rec["t_done"] - rec["t_arrival"]) * 1e3
        ok = bool((rec["status"] == 0).all()) and d["failed_tasks"] == 0
        res = {"rate_hz": None if rate is None else round(rate, 2), "requests": nm, "seconds": round(span, 4),
               "requests_per_s": round(nm / span, 2),
               "decoded_gvoxel_s": round(d["decoded_elements"] / span / 1e9, 3),
               "served_gvoxel_s": round(d["requested_elements"] / span / 1e9, 3),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "hit_fraction": round((d["hits"] + d["joined"]) / max(d["pairs_requested"], 1), 4),
               "batches": d["batches"], "decoded_pairs": d["decoded"], "evictions": d["evictions"],
               "splits": d["splits"], "resets": d["resets"], "kernel_ms": round(d["kernel_ms"], 3), "all_ok": ok}
        return res, d

    sat, sat_d = run(None)
    _log("%s: saturation %.0f req/s, %.2f GVoxel/s decoded, p50 %.2f ms" % (
        wl.name, sat["requests_per_s"], sat["decoded_gvoxel_s"], sat["p50_ms"]))
    loads = {}
    for f in (0.5, 0.8):
        loads["load_%.1f" % f], _ = run(f * sat["requests_per_s"])
        _log("%s: %.1fx load: p50 %.3f ms p99 %.3f ms" % (wl.name, f, loads["load_%.1f" % f]["p50_ms"],
                                                           loads["load_%.1f" % f]["p99_ms"]))
    # the decode kernel over the saturation run: algorithmic bytes / kernel time
    alg = sat_d["record_bytes"] + 4.0 * sat_d["decoded_elements"]
    kgbs = alg / (sat_d["kernel_ms"] * 1e-3) / 1e9 if sat_d["kernel_ms"] > 0 else 0.0

    # bit-exactness: pinned requests of the measured trace against the oracle
    n_req = len(m_starts) - 1
    sizes = np.diff(m_starts.astype(np.int64))
    check = [r for r in range(n_req) if sizes[r] <= 1024][:args.serve_check]
    srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=args.serve_streams,
                             max_batch=args.serve_batch, keep_pinned=True, n_shards=args.serve_shards)
    exact = True
    c_ids, c_lods, c_got = [], [], []
    for r in check:
        a, b = int(m_starts[r]), int(m_starts[r + 1])
        rid, rl = m_ids[a:b], m_lods[a:b]
        q = srv.submit(rid, rl, srv.clock())
        done = []
        while not done:
            srv.step()
            done = srv.drain()
        exact &= all(d.status == 0 for d in done)
        torch.cuda.synchronize()
        for i, l in zip(rid, rl):
            o = srv.where(int(i), int(l))
            c_got.append(cache[o:o + (32 >> int(l)) ** 3].cpu().numpy().view(np.uint32))
        c_ids.append(rid)
        c_lods.append(rl)
        srv.release(q)
    account(srv.stats())
    srv.destroy()
    c_ids, c_lods = np.concatenate(c_ids), np.concatenate(c_lods)
    offs, total = P.dense_offsets(np.full(len(c_ids), 5, np.uint8), c_lods)
    want, wst = oracle.decode_tasks(wl.container, c_ids, c_lods, offs, total, 4, nthreads=cpu_threads())
    exact = exact and bool((wst == 0).all()) and bool(np.array_equal(np.concatenate(c_got), want))
    _log("%s: %d pinned requests (%d pairs) bit-exact vs oracle: %s" % (wl.name, len(check), len(c_ids), exact))
    staged = None if args.no_dcache else device_staged(P, dv, cache, cache_elems, wl.container, ids, lods, starts, nw,
                                                        args.dcache_chunk, args.dcache_keep, proc)
    del cache, dv
    torch.cuda.empty_cache()

    # HBM traffic: the profiled process's decode dispatches moved hbm_total bytes for the
    # algorithmic bytes proc["alg"] of the same work (the served pairs do not depend on
    # timing); that ratio, applied to a saturation launch, is its traffic per launch
    alg_launch = alg / max(sat_d["batches"], 1)
    hbm_total = profiled_traffic(wl.name, "hbm_bytes_total")
    ratio = hbm_total / proc["alg"] if hbm_total and proc["alg"] > 0 else None
    res = {
        "value": sat["decoded_gvoxel_s"], "ms_per_step": round(1e3 * sat["seconds"] / nm, 4),
        "config": dict(wl.config, warmup_requests=nw, measured_requests=nm, lod_histogram=lod_hist,
                       streams=args.serve_streams, max_batch=args.serve_batch, shards=args.serve_shards),
        "roofline": {"bound": "hbm", "achieved": round(kgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kgbs / HBM_PEAK_GBS, 4),
                     "traffic": round(ratio * alg_launch, 1) if ratio else None,
                     "traffic_over_alg": round(ratio, 4) if ratio else None,
                     "kernel": DECODE_KERNEL, "kernel_ms_total": round(sat_d["kernel_ms"], 3),
                     "launches": sat_d["batches"], "alg_bytes_total": alg,
                     "alg_bytes_per_launch": round(alg_launch, 1),
                     "process_alg_bytes": proc["alg"], "process_dispatches": proc["dispatches"],
                     "note": "over the saturation run: sum of algorithmic bytes / sum of decode-kernel times "
                             "(launches of several shards overlap); traffic = the profiled process's HBM bytes "
                             "over all decode dispatches / its algorithmic bytes, times alg_bytes_per_launch"},
        "served": {"saturation": sat, **loads, "checked_requests": len(check), "checked_pairs": int(len(c_ids)),
                   "device_staged": staged},
        "bit_exact": exact and sat["all_ok"] and all(v["all_ok"] for v in loads.values())
        and (staged is None or staged["bit_exact"]),
        "shape": {"wg_size": "default", "sort_tasks": "default"},
        "autotune": None,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_served(wl, m_ids, m_lods, m_starts)
    return res


def chunk_schedule(ids, lods, starts, n_warm, chunk_pairs, keep):
    """Chunks of whole requests (at most chunk_pairs pairs unless one request is larger; the first
    measured request starts a chunk) and the release schedule: a pair used in chunk c and not again
    in chunks c+1..c+keep is released right after chunk c+keep (pairs still in use at the end stay).
    Returns the chunks' pair boundaries, the first measured chunk, the released keys (id * 8 + lod)
    ordered by chunk, and per chunk the range of its releases in that list."""
    n_req = len(starts) - 1
    sizes = np.diff(starts.astype(np.int64))
    bounds, acc = [0], 0
    for r in range(n_req):
        if (acc + sizes[r] > chunk_pairs and acc > 0) or (r == n_warm and r > 0):
            bounds.append(r)
            acc = 0
        acc += int(sizes[r])
    bounds.append(n_req)
    pb = [int(starts[b]) for b in bounds]
    n_chunks = len(bounds) - 1
    first_measured = bounds.index(n_warm) if n_warm < n_req else n_chunks
    chunk_of = np.repeat(np.arange(n_chunks), np.diff(pb))
    key = ids.astype(np.int64) * 8 + lods.astype(np.int64)
    kc = np.unique(key * n_chunks + chunk_of)
    k, c = kc // n_chunks, kc % n_chunks
    nxt = np.full(len(kc), 1 << 40, np.int64)
    same = k[1:] == k[:-1]
    nxt[:-1][same] = c[1:][same]
    rel = (nxt - c > keep) & (c + keep < n_chunks)
    rk, rat = k[rel], c[rel] + keep
    order = np.argsort(rat, kind="stable")
    rk, rat = rk[order], rat[order]
    return pb, first_measured, rk, np.searchsorted(rat, np.arange(n_chunks + 1))


def device_staged(P, dv, cache, cache_elems, container, ids, lods, starts, n_warm, chunk_pairs, keep=16, proc=None):
    """The served trace with the cache stages on the device: whole requests
    concatenated into chunks of at most chunk_pairs pairs, each distinct pair
    of a chunk requested once; per chunk one request/provision/assign call, one decode launch over the chunk's request
    arrays (non-tasks are rejected by the decoder), then the release of every
    pair whose last use was `keep` chunks ago (the no-longer-requested pairs go
    onto the free stacks).  Every chunk is enqueued on one stream up front: no
    host round trip.  Saturation only (all requests at t = 0); the warm-up
    requests run first, untimed.  Bit-exactness: the last chunk's pairs, which
    are still resident at the end, against the CPU oracle."""
    import torch
    import oracle
    dev = cache.device
    n_req = len(starts) - 1
    pb, first_measured, rk, rel_b = chunk_schedule(ids, lods, starts, n_warm, chunk_pairs, keep)
    n_chunks = len(pb) - 1
    d_rel_ids = torch.from_numpy((rk // 8).astype(np.uint32).view(np.int32)).to(dev)
    d_rel_lods = torch.from_numpy((rk % 8).astype(np.uint8)).to(dev)

    # a chunk's request list names each pair once, as the paper's request stage does per frame
    served = float((np.int64(1) << (3 * (5 - lods[pb[first_measured]:].astype(np.int64)))).sum())
    req_pairs = int(starts[-1]) - int(starts[n_warm])
    chunk_of = np.repeat(np.arange(n_chunks, dtype=np.int64), np.diff(pb))
    uk = np.unique((chunk_of << 40) + ids.astype(np.int64) * 8 + lods.astype(np.int64))
    ub = [int(v) for v in np.searchsorted(uk >> 40, np.arange(n_chunks + 1))]
    ids = ((uk & ((1 << 40) - 1)) // 8).astype(np.uint32)
    lods = ((uk & ((1 << 40) - 1)) % 8).astype(np.uint8)
    pb = ub
    n = len(uk)
    d_ids = torch.from_numpy(ids.view(np.int32)).to(dev)
    d_lods = torch.from_numpy(lods).to(dev)
    task = torch.empty(n, dtype=torch.int32, device=dev)
    slot = torch.empty(n, dtype=torch.int64, device=dev)
    state = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    dc = P.csgv.csgv_dcache(dv.info, dv.tensor, cache_elems, stream=stream)
    plan = P.csgv_plan(dv.info, max(int(np.diff(pb).max()), 1))
    plan.set_graph(False)  # every chunk has its own arrays and count: a captured graph would be rebuilt each time
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.time()
    for ch in range(n_chunks):
        if ch == first_measured:
            ev0.record(stream)
        a, b = pb[ch], pb[ch + 1]
        if b > a:
            dc.request(stream, d_ids[a:], d_lods[a:], b - a, task[a:], slot[a:], state[a:])
            plan.launch(stream, dv.tensor, task[a:], d_lods[a:], slot[a:], b - a, cache, cache_elems, status[a:])
        r0, r1 = int(rel_b[ch]), int(rel_b[ch + 1])
        if r1 > r0:
            dc.free(stream, d_rel_ids[r0:], d_rel_lods[r0:], r1 - r0)
    ev1.record(stream)
    host_s = time.time() - t0  # enqueueing every chunk, warm-up included (the device may still be busy)
    torch.cuda.synchronize()
    secs = ev0.elapsed_time(ev1) * 1e-3
    st = state.cpu().numpy()
    ts = status.cpu().numpy()
    sl = slot.cpu().numpy().view(np.uint64)
    m0 = pb[first_measured]
    new = st == 0
    units = np.int64(1) << (3 * (5 - lods.astype(np.int64)))
    ok = bool((ts[new] == 0).all())
    full = int((st[m0:] == 3).sum())
    if proc is not None:  # algorithmic bytes of every decode dispatch of this run (warm-up included)
        recs = np.frombuffer(container, dtype=np.uint64, count=dv.info.n_bricks + 1, offset=int(dv.info.offsets_pos))
        nid = ids[new].astype(np.int64)
        proc["alg"] += float((recs[nid + 1] - recs[nid]).sum()) + 4.0 * float(units[new].sum())
        proc["dispatches"] += sum(1 for ch in range(n_chunks) if pb[ch + 1] > pb[ch])
    # the last chunk's pairs against the oracle (a bounded sample)
    a = pb[-2]
    pick = np.arange(a, n)[:512]
    host = [cache[int(sl[i]):int(sl[i]) + int(units[i])].cpu().numpy().view(np.uint32) for i in pick
            if st[i] in (0, 1, 2)]
    pids, plods = ids[pick][np.isin(st[pick], (0, 1, 2))], lods[pick][np.isin(st[pick], (0, 1, 2))]
    offs, total = P.dense_offsets(np.full(len(pids), 5, np.uint8), plods)
    want, wst = oracle.decode_tasks(container, pids, plods, offs, total, 4, nthreads=cpu_threads())
    exact = ok and bool((wst == 0).all()) and bool(np.array_equal(np.concatenate(host), want)) if len(host) else ok
    top, _ = dc.query(stream)
    dc.destroy()
    n_meas = n_req - n_warm
    res = {"requests": n_meas, "chunks": n_chunks - first_measured, "max_chunk_pairs": chunk_pairs,
           "release_after_chunks": keep, "seconds": round(secs, 4), "requests_per_s": round(n_meas / secs, 2),
           "decoded_gvoxel_s": round(float(units[m0:][new[m0:]].sum()) / secs / 1e9, 3),
           "served_gvoxel_s": round(served / secs / 1e9, 3),
           "chunk_pairs": n - m0,
           "hit_fraction": round(1.0 - float(new[m0:].sum() + full) / max(req_pairs, 1), 4),
           "full_pairs": full, "cache_top_elements": top, "host_enqueue_s": round(host_s, 3),
           "checked_pairs": int(len(pids)), "bit_exact": exact}
    _log("device-staged: %.0f req/s, %.2f GVoxel/s decoded, %d chunks, hit fraction %.3f, full %d, exact %s" % (
        res["requests_per_s"], res["decoded_gvoxel_s"], res["chunks"], res["hit_fraction"], full, exact))
    return res


ABLATION = [("adv", 0), ("+parent", 1), ("+nx", 3), ("+ny", 7), ("+nz", 15), ("+last", 31), ("+delta", 63),
            ("+delta<=16", 127)]


def op_ablation(args, dev):
    """Operation-set ablation: every prefix of PARENT, NX, NY, NZ, LAST, DELTA
    (ADV always on) and DELTA limited to 16 entries, on voronoi512 (LOD 0) and
    neurite1024 (its LOD mix): compressed bytes, bits per voxel, palette
    lengths and duplicates, and batched decode GVoxel/s (default shape), each
    run bit-exact against the raw volume or the CPU oracle."""
    import torch
    import oracle
    import paper_2609_36898_amd as P
    from synth import workloads as W
    rows = []
    for name in ("voronoi512", "neurite1024"):
        vol = W.voronoi512() if name == "voronoi512" else W.neurite1024()
        n_b = (vol.shape[0] // 32) ** 3
        lods = np.zeros(n_b, np.uint8) if name == "voronoi512" else W.neurite1024_lods(n_b)
        raw = P.bricks_of_volume(vol, 5) if name == "voronoi512" else None
        for label, mask in ABLATION:
            t0 = time.time()
            c = P.encode_volume(vol, 5, op_mask=mask)
            enc_s = time.time() - t0
            info = P.csgv_volume_parse(c)
            pals = np.array([int(np.frombuffer(c, np.uint32, count=1, offset=int(o) + 4)[0])
                             for o in np.frombuffer(c, np.uint64, count=n_b, offset=int(info.offsets_pos))])
            dv = P.DeviceVolume(c, device=dev)
            ids = np.arange(n_b, dtype=np.uint32)
            d_ids, d_lods, d_offs, offs, total = dv.tasks(ids, lods, dev)
            out = torch.empty(total, dtype=dv.dtype, device=dev)
            status = torch.full((n_b,), -1, dtype=torch.int32, device=dev)
            plan = P.csgv_plan(dv.info, n_b)
            stream = torch.cuda.current_stream(dev)
            for _ in range(args.warmup):
                plan.launch(stream, dv.tensor, d_ids, d_lods, d_offs, n_b, out, total, status)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                plan.launch(stream, dv.tensor, d_ids, d_lods, d_offs, n_b, out, total, status)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            plan.destroy()
            got = out.cpu().numpy().view(np.uint32)
            if raw is not None:
                exact = bool(np.array_equal(got, raw))
            else:
                want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 4, nthreads=cpu_threads())
                exact = bool(np.array_equal(got, want)) and bool((wst == 0).all())
            exact = exact and bool((status == 0).all().item())
            del out, dv
            torch.cuda.empty_cache()
            row = {"workload": name, "ops": label, "op_mask": mask, "compressed_bytes": len(c),
                   "bits_per_voxel": round(8.0 * len(c) / vol.size, 4), "palette_mean": round(float(pals.mean()), 2),
                   "palette_max": int(pals.max()), "decode_gvoxel_s": round(total / (ms * 1e-3) / 1e9, 2) if exact else None,
                   "ms_per_step": round(ms, 4), "bit_exact": exact, "encode_s": round(enc_s, 2)}
            _log(json.dumps(row))
            rows.append(row)
        del vol
    return rows


def cpu_baseline_served(wl: Workload, ids, lods, starts):
    """The oracle decoding every pair of the first measured requests (about
    1/20 of the trace's pairs, cache hits included) on all host cores."""
    import oracle
    import paper_2609_36898_amd as P
    threads = cpu_threads()
    k = int(np.searchsorted(starts.astype(np.int64), len(ids) // 20))
    a = int(starts[k])
    s_ids, s_lods = ids[:a], lods[:a]
    offs, total = P.dense_offsets(np.full(len(s_ids), 5, np.uint8), s_lods)
    out = np.empty(total, dtype=np.uint32)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.decode_tasks(wl.container, s_ids, s_lods, offs, total, 4, nthreads=threads, out=out)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    info = host_info()
    return {"value": round(total / dt / 1e9, 4), "unit": "GVoxel/s", "cores": threads, "kind": "oracle",
            "sample": "every pair of the first %d measured requests (%d pairs, %d voxels), OpenMP over pairs on "
                      "%d threads, median of 3 runs of %.2f s" % (k, a, total, threads, dt),
            "nproc": info["nproc"], "cpu_model": info["cpu_model"]}


def cpu_baseline(wl: Workload, offs, total, gpu_out):
    """The oracle decoding the same task list: all host cores (16 at most) over
    every task, and one thread over a bounded sample (about 2 s)."""
    import oracle
    lb = wl.label_bytes
    threads = cpu_threads()
    cpu_out = np.empty(total, dtype=np.uint64 if lb == 8 else np.uint32)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        cpu_out, st = oracle.decode_tasks(wl.container, wl.ids, wl.lods, offs, total, lb, nthreads=threads,
                                          out=cpu_out)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    matches = bool(np.array_equal(cpu_out, gpu_out)) and bool((st == 0).all())
    del cpu_out
    n = len(wl.ids)
    k = max(1, min(n, int(n * min(1.0, 2.0 / max(dt * threads, 1e-3)))))
    sel = np.linspace(0, n - 1, k).astype(np.int64)
    s_offs, s_total = _dense(wl, sel)
    t0 = time.perf_counter()
    oracle.decode_tasks(wl.container, wl.ids[sel], wl.lods[sel], s_offs, s_total, lb, nthreads=1)
    dt1 = time.perf_counter() - t0
    info = host_info()
    return {"value": round(total / dt / 1e9, 4), "unit": "GVoxel/s", "cores": threads, "kind": "oracle",
            "sample": "every task (%d), OpenMP over tasks on %d threads, median of 3 runs of %.2f s" %
                      (n, threads, dt),
            "single_thread": {"value": round(s_total / dt1 / 1e9, 4), "unit": "GVoxel/s",
                              "sample": "%d of %d tasks evenly spaced, %.2f s" % (k, n, dt1)},
            "nproc": info["nproc"], "cpu_model": info["cpu_model"], "matches_gpu": matches}


def _dense(wl, sel):
    import paper_2609_36898_amd as P
    log2b = P.brick_log2b(wl.container)
    return P.dense_offsets(log2b[wl.ids[sel].astype(np.int64)], wl.lods[sel])


# ------------------------------------------------------------ profile summary
def summarize_rocprof(directory: str, workload: str) -> str:
    """Text summary of a rocprofv3 run of this script (its SQLite output, or
    CSV): kernel-trace statistics and/or per-kernel counter means."""
    import csv
    import sqlite3
    lines = ["workload: %s" % workload, "kernel_source_sha256_16: %s" % kernel_source_hash()]
    for path in sorted(glob.glob(os.path.join(directory, "**", "*_results.db"), recursive=True)):
        con = sqlite3.connect(path)
        try:
            rows = con.execute("select name, total_calls, average, total_duration, percentage from top_kernels "
                               "order by total_duration desc limit 12").fetchall()
            if rows:
                # the top_kernels view reports microseconds
                lines.append("# kernel trace (%s), durations in ns" % os.path.basename(path))
                for name, calls, avg, tot, pct in rows:
                    lines.append("%-64s calls %5d  avg_ns %12.1f  total_ns %14.1f  pct %5.1f" % (
                        name[:64], calls, 1e3 * avg, 1e3 * tot, pct))
        except sqlite3.Error:
            pass
        try:
            rows = con.execute("select kernel_name, counter_name, count(*), avg(value) from counters_collection "
                               "group by kernel_name, counter_name").fetchall()
            if rows:
                lines.append("# counters (%s): mean per dispatch" % os.path.basename(path))
                for name, ctr, n, mean in sorted(rows, key=lambda r: (DECODE_KERNEL not in r[0], r[0], r[1])):
                    kind = "decode_kernel" if DECODE_KERNEL in name else name.split("(")[0][-40:]
                    lines.append("%-40s %-24s dispatches %4d  mean %.6g" % (kind, ctr, n, mean))
        except sqlite3.Error:
            pass
        con.close()
    for path in sorted(glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True)):
        lines.append("# %s" % os.path.relpath(path, directory))
        with open(path) as f:
            for row in csv.DictReader(f):
                lines.append("%-60s calls %6s  avg_ns %12s  total_ns %14s  pct %s" % (
                    row.get("Name", "")[:60], row.get("Calls"), row.get("AverageNs"), row.get("TotalDurationNs"),
                    row.get("Percentage")))
    return "\n".join(lines) + "\n"


CALIB_COPY_BYTES = 1 << 30  # --calib-copy moves this many bytes per copy


def _counter_values(directory: str, counter: str):
    """Per-dispatch values of one counter: {kernel kind: [values]} from rocprofv3's SQLite output."""
    import sqlite3
    vals = {}
    for path in sorted(glob.glob(os.path.join(directory, "**", "*_results.db"), recursive=True)):
        con = sqlite3.connect(path)
        for name, v in con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                                   (counter,)):
            kind = DECODE_KERNEL if DECODE_KERNEL in name else name.split("(")[0].split()[-1]
            vals.setdefault(kind, []).append(float(v))
        con.close()
    return vals


def summarize_traffic(fetch_dir: str, write_dir: str, workload: str) -> str:
    """HBM bytes per decode launch from FETCH_SIZE and WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the same counter reads for the calibration
    copy of CALIB_COPY_BYTES."""
    f = _counter_values(fetch_dir, "FETCH_SIZE")
    w = _counter_values(write_dir, "WRITE_SIZE")
    copy_f = max(f.get("__amd_rocclr_copyBuffer", [0.0]))
    copy_w = max(w.get("__amd_rocclr_copyBuffer", [0.0]))
    if not f.get(DECODE_KERNEL) or not w.get(DECODE_KERNEL) or copy_f <= 0 or copy_w <= 0:
        raise SystemExit("need decode and calibration-copy dispatches in both runs")
    kf = CALIB_COPY_BYTES / 1024.0 / copy_f
    kw = CALIB_COPY_BYTES / 1024.0 / copy_w
    df, dw = float(np.mean(f[DECODE_KERNEL])), float(np.mean(w[DECODE_KERNEL]))
    rd, wr = df * kf * 1024.0, dw * kw * 1024.0
    # over all decode dispatches of a run (each counter run does the same work)
    tot = (float(np.sum(f[DECODE_KERNEL])) * kf + float(np.sum(w[DECODE_KERNEL])) * kw) * 1024.0
    return "\n".join([
        "workload: %s" % workload,
        "kernel_source_sha256_16: %s" % kernel_source_hash(),
        "calibration copy of %d bytes: FETCH_SIZE %.1f KiB (scale %.4f), WRITE_SIZE %.1f KiB (scale %.4f)" % (
            CALIB_COPY_BYTES, copy_f, kf, copy_w, kw),
        "decode_kernel dispatches: FETCH_SIZE %d, WRITE_SIZE %d" % (len(f[DECODE_KERNEL]), len(w[DECODE_KERNEL])),
        "decode_kernel FETCH_SIZE mean %.1f KiB -> read bytes %.0f" % (df, rd),
        "decode_kernel WRITE_SIZE mean %.1f KiB -> written bytes %.0f" % (dw, wr),
        "hbm_bytes_per_launch: %.0f" % (rd + wr),
        "hbm_bytes_total: %.0f" % tot,
    ]) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--workload", nargs="*", default=None,
                    help="workloads to run (first = headline); default: %s %s" % (HEADLINE, " ".join(SECONDARY)))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain one-launch-per-brick legs")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape instead of the autotuner")
    ap.add_argument("--shape", default=None, metavar="WG,SLOTS,WGS_PER_CU",
                    help="fixed launch shape of the batched legs instead of the autotuner (profiling runs)")
    ap.add_argument("--no-paletted", action="store_true", help="skip the cache-paletted leg of neurite1024")
    ap.add_argument("--ablation", action="store_true",
                    help="operation-set ablation (compressed size and decode GVoxel/s per op prefix) instead")
    ap.add_argument("--tune-cache", default=os.environ.get("CSGV_TUNE_CACHE", "/tmp/csgv_autotune.txt"))
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run device-to-device copies of CALIB_COPY_BYTES (reference kernel for HBM counter scaling)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="measured requests of the served workload")
    ap.add_argument("--serve-warmup", type=int, default=1000, help="warm-up requests before each served run")
    ap.add_argument("--serve-streams", type=int, default=2, help="HIP streams per cache shard")
    ap.add_argument("--serve-shards", type=int, default=16, help="cache shards (host threads) of the server")
    ap.add_argument("--serve-batch", type=int, default=16384, help="tasks per served batch (per shard stream)")
    ap.add_argument("--no-dcache", action="store_true", help="skip the device-staged served run")
    ap.add_argument("--dcache-chunk", type=int, default=65536, help="device-staged run: request pairs per chunk")
    ap.add_argument("--dcache-keep", type=int, default=16,
                    help="device-staged run: a pair not requested for this many chunks is released")
    ap.add_argument("--serve-check", type=int, default=24, help="pinned requests checked against the oracle")
    ap.add_argument("--summarize-rocprof", default=None, metavar="DIR")
    ap.add_argument("--summarize-traffic", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"))
    args = ap.parse_args()
    if args.summarize_traffic:
        sys.stdout.write(summarize_traffic(*args.summarize_traffic, (args.workload or [HEADLINE])[0]))
        return
    if args.summarize_rocprof:
        sys.stdout.write(summarize_rocprof(args.summarize_rocprof, (args.workload or [HEADLINE])[0]))
        return
    if args.ablation:
        import torch
        dev = torch.device("cuda:0")
        rows = op_ablation(args, dev)
        print(json.dumps({"op_ablation": rows, "kernel_source": kernel_source_hash()}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the decode path has no multi-GPU form in this build (bricks are "
              "independent; a multi-GPU form would shard tasks by brick-id range with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    names = args.workload if args.workload else [HEADLINE] + SECONDARY
    results = []
    for name in names:
        wl = build_workload(name)
        r = measure_served(wl, args, dev) if wl.served else measure(wl, args, dev)
        if name == "neurite1024" and not args.no_paletted:
            r["paletted"] = measure_paletted(wl, args, dev, r["shape"])
            _log("%s paletted: %.2f GVoxel/s, bit_exact %s" % (name, r["paletted"]["value"] or 0.0,
                                                                r["paletted"]["bit_exact"]))
        _log("%s: %.2f GVoxel/s, roofline %.3f, bit_exact %s" % (
            name, r["value"], r["roofline"]["frac"], r["bit_exact"]))
        if "served" in r:
            _log("%s: served %s" % (name, json.dumps(r["served"])))
        results.append(r)
        del wl
    head = results[0]
    served = "served" in head
    line = {
        "metric": "decoded GVoxel/s (bit-exact) batched vs plain; p50/p99 brick-request latency",
        "value": head["value"] if head["bit_exact"] else None,
        "unit": "GVoxel/s",
        "n_gpus": 1,
        # served workload: a step is one request of the measured trace
        "steps": args.serve_requests if served else args.steps,
        "warmup": args.serve_warmup if served else args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if head["config"].get("label_bytes") == 8 else "u32",
        "data": "synthetic",
        "config": head["config"],
        "bit_exact": head["bit_exact"],
        "roofline": head["roofline"],
        "shape": head["shape"],
        "autotune": head["autotune"],
    }
    if "cpu_baseline" in head:
        line["cpu_baseline"] = head["cpu_baseline"]
    if "plain" in head:
        line["plain"] = head["plain"]
    if served:
        line["served"] = head["served"]
    line["secondary"] = results[1:]
    line["env"] = dict(host_info(), gpu=torch.cuda.get_device_name(dev), kernel_source=kernel_source_hash())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
