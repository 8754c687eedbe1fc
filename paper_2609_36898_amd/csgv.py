"""Python binding of libcsgv (ctypes; argument marshalling only).

Every function here forwards to the C ABI of the same name in
include/csgv.h; all decoding runs in the HIP kernels of libcsgv.so.  Device
buffers are passed as torch tensors on a ROCm device (torch names HIP devices
"cuda") or as raw integer addresses.  There is no CPU fallback: importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsgv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcsgv.so is not built (run __graft_entry__.build() or python -m paper_2609_36898_amd._build)")

_lib = ctypes.CDLL(LIB_PATH)

CSGV_OK, CSGV_EINVAL, CSGV_ECORRUPT, CSGV_ENOMEM, CSGV_EHIP = 0, -1, -2, -3, -4
TASK_OK, TASK_INVALID, TASK_CORRUPT = 0, 1, 2
MODE_PLAIN, MODE_PERSISTENT = 0, 2
ALL_OPS = 63


class VolumeInfo(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_uint32 * 3),
        ("log2b", ctypes.c_uint32),
        ("label_bytes", ctypes.c_uint32),
        ("op_mask", ctypes.c_uint32),
        ("n_bricks", ctypes.c_uint32),
        ("grid", ctypes.c_uint32 * 3),
        ("rans_freq", ctypes.c_uint16 * 16),
        ("offsets_pos", ctypes.c_uint64),
        ("dir_pos", ctypes.c_uint64),
        ("total_bytes", ctypes.c_uint64),
        ("neighbor_mode", ctypes.c_uint32),
        ("max_log2b", ctypes.c_uint32),
        ("max_palette", ctypes.c_uint32),
    ]


class DecodeOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("wg_size", ctypes.c_int), ("wgs_per_cu", ctypes.c_int),
                ("sort_tasks", ctypes.c_int), ("bricks_per_wave", ctypes.c_int), ("lds_slots", ctypes.c_int),
                ("palette_bits", ctypes.c_int)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class CsgvError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.csgv_last_error().decode(errors="replace")
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


_P, _U32, _U64, _I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_lib.csgv_last_error.restype = ctypes.c_char_p
_lib.csgv_volume_parse.argtypes = [_P, _U64, ctypes.POINTER(VolumeInfo)]
_lib.csgv_decode_bricks.argtypes = [_P, ctypes.POINTER(VolumeInfo), _P, _P, _P, _P, _U32, _P, _U64, _P,
                                    ctypes.POINTER(DecodeOpts)]
_lib.csgv_decode_bricks_noalloc.argtypes = _lib.csgv_decode_bricks.argtypes
_lib.csgv_check_status.argtypes = [_P, _U32, _P]
_lib.csgv_plan_create.argtypes = [ctypes.POINTER(VolumeInfo), _U32, ctypes.POINTER(DecodeOpts), ctypes.POINTER(_P)]
_lib.csgv_plan_launch.argtypes = [_P, _P, _P, _P, _P, _P, _U32, _P, _U64, _P]
_lib.csgv_plan_set_graph.argtypes = [_P, _I]
_lib.csgv_plan_set_timing.argtypes = [_P, _I]
_lib.csgv_plan_set_opts.argtypes = [_P, ctypes.POINTER(DecodeOpts)]
_lib.csgv_plan_get_opts.argtypes = [_P, ctypes.POINTER(DecodeOpts)]
_lib.csgv_plan_last_kernel_ms.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
_lib.csgv_plan_destroy.argtypes = [_P]


class TuneReport(ctypes.Structure):
    _fields_ = [("from_cache", ctypes.c_int), ("tried", ctypes.c_int), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float), ("chosen", DecodeOpts)]


_lib.csgv_plan_autotune.argtypes = [_P, _P, _P, _P, _P, _P, _U32, _P, _U64, _P, ctypes.c_char_p,
                                    ctypes.POINTER(TuneReport)]
_lib.csgv_encode_bricks.argtypes = [_P, _P, _U32, _U32, _P, _U32, _P, _P, _U32, _U32, _U32, _U32, _I,
                                    ctypes.POINTER(_P), ctypes.POINTER(_U64)]
_lib.csgv_free_host.argtypes = [_P]
_lib.csgv_encoder_create.argtypes = [_U32, _P, _U32, _P, _I, _U32, _U32, _U32, _U32, _I, ctypes.POINTER(_P)]
_lib.csgv_encoder_add.argtypes = [_P, _P, _P, _U32, _P]
_lib.csgv_encoder_finish.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(_U64)]
_lib.csgv_encoder_destroy.argtypes = [_P]

EXPORTED = [
    "csgv_volume_parse", "csgv_decode_bricks", "csgv_decode_bricks_noalloc", "csgv_check_status", "csgv_plan_create",
    "csgv_plan_launch",
    "csgv_plan_set_graph", "csgv_plan_set_timing", "csgv_plan_set_opts", "csgv_plan_get_opts",
    "csgv_plan_last_kernel_ms", "csgv_plan_destroy", "csgv_plan_autotune", "csgv_encode_bricks", "csgv_free_host", "csgv_last_error",
    "csgv_encoder_create", "csgv_encoder_add", "csgv_encoder_finish", "csgv_encoder_destroy",
]


def _check(rc: int, where: str):
    if rc != CSGV_OK:
        raise CsgvError(rc, where)


def _ptr(x) -> int | None:
    """Device/host address of a torch tensor, numpy array or int (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError("cannot take the address of %r" % type(x))


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def csgv_volume_parse(container) -> VolumeInfo:
    """Header of a container held in host memory (bytes or uint8 numpy array)."""
    buf = np.frombuffer(container, dtype=np.uint8) if isinstance(container, (bytes, bytearray)) else container
    info = VolumeInfo()
    _check(_lib.csgv_volume_parse(buf.ctypes.data, buf.nbytes, ctypes.byref(info)), "csgv_volume_parse")
    return info


def _opts(mode=None, wg_size=0, wgs_per_cu=0, sort_tasks=-1, bricks_per_wave=0, lds_slots=0, palette_bits=0):
    if mode is None and not palette_bits:
        return None
    return DecodeOpts(MODE_PLAIN if mode is None else mode, wg_size, wgs_per_cu, sort_tasks, bricks_per_wave,
                      lds_slots, palette_bits)


def csgv_decode_bricks(stream, vol: VolumeInfo, d_container, d_brick_ids, d_lods, d_out_offsets, n: int, d_out,
                       out_capacity: int, d_status=None, mode=None, wg_size=0, wgs_per_cu=0, sort_tasks=-1,
                       bricks_per_wave=0, lds_slots=0, palette_bits=0):
    o = _opts(mode, wg_size, wgs_per_cu, sort_tasks, bricks_per_wave, lds_slots, palette_bits)
    rc = _lib.csgv_decode_bricks(_stream(stream), ctypes.byref(vol), _ptr(d_container), _ptr(d_brick_ids),
                                 _ptr(d_lods), _ptr(d_out_offsets), n, _ptr(d_out), out_capacity, _ptr(d_status),
                                 None if o is None else ctypes.byref(o))
    _check(rc, "csgv_decode_bricks")


def csgv_decode_bricks_noalloc(stream, vol: VolumeInfo, d_container, d_brick_ids, d_lods, d_out_offsets, n: int,
                               d_out, out_capacity: int, d_status=None, mode=None, wg_size=0, wgs_per_cu=0,
                               sort_tasks=-1, bricks_per_wave=0, lds_slots=0, palette_bits=0):
    """csgv_decode_bricks on the library's fixed scratch (no allocation; calls on one GPU must not overlap)."""
    o = _opts(mode, wg_size, wgs_per_cu, sort_tasks, bricks_per_wave, lds_slots, palette_bits)
    rc = _lib.csgv_decode_bricks_noalloc(_stream(stream), ctypes.byref(vol), _ptr(d_container), _ptr(d_brick_ids),
                                         _ptr(d_lods), _ptr(d_out_offsets), n, _ptr(d_out), out_capacity,
                                         _ptr(d_status), None if o is None else ctypes.byref(o))
    _check(rc, "csgv_decode_bricks_noalloc")


def palette_bits_for(max_palette: int) -> int:
    """Index width that fits every brick of a volume: max(1, ceil(log2(max_palette)))."""
    return max(1, int(max(int(max_palette), 1) - 1).bit_length())


def paletted_words(voxels, bits: int):
    """32-bit words of a cube of `voxels` packed palette indices (CSGV_PALETTED_WORDS)."""
    e = 32 // bits
    return (np.asarray(voxels, dtype=np.int64) + e - 1) // e


def csgv_check_status(d_status, n: int, stream=None) -> bool:
    rc = _lib.csgv_check_status(_ptr(d_status), n, _stream(stream))
    if rc == CSGV_ECORRUPT:
        return False
    _check(rc, "csgv_check_status")
    return True


class csgv_plan:
    """Owner of a csgv_plan* (csgv_plan_create / csgv_plan_destroy)."""

    def __init__(self, vol: VolumeInfo, max_tasks: int, wg_size: int = 0, wgs_per_cu: int = 0, sort_tasks: int = -1,
                 bricks_per_wave: int = 0, lds_slots: int = 0, palette_bits: int = 0):
        self._vol = vol
        self._h = ctypes.c_void_p()
        o = DecodeOpts(MODE_PERSISTENT, wg_size, wgs_per_cu, sort_tasks, bricks_per_wave, lds_slots, palette_bits)
        _check(_lib.csgv_plan_create(ctypes.byref(vol), max_tasks, ctypes.byref(o), ctypes.byref(self._h)),
               "csgv_plan_create")

    def launch(self, stream, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity, d_status=None):
        rc = _lib.csgv_plan_launch(self._h, _stream(stream), _ptr(d_container), _ptr(d_brick_ids), _ptr(d_lods),
                                   _ptr(d_out_offsets), n, _ptr(d_out), out_capacity, _ptr(d_status))
        _check(rc, "csgv_plan_launch")

    def set_graph(self, enable: bool):
        _check(_lib.csgv_plan_set_graph(self._h, int(enable)), "csgv_plan_set_graph")

    def set_timing(self, enable: bool):
        _check(_lib.csgv_plan_set_timing(self._h, int(enable)), "csgv_plan_set_timing")

    def set_opts(self, wg_size: int = 0, wgs_per_cu: int = -1, sort_tasks: int = -1, bricks_per_wave: int = 0,
                 lds_slots: int = 0, palette_bits: int = -1):
        o = DecodeOpts(MODE_PERSISTENT, wg_size, wgs_per_cu, sort_tasks, bricks_per_wave, lds_slots, palette_bits)
        _check(_lib.csgv_plan_set_opts(self._h, ctypes.byref(o)), "csgv_plan_set_opts")

    def get_opts(self) -> DecodeOpts:
        o = DecodeOpts()
        _check(_lib.csgv_plan_get_opts(self._h, ctypes.byref(o)), "csgv_plan_get_opts")
        return o

    def autotune(self, stream, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity,
                 d_status=None, cache_path: str | None = None) -> TuneReport:
        rep = TuneReport()
        rc = _lib.csgv_plan_autotune(self._h, _stream(stream), _ptr(d_container), _ptr(d_brick_ids), _ptr(d_lods),
                                     _ptr(d_out_offsets), n, _ptr(d_out), out_capacity, _ptr(d_status),
                                     None if cache_path is None else cache_path.encode(), ctypes.byref(rep))
        _check(rc, "csgv_plan_autotune")
        return rep

    def last_kernel_ms(self) -> float:
        v = ctypes.c_float()
        _check(_lib.csgv_plan_last_kernel_ms(self._h, ctypes.byref(v)), "csgv_plan_last_kernel_ms")
        return float(v.value)

    def destroy(self):
        if self._h:
            _lib.csgv_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def csgv_encode_bricks(voxels: np.ndarray, log2b, label_bytes: int, dims=(0, 0, 0), default_log2b: int = 5,
                       grid=None, origins=None, op_mask: int = ALL_OPS, neighbor_mode: int = 0,
                       coder_policy: int = 0, lane_syms: int = 64, n_threads: int = 0) -> bytes:
    """CPU encoder: concatenated bricks (brick k = (2^log2b[k])^3 labels, x fastest) -> container bytes."""
    vox = np.ascontiguousarray(voxels, dtype=np.uint64 if label_bytes == 8 else np.uint32)
    l2 = np.ascontiguousarray(np.asarray(log2b, dtype=np.uint8))
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.uint32))
    g = None if grid is None else np.ascontiguousarray(np.asarray(grid, dtype=np.uint32))
    org = None if origins is None else np.ascontiguousarray(np.asarray(origins, dtype=np.uint32).reshape(-1))
    out = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    rc = _lib.csgv_encode_bricks(vox.ctypes.data, l2.ctypes.data, len(l2), label_bytes, d.ctypes.data, default_log2b,
                                 None if g is None else g.ctypes.data, None if org is None else org.ctypes.data,
                                 op_mask, neighbor_mode, coder_policy, lane_syms, n_threads, ctypes.byref(out),
                                 ctypes.byref(nbytes))
    _check(rc, "csgv_encode_bricks")
    try:
        return ctypes.string_at(out.value, nbytes.value)
    finally:
        _lib.csgv_free_host(out)


class csgv_encoder:
    """Streaming encoder (csgv_encoder_create / add / finish / destroy)."""

    def __init__(self, label_bytes: int, dims=(0, 0, 0), default_log2b: int = 5, grid=None, with_directory=False,
                 op_mask: int = ALL_OPS, neighbor_mode: int = 0, coder_policy: int = 0, lane_syms: int = 64,
                 n_threads: int = 0):
        self.label_bytes = label_bytes
        self._dims = np.ascontiguousarray(np.asarray(dims, dtype=np.uint32))
        self._grid = None if grid is None else np.ascontiguousarray(np.asarray(grid, dtype=np.uint32))
        self._h = ctypes.c_void_p()
        _check(_lib.csgv_encoder_create(label_bytes, self._dims.ctypes.data, default_log2b,
                                        None if self._grid is None else self._grid.ctypes.data, int(with_directory),
                                        op_mask, neighbor_mode, coder_policy, lane_syms, n_threads,
                                        ctypes.byref(self._h)), "csgv_encoder_create")

    def add(self, voxels: np.ndarray, log2b, origins=None):
        vox = np.ascontiguousarray(voxels, dtype=np.uint64 if self.label_bytes == 8 else np.uint32)
        l2 = np.ascontiguousarray(np.asarray(log2b, dtype=np.uint8))
        org = None if origins is None else np.ascontiguousarray(np.asarray(origins, dtype=np.uint32).reshape(-1))
        _check(_lib.csgv_encoder_add(self._h, vox.ctypes.data, l2.ctypes.data, len(l2),
                                     None if org is None else org.ctypes.data), "csgv_encoder_add")

    def finish(self) -> bytes:
        out = ctypes.c_void_p()
        nbytes = ctypes.c_uint64()
        _check(_lib.csgv_encoder_finish(self._h, ctypes.byref(out), ctypes.byref(nbytes)), "csgv_encoder_finish")
        try:
            return ctypes.string_at(out.value, nbytes.value)
        finally:
            _lib.csgv_free_host(out)

    def destroy(self):
        if self._h:
            _lib.csgv_encoder_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
class ServerConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int), ("max_batch", ctypes.c_uint32), ("keep_pinned", ctypes.c_int),
                ("shape", DecodeOpts), ("n_shards", ctypes.c_int)]


class RequestDone(ctypes.Structure):
    _fields_ = [("req", ctypes.c_uint64), ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("n_pairs", ctypes.c_uint32), ("n_decoded", ctypes.c_uint32),
                ("status", ctypes.c_int32)]


# numpy view of csgv_request_done (48 bytes: 4 bytes of tail padding)
REQUEST_DONE_DTYPE = np.dtype([("req", "<u8"), ("t_arrival", "<f8"), ("t_admit", "<f8"), ("t_done", "<f8"),
                               ("n_pairs", "<u4"), ("n_decoded", "<u4"), ("status", "<i4"), ("_pad", "<i4")])
assert REQUEST_DONE_DTYPE.itemsize == ctypes.sizeof(RequestDone)


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("requests_done", "pairs_requested", "hits", "joined", "decoded",
                                               "evictions", "resets", "batches", "decoded_elements",
                                               "requested_elements", "cache_top", "resident", "pinned",
                                               "failed_tasks", "splits", "record_bytes")] + \
        [("kernel_ms", ctypes.c_double), ("max_batch_seen", ctypes.c_uint32)]

    def as_dict(self):
        return {f: (float if f == "kernel_ms" else int)(getattr(self, f)) for f, _ in self._fields_}


_lib.csgv_server_create.argtypes = [ctypes.POINTER(VolumeInfo), _P, _P, _P, _U64, ctypes.POINTER(ServerConfig),
                                    ctypes.POINTER(_P)]
_lib.csgv_server_clock.argtypes = [_P]
_lib.csgv_server_clock.restype = ctypes.c_double
_lib.csgv_server_submit.argtypes = [_P, _P, _P, _U32, ctypes.c_double, ctypes.POINTER(_U64)]
_lib.csgv_server_step.argtypes = [_P, ctypes.POINTER(_I)]
_lib.csgv_server_drain.argtypes = [_P, ctypes.POINTER(RequestDone), _U32, ctypes.POINTER(_U32)]
_lib.csgv_server_release.argtypes = [_P, _U64]
_lib.csgv_server_where.argtypes = [_P, _U32, ctypes.c_uint8, ctypes.POINTER(_U64)]
_lib.csgv_server_run.argtypes = [_P, _P, _P, _P, _U32, _P, ctypes.POINTER(RequestDone)]
_lib.csgv_server_get_stats.argtypes = [_P, ctypes.POINTER(ServerStats)]
_lib.csgv_server_last_error.restype = ctypes.c_char_p
_lib.csgv_server_destroy.argtypes = [_P]
EXPORTED += ["csgv_server_create", "csgv_server_clock", "csgv_server_submit", "csgv_server_step", "csgv_server_drain",
             "csgv_server_release", "csgv_server_where", "csgv_server_run", "csgv_server_get_stats",
             "csgv_server_last_error", "csgv_server_destroy"]


def _scheck(rc: int, where: str):
    if rc != CSGV_OK:
        msg = _lib.csgv_server_last_error().decode(errors="replace")
        err = CsgvError(rc, where)
        err.args = ("%s failed (%d): %s" % (where, rc, msg),)
        raise err


class csgv_server:
    """Owner of a csgv_server* (served decode with a brick cache in d_cache)."""

    def __init__(self, vol: VolumeInfo, d_container, d_cache, cache_elements: int, brick_log2b=None,
                 n_streams: int = 2, max_batch: int = 4096, keep_pinned: bool = False, wg_size: int = 0,
                 lds_slots: int = 0, sort_tasks: int = -1, n_shards: int = 1):
        self._h = ctypes.c_void_p()
        self._l2 = None if brick_log2b is None else np.ascontiguousarray(np.asarray(brick_log2b, dtype=np.uint8))
        cfg = ServerConfig(n_streams, max_batch, int(keep_pinned),
                           DecodeOpts(MODE_PERSISTENT, wg_size, 0, sort_tasks, 0, lds_slots, 0), n_shards)
        _scheck(_lib.csgv_server_create(ctypes.byref(vol), _ptr(d_container),
                                        None if self._l2 is None else self._l2.ctypes.data, _ptr(d_cache),
                                        cache_elements, ctypes.byref(cfg), ctypes.byref(self._h)),
                "csgv_server_create")

    def clock(self) -> float:
        return float(_lib.csgv_server_clock(self._h))

    def submit(self, ids, lods, t_arrival: float) -> int:
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        lods = np.ascontiguousarray(np.asarray(lods, dtype=np.uint8))
        req = ctypes.c_uint64()
        _scheck(_lib.csgv_server_submit(self._h, ids.ctypes.data, lods.ctypes.data, len(ids), t_arrival,
                                        ctypes.byref(req)), "csgv_server_submit")
        return int(req.value)

    def step(self) -> bool:
        busy = ctypes.c_int()
        _scheck(_lib.csgv_server_step(self._h, ctypes.byref(busy)), "csgv_server_step")
        return bool(busy.value)

    def drain(self, cap: int = 4096):
        buf = (RequestDone * cap)()
        n = ctypes.c_uint32()
        _scheck(_lib.csgv_server_drain(self._h, buf, cap, ctypes.byref(n)), "csgv_server_drain")
        return [buf[i] for i in range(n.value)]

    def release(self, req: int):
        _scheck(_lib.csgv_server_release(self._h, req), "csgv_server_release")

    def where(self, brick_id: int, lod: int) -> int:
        off = ctypes.c_uint64()
        _scheck(_lib.csgv_server_where(self._h, brick_id, lod, ctypes.byref(off)), "csgv_server_where")
        return int(off.value)

    def run(self, ids, lods, starts, arrivals):
        """Serve a whole trace; returns a structured array of per-request records."""
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        lods = np.ascontiguousarray(np.asarray(lods, dtype=np.uint8))
        starts = np.ascontiguousarray(np.asarray(starts, dtype=np.uint64))
        arrivals = np.ascontiguousarray(np.asarray(arrivals, dtype=np.float64))
        n = len(starts) - 1
        rec = np.zeros(max(n, 1), dtype=REQUEST_DONE_DTYPE)
        out = ctypes.cast(rec.ctypes.data, ctypes.POINTER(RequestDone))
        _scheck(_lib.csgv_server_run(self._h, ids.ctypes.data, lods.ctypes.data, starts.ctypes.data, n,
                                     arrivals.ctypes.data, out), "csgv_server_run")
        return rec[:n]

    def stats(self) -> dict:
        s = ServerStats()
        _scheck(_lib.csgv_server_get_stats(self._h, ctypes.byref(s)), "csgv_server_get_stats")
        return s.as_dict()

    def destroy(self):
        if self._h:
            _lib.csgv_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------- device-resident cache stages
DC_NEW, DC_HIT, DC_JOINED, DC_FULL, DC_INVALID = 0, 1, 2, 3, 4
DC_NO_TASK = 0xFFFFFFFF
DC_NO_SLOT = 0xFFFFFFFFFFFFFFFF

_lib.csgv_dcache_create.argtypes = [ctypes.POINTER(VolumeInfo), _P, _U64, _U32, _P, ctypes.POINTER(_P)]
_lib.csgv_dcache_request.argtypes = [_P, _P, _P, _P, _U32, _P, _P, _P]
_lib.csgv_dcache_free.argtypes = [_P, _P, _P, _P, _U32]
_lib.csgv_dcache_reset.argtypes = [_P, _P]
_lib.csgv_dcache_query.argtypes = [_P, _P, _P, _P]
_lib.csgv_dcache_last_error.restype = ctypes.c_char_p
_lib.csgv_dcache_destroy.argtypes = [_P]
EXPORTED += ["csgv_dcache_create", "csgv_dcache_request", "csgv_dcache_free", "csgv_dcache_reset",
             "csgv_dcache_query", "csgv_dcache_last_error", "csgv_dcache_destroy"]


def _dcheck(rc: int, where: str):
    if rc != CSGV_OK:
        msg = _lib.csgv_dcache_last_error().decode(errors="replace")
        err = CsgvError(rc, where)
        err.args = ("%s failed (%d): %s" % (where, rc, msg),)
        raise err


class csgv_dcache:
    """Owner of a csgv_dcache* (slot table, free stacks and cache top on the device)."""

    def __init__(self, vol: VolumeInfo, d_container, cache_elements: int, stack_cap: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        _dcheck(_lib.csgv_dcache_create(ctypes.byref(vol), _ptr(d_container), cache_elements, stack_cap,
                                        _stream(stream), ctypes.byref(self._h)), "csgv_dcache_create")

    def request(self, stream, d_ids, d_lods, n: int, d_task_ids, d_slot, d_state):
        _dcheck(_lib.csgv_dcache_request(self._h, _stream(stream), _ptr(d_ids), _ptr(d_lods), n, _ptr(d_task_ids),
                                         _ptr(d_slot), _ptr(d_state)), "csgv_dcache_request")

    def free(self, stream, d_ids, d_lods, n: int):
        _dcheck(_lib.csgv_dcache_free(self._h, _stream(stream), _ptr(d_ids), _ptr(d_lods), n), "csgv_dcache_free")

    def reset(self, stream=None):
        _dcheck(_lib.csgv_dcache_reset(self._h, _stream(stream)), "csgv_dcache_reset")

    def query(self, stream=None):
        """(top in elements, free-stack counts per size class); synchronizes the stream."""
        top = np.zeros(1, np.uint64)
        counts = np.zeros(7, np.int32)
        _dcheck(_lib.csgv_dcache_query(self._h, _stream(stream), top.ctypes.data, counts.ctypes.data),
                "csgv_dcache_query")
        return int(top[0]), counts

    def destroy(self):
        if self._h:
            _lib.csgv_dcache_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
