"""Python binding of the carving library's C ABI (include/carve.h).

Argument marshalling only: every step of the scan runs in the HIP kernels of
libcarve.so. torch provides device memory and the current HIP stream. There
is no CPU fallback: without the built library on a GPU, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcarve.so")
SECTOR = 512

CARVE_OK, CARVE_EINVAL, CARVE_ENOMEM, CARVE_ETRUNC, CARVE_EDEVICE, CARVE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CARVE_SIG_DJB2_64, CARVE_SIG_CRC64_ISO = 0, 1
CARVE_TAU_PER_CLUSTER, CARVE_TAU_ANY = 0, 1
CARVE_LAYOUT_BUCKETED, CARVE_LAYOUT_LINEAR, CARVE_LAYOUT_SORTED = 0, 1, 2
CARVE_SPLIT_AUTO, CARVE_SPLIT_OFF, CARVE_SPLIT_ON = 0, 1, 2

MATCH_DTYPE = np.dtype([("disk_sector", "<u8"), ("file_id", "<u4"), ("sector_in_file", "<u4")])
BATCH_MATCH_DTYPE = np.dtype([("disk_sector", "<u8"), ("file_id", "<u4"), ("sector_in_file", "<u4"),
                              ("image", "<u4"), ("reserved", "<u4")])
# carve_image_desc and carve_job_done as numpy records (bulk submission and polling)
IMAGE_DESC_DTYPE = np.dtype([("image", "<u8"), ("n_bytes", "<u8"), ("tau0", "<u4"), ("tau_mode", "<u4")])
JOB_DONE_DTYPE = np.dtype([("job_id", "<u8"), ("n_flagged", "<u8"), ("n_confirmed", "<u8"), ("status", "<i4"),
                           ("reserved", "<u4")])

EXPORTS = ("build_master_index", "scan_image", "flagged_sectors", "confirm_matches", "sector_signatures",
           "sector_signatures_kind", "index_stats", "index_set_scan_config", "index_get_scan_config",
           "autotune_scan", "scan_batch", "batch_flag_counts", "batch_flagged_sectors", "batch_confirm_matches",
           "scan_set_timing", "scan_kernel_ms", "scan_kernel_ms_recent", "confirm_enqueue", "batch_confirm_enqueue", "server_create",
           "server_submit", "server_submit_many", "server_poll", "server_job_flags", "server_job_matches",
           "server_release", "server_release_many", "server_stats", "server_free", "free_index", "free_scan",
           "free_batch", "carve_last_error", "build_fragment_index", "scan_fragments", "ingest_create",
           "ingest_scan", "ingest_flagged_sectors", "ingest_matches", "ingest_stats", "ingest_free",
           "scan_image_noalloc", "read_ceiling_probe", "autotune_index", "confirm_enqueue_to",
           "flagged_sectors_enqueue", "scan_counts", "server_fail_next_launches", "scan_wait_kernel")


class CarveError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"carve error {code}: {msg}")
        self.code = code


CARVE_BLOOM_OFF = 0xFFFFFFFF
CARVE_ALL_IMAGES = 0xFFFFFFFF
CARVE_NOT_CONFIRMED = 0xFFFFFFFFFFFFFFFF   # scan_counts: no confirmation ran after the latest scan


class _IndexParams(ctypes.Structure):
    _fields_ = [("sig_kind", ctypes.c_uint32), ("max_load", ctypes.c_float), ("bloom_bits_per_key", ctypes.c_uint32),
                ("layout", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 4)]


class _ScanConfig(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_uint32), ("tiles_per_chunk", ctypes.c_uint32),
                ("split", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _TuneSpace(ctypes.Structure):
    _fields_ = [("layouts", ctypes.c_uint32), ("n_bloom", ctypes.c_uint32), ("bloom_bits", ctypes.c_uint32 * 8),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("params", _IndexParams), ("config", _ScanConfig), ("kernel_ms", ctypes.c_float),
                ("candidates", ctypes.c_uint32), ("from_cache", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


CARVE_TUNE_NO_CACHE, CARVE_TUNE_CONTIGUOUS = 1, 2


class _ImageDesc(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("n_bytes", ctypes.c_uint64), ("tau0", ctypes.c_uint32),
                ("tau_mode", ctypes.c_uint32)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_uint32), ("max_jobs_per_batch", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("confirm", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 3)]


class _JobDone(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_uint64), ("n_flagged", ctypes.c_uint64), ("n_confirmed", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("queued_jobs", ctypes.c_uint64), ("running_jobs", ctypes.c_uint64), ("done_jobs", ctypes.c_uint64),
                ("in_flight_bytes", ctypes.c_uint64), ("batches_launched", ctypes.c_uint64),
                ("jobs_completed", ctypes.c_uint64), ("host_launch_s", ctypes.c_double),
                ("host_retire_s", ctypes.c_double)]


class _IngestParams(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_uint64), ("confirm", ctypes.c_uint32), ("copy_threads", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 4)]


class _IngestStats(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64), ("chunks", ctypes.c_uint64), ("seconds", ctypes.c_double),
                ("pinned_source", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _IndexStats(ctypes.Structure):
    _fields_ = [("n_master_sectors", ctypes.c_uint64), ("n_unique_signatures", ctypes.c_uint64),
                ("n_buckets", ctypes.c_uint64), ("n_overflow_keys", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("bloom_bytes", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """The compiled library; raises if it has not been built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_0901_1307_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, U64, U32, I32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    PU64 = ctypes.POINTER(ctypes.c_uint64)
    lib.build_master_index.restype = I32
    lib.build_master_index.argtypes = [P, P, U32, ctypes.POINTER(_IndexParams), P, PP]
    lib.scan_image.restype = I32
    lib.scan_image.argtypes = [P, P, U64, U32, U32, P, PP]
    lib.autotune_index.restype = I32
    lib.autotune_index.argtypes = [P, P, U32, ctypes.POINTER(_IndexParams), ctypes.POINTER(_TuneSpace), P, U64, P, PP,
                                   ctypes.POINTER(_TuneResult)]
    lib.read_ceiling_probe.restype = I32
    lib.read_ceiling_probe.argtypes = [P, U64, U32, U32, P, ctypes.POINTER(ctypes.c_float)]
    lib.scan_image_noalloc.restype = I32
    lib.scan_image_noalloc.argtypes = [P, P, U64, U32, U32, P, P, U64, P]
    lib.flagged_sectors.restype = I32
    lib.flagged_sectors.argtypes = [P, P, U64, PU64]
    lib.confirm_matches.restype = I32
    lib.confirm_matches.argtypes = [P, P, P, U64, PU64]
    lib.sector_signatures.restype = I32
    lib.sector_signatures.argtypes = [P, U64, P, P]
    lib.sector_signatures_kind.restype = I32
    lib.sector_signatures_kind.argtypes = [U32, P, U64, P, P]
    lib.ingest_create.restype = I32
    lib.ingest_create.argtypes = [P, ctypes.POINTER(_IngestParams), PP]
    lib.ingest_scan.restype = I32
    lib.ingest_scan.argtypes = [P, P, U64, U32, U32]
    lib.ingest_flagged_sectors.restype = I32
    lib.ingest_flagged_sectors.argtypes = [P, P, U64, PU64]
    lib.ingest_matches.restype = I32
    lib.ingest_matches.argtypes = [P, P, U64, PU64]
    lib.ingest_stats.restype = I32
    lib.ingest_stats.argtypes = [P, ctypes.POINTER(_IngestStats)]
    lib.ingest_free.restype = None
    lib.ingest_free.argtypes = [P]
    lib.build_fragment_index.restype = I32
    lib.build_fragment_index.argtypes = [P, P, U32, ctypes.POINTER(_IndexParams), P, PP]
    lib.scan_fragments.restype = I32
    lib.scan_fragments.argtypes = [P, P, U64, P, PP]
    lib.index_stats.restype = I32
    lib.index_stats.argtypes = [P, ctypes.POINTER(_IndexStats)]
    lib.index_set_scan_config.restype = I32
    lib.index_set_scan_config.argtypes = [P, ctypes.POINTER(_ScanConfig)]
    lib.index_get_scan_config.restype = I32
    lib.index_get_scan_config.argtypes = [P, ctypes.POINTER(_ScanConfig)]
    lib.autotune_scan.restype = I32
    lib.autotune_scan.argtypes = [P, P, U64, P, ctypes.POINTER(_ScanConfig)]
    lib.scan_batch.restype = I32
    lib.scan_batch.argtypes = [P, ctypes.POINTER(_ImageDesc), U32, P, PP]
    lib.batch_flag_counts.restype = I32
    lib.batch_flag_counts.argtypes = [P, P, U32]
    lib.batch_flagged_sectors.restype = I32
    lib.batch_flagged_sectors.argtypes = [P, U32, P, U64, PU64]
    lib.batch_confirm_matches.restype = I32
    lib.batch_confirm_matches.argtypes = [P, P, P, U64, PU64]
    lib.server_create.restype = I32
    lib.server_create.argtypes = [P, ctypes.POINTER(_ServerParams), PP]
    lib.server_submit.restype = I32
    lib.server_submit.argtypes = [P, ctypes.POINTER(_ImageDesc), PU64]
    lib.server_poll.restype = I32
    lib.server_poll.argtypes = [P, ctypes.POINTER(_JobDone), U32, ctypes.POINTER(ctypes.c_uint32)]
    lib.server_job_flags.restype = I32
    lib.server_job_flags.argtypes = [P, U64, P, U64, PU64]
    lib.server_job_matches.restype = I32
    lib.server_job_matches.argtypes = [P, U64, P, U64, PU64]
    lib.server_release.restype = I32
    lib.server_release.argtypes = [P, U64]
    lib.server_submit_many.restype = I32
    lib.server_submit_many.argtypes = [P, P, U32, P]
    lib.server_release_many.restype = I32
    lib.server_release_many.argtypes = [P, P, U32]
    lib.server_stats.restype = I32
    lib.server_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.server_fail_next_launches.restype = I32
    lib.server_fail_next_launches.argtypes = [P, U32]
    lib.scan_wait_kernel.restype = I32
    lib.scan_wait_kernel.argtypes = [P, P]
    lib.server_free.restype = None
    lib.server_free.argtypes = [P]
    lib.confirm_enqueue.restype = I32
    lib.confirm_enqueue.argtypes = [P, P]
    lib.batch_confirm_enqueue.restype = I32
    lib.batch_confirm_enqueue.argtypes = [P, P]
    lib.confirm_enqueue_to.restype = I32
    lib.confirm_enqueue_to.argtypes = [P, P, P, U64]
    lib.flagged_sectors_enqueue.restype = I32
    lib.flagged_sectors_enqueue.argtypes = [P, P, U64]
    lib.scan_counts.restype = I32
    lib.scan_counts.argtypes = [P, PU64, PU64]
    lib.free_batch.restype = None
    lib.free_batch.argtypes = [P]
    lib.scan_set_timing.restype = I32
    lib.scan_set_timing.argtypes = [P, I32]
    lib.scan_kernel_ms.restype = I32
    lib.scan_kernel_ms.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
    lib.scan_kernel_ms_recent.restype = I32
    lib.scan_kernel_ms_recent.argtypes = [P, ctypes.POINTER(ctypes.c_float), U32, ctypes.POINTER(ctypes.c_uint32)]
    lib.free_index.restype = None
    lib.free_index.argtypes = [P]
    lib.free_scan.restype = None
    lib.free_scan.argtypes = [P]
    lib.carve_last_error.restype = ctypes.c_char_p
    lib.carve_last_error.argtypes = []
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(rc: int, allow_trunc: bool = False) -> int:
    if rc == CARVE_OK or (allow_trunc and rc == CARVE_ETRUNC):
        return rc
    raise CarveError(rc, _lib.carve_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _u8_any(t: torch.Tensor, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type not in ("cuda", "cpu"):
        raise TypeError(f"{what} must be a GPU or host tensor")
    if t.dtype != torch.uint8 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous uint8 tensor")
    return t


def _dev_u8(t: torch.Tensor, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != torch.uint8 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous uint8 tensor")
    return t


class Index:
    """Resident master-signature index (owns the C handle, keeps the master bytes alive)."""

    def __init__(self, handle: int, masters: torch.Tensor, file_offsets: Sequence[int]):
        self.handle = handle
        self.masters = masters
        self.file_offsets = list(file_offsets)

    def stats(self) -> dict:
        st = _IndexStats()
        _check(load_library().index_stats(self.handle, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in _IndexStats._fields_}

    def scan_config(self) -> dict:
        c = _ScanConfig()
        _check(load_library().index_get_scan_config(self.handle, ctypes.byref(c)))
        return {"blocks_per_cu": int(c.blocks_per_cu), "tiles_per_chunk": int(c.tiles_per_chunk),
                "split": int(c.split)}

    def set_scan_config(self, blocks_per_cu: int = 0, tiles_per_chunk: int = 0, split: int = CARVE_SPLIT_AUTO):
        c = _ScanConfig(int(blocks_per_cu), int(tiles_per_chunk), int(split))
        _check(load_library().index_set_scan_config(self.handle, ctypes.byref(c)))

    def autotune(self, sample: torch.Tensor, stream=None) -> dict:
        """Time the candidate launch shapes on a sample image; keep the fastest."""
        img = _dev_u8(sample, "sample")
        c = _ScanConfig()
        _check(load_library().autotune_scan(self.handle, img.data_ptr(), img.numel(), _stream_ptr(stream),
                                            ctypes.byref(c)))
        return {"blocks_per_cu": int(c.blocks_per_cu), "tiles_per_chunk": int(c.tiles_per_chunk),
                "split": int(c.split)}

    def close(self):
        h, self.handle = self.handle, None
        if h:
            load_library().free_index(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scan:
    """Result buffers of a scan (owns the C handle, keeps the image alive)."""

    def __init__(self):
        self.handle = None
        self.image = None
        self.pending = []   # device outputs of enqueued work, kept alive until a synchronization

    def set_timing(self, enable: bool = True):
        _check(load_library().scan_set_timing(self.handle, int(enable)))

    def kernel_ms(self) -> float:
        ms = ctypes.c_float()
        _check(load_library().scan_kernel_ms(self.handle, ctypes.byref(ms)))
        return float(ms.value)

    def kernel_ms_recent(self, n: int) -> list:
        """Kernel durations (ms) of the last n timed launches, oldest first (one synchronization)."""
        buf = (ctypes.c_float * max(1, n))()
        got = ctypes.c_uint32()
        _check(load_library().scan_kernel_ms_recent(self.handle, buf, n, ctypes.byref(got)))
        return [float(buf[i]) for i in range(got.value)]

    def close(self):
        h, self.handle = self.handle, None
        if h:
            load_library().free_scan(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Result buffers of a batch scan (owns the C handle, keeps the images alive)."""

    def __init__(self):
        self.handle = None
        self.images = None

    def set_timing(self, enable: bool = True):
        _check(load_library().scan_set_timing(self.handle, int(enable)))

    def kernel_ms(self) -> float:
        ms = ctypes.c_float()
        _check(load_library().scan_kernel_ms(self.handle, ctypes.byref(ms)))
        return float(ms.value)

    def kernel_ms_recent(self, n: int) -> list:
        """Kernel durations (ms) of the last n timed launches, oldest first (one synchronization)."""
        buf = (ctypes.c_float * max(1, n))()
        got = ctypes.c_uint32()
        _check(load_library().scan_kernel_ms_recent(self.handle, buf, n, ctypes.byref(got)))
        return [float(buf[i]) for i in range(got.value)]

    def close(self):
        h, self.handle = self.handle, None
        if h:
            load_library().free_batch(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_master_index(master_sectors: torch.Tensor, file_sector_offsets: Sequence[int], max_load: float = 0.0,
                       bloom_bits_per_key: int = 0, stream=None, sig_kind: int = CARVE_SIG_DJB2_64,
                       layout: int = CARVE_LAYOUT_BUCKETED) -> Index:
    """Index of packed master sectors (uint8 device tensor, file after file).

    bloom_bits_per_key: 0 = automatic, CARVE_BLOOM_OFF = no prefilter.
    sig_kind: CARVE_SIG_DJB2_64 or CARVE_SIG_CRC64_ISO (every scan with this
    index uses the same signature). layout: CARVE_LAYOUT_BUCKETED, _LINEAR
    (the paper's Eq. (3) table) or _SORTED (binary search); max_load sizes the
    probed table."""
    lib = load_library()
    m = _dev_u8(master_sectors, "master_sectors")
    off = np.ascontiguousarray(file_sector_offsets, dtype=np.uint64)
    if off.size < 1:
        raise ValueError("file_sector_offsets needs at least one entry")
    if m.numel() != int(off[-1]) * SECTOR:
        raise ValueError("master_sectors size does not match file_sector_offsets[-1] sectors")
    p = _IndexParams(int(sig_kind), float(max_load), int(bloom_bits_per_key), int(layout))
    h = ctypes.c_void_p()
    _check(lib.build_master_index(m.data_ptr() if m.numel() else None, off.ctypes.data, off.size - 1,
                                  ctypes.byref(p), _stream_ptr(stream), ctypes.byref(h)))
    return Index(h.value, m, off.tolist())


def autotune_index(master_sectors: torch.Tensor, file_sector_offsets: Sequence[int], sample: torch.Tensor,
                   sig_kind: int = CARVE_SIG_DJB2_64, max_load: float = 0.0, layouts: int = 0, bloom_bits=(),
                   contiguous_only: bool = False, no_cache: bool = False, stream=None):
    """build_master_index with the layout, prefilter size and launch shape
    timed on a sample image (device tensor); returns (Index, pick) where pick
    names the chosen parameters."""
    lib = load_library()
    m = _dev_u8(master_sectors, "master_sectors")
    smp = _dev_u8(sample, "sample")
    off = np.ascontiguousarray(file_sector_offsets, dtype=np.uint64)
    if off.size < 1 or m.numel() != int(off[-1]) * SECTOR:
        raise ValueError("master_sectors size does not match file_sector_offsets[-1] sectors")
    base = _IndexParams(int(sig_kind), float(max_load), 0, 0)
    bb = list(bloom_bits)
    if len(bb) > 8:
        raise ValueError("at most 8 bloom_bits candidates")
    sp = _TuneSpace(int(layouts), len(bb), (ctypes.c_uint32 * 8)(*bb),
                    (CARVE_TUNE_CONTIGUOUS if contiguous_only else 0) | (CARVE_TUNE_NO_CACHE if no_cache else 0))
    h = ctypes.c_void_p()
    r = _TuneResult()
    _check(lib.autotune_index(m.data_ptr() if m.numel() else None, off.ctypes.data, off.size - 1, ctypes.byref(base),
                              ctypes.byref(sp), smp.data_ptr(), smp.numel(), _stream_ptr(stream), ctypes.byref(h),
                              ctypes.byref(r)))
    names = {CARVE_LAYOUT_BUCKETED: "bucketed", CARVE_LAYOUT_LINEAR: "linear", CARVE_LAYOUT_SORTED: "sorted"}
    bits = int(r.params.bloom_bits_per_key)
    pick = {"layout": names.get(int(r.params.layout), str(r.params.layout)),
            "bloom_bits_per_key": "auto" if bits == 0 else ("off" if bits == CARVE_BLOOM_OFF else bits),
            "blocks_per_cu": int(r.config.blocks_per_cu), "tiles_per_chunk": int(r.config.tiles_per_chunk),
            "split": {CARVE_SPLIT_AUTO: "auto", CARVE_SPLIT_OFF: "off", CARVE_SPLIT_ON: "on"}[int(r.config.split)],
            "kernel_ms_on_sample": round(float(r.kernel_ms), 4), "candidates": int(r.candidates),
            "from_cache": bool(r.from_cache)}
    return Index(h.value, m, off.tolist()), pick


def scan_image(index: Index, image: torch.Tensor, tau0: int = 0, tau_mode: int = CARVE_TAU_PER_CLUSTER,
               stream=None, scan: Optional[Scan] = None, n_bytes: Optional[int] = None) -> Scan:
    """Flag the sectors of a device-resident image (asynchronous on the stream)."""
    lib = load_library()
    img = _dev_u8(image, "image")
    nb = img.numel() if n_bytes is None else int(n_bytes)
    if nb > img.numel():
        raise ValueError("n_bytes exceeds the image tensor")
    sc = scan if scan is not None else Scan()
    h = ctypes.c_void_p(sc.handle)
    _check(lib.scan_image(index.handle, img.data_ptr() if nb else None, nb, tau0, tau_mode, _stream_ptr(stream),
                          ctypes.byref(h)))
    sc.handle = h.value
    sc.image = img
    sc.index = index
    return sc


def scan_image_noalloc(index: Index, image: torch.Tensor, ids: torch.Tensor, count: torch.Tensor, tau0: int = 0,
                       tau_mode: int = CARVE_TAU_PER_CLUSTER, stream=None, n_bytes: Optional[int] = None) -> None:
    """scan_image + flagged_sectors with no allocation (asynchronous): the
    ascending flagged ids into `ids` (int64 device tensor, the first
    ids.numel() of them) and their number into `count` (int64 device tensor,
    one element)."""
    lib = load_library()
    img = _dev_u8(image, "image")
    nb = img.numel() if n_bytes is None else int(n_bytes)
    if nb > img.numel():
        raise ValueError("n_bytes exceeds the image tensor")
    for t, what in ((ids, "ids"), (count, "count")):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.int64 or \
                not t.is_contiguous():
            raise TypeError(f"{what} must be a contiguous int64 CUDA (HIP) tensor")
    if count.numel() < 1:
        raise ValueError("count needs one element")
    _check(lib.scan_image_noalloc(index.handle, img.data_ptr() if nb else None, nb, tau0, tau_mode,
                                  _stream_ptr(stream), ids.data_ptr() if ids.numel() else None, ids.numel(),
                                  count.data_ptr()))


def read_ceiling_probe(image: torch.Tensor, split: bool = False, blocks_per_cu: int = 0, stream=None) -> float:
    """Duration (ms) of one streaming read of the image's whole sectors with a
    scan kernel's access pattern (contiguous, or split by cluster position)."""
    img = _dev_u8(image, "image")
    ms = ctypes.c_float()
    _check(load_library().read_ceiling_probe(img.data_ptr(), img.numel(), int(bool(split)), int(blocks_per_cu),
                                             _stream_ptr(stream), ctypes.byref(ms)))
    return float(ms.value)


FRAGMENT = 64      # bytes of a master fragment and of an image window
WINDOW_STRIDE = 4  # windows start on 4-byte boundaries


def build_fragment_index(master_fragments: torch.Tensor, file_fragment_offsets: Sequence[int], max_load: float = 0.0,
                         bloom_bits_per_key: int = 0, stream=None) -> Index:
    """Index of packed 64-byte master fragments (uint8 device tensor, file after
    file; see pack_fragment_files), for scan_fragments."""
    lib = load_library()
    m = _dev_u8(master_fragments, "master_fragments")
    off = np.ascontiguousarray(file_fragment_offsets, dtype=np.uint64)
    if off.size < 1:
        raise ValueError("file_fragment_offsets needs at least one entry")
    if m.numel() != int(off[-1]) * FRAGMENT:
        raise ValueError("master_fragments size does not match file_fragment_offsets[-1] fragments")
    p = _IndexParams(CARVE_SIG_DJB2_64, float(max_load), int(bloom_bits_per_key), CARVE_LAYOUT_BUCKETED)
    h = ctypes.c_void_p()
    _check(lib.build_fragment_index(m.data_ptr() if m.numel() else None, off.ctypes.data, off.size - 1,
                                    ctypes.byref(p), _stream_ptr(stream), ctypes.byref(h)))
    return Index(h.value, m, off.tolist())


def scan_fragments(index: Index, image: torch.Tensor, stream=None, scan: Optional[Scan] = None,
                   n_bytes: Optional[int] = None) -> Scan:
    """Flag every 64-byte window at a 4-byte boundary of a device-resident image;
    flagged_sectors then returns window ids (byte offset 4j) and
    confirm_matches the (window, file, fragment) records."""
    lib = load_library()
    img = _dev_u8(image, "image")
    nb = img.numel() if n_bytes is None else int(n_bytes)
    if nb > img.numel():
        raise ValueError("n_bytes exceeds the image tensor")
    sc = scan if scan is not None else Scan()
    h = ctypes.c_void_p(sc.handle)
    _check(lib.scan_fragments(index.handle, img.data_ptr() if nb else None, nb, _stream_ptr(stream),
                              ctypes.byref(h)))
    sc.handle = h.value
    sc.image = img
    sc.index = index
    return sc


def pack_fragment_files(files: Sequence[torch.Tensor]):
    """Whole 64-byte fragments of each file, packed file after file, and the
    CSR of their fragment ranges (a trailing partial fragment is not one)."""
    parts, offsets = [], [0]
    for f in files:
        n = f.numel() // FRAGMENT
        parts.append(f.reshape(-1)[:n * FRAGMENT])
        offsets.append(offsets[-1] + n)
    data = torch.cat(parts) if parts else torch.empty(0, dtype=torch.uint8)
    return data, offsets


def flagged_sectors(scan: Scan, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Ascending flagged sector ids as int64: into `out` (host or device) if
    given, else a new CPU tensor. Synchronizes the scan's stream."""
    lib = load_library()
    n = ctypes.c_uint64()
    if out is None:
        _check(lib.flagged_sectors(scan.handle, None, 0, ctypes.byref(n)), allow_trunc=True)
        out = torch.empty(int(n.value), dtype=torch.int64)
        if out.numel() == 0:
            return out
    if out.dtype != torch.int64 or not out.is_contiguous():
        raise TypeError("out must be a contiguous int64 tensor")
    rc = _check(lib.flagged_sectors(scan.handle, out.data_ptr() if out.numel() else None, out.numel(),
                                    ctypes.byref(n)), allow_trunc=True)
    if rc == CARVE_ETRUNC:
        raise CarveError(rc, f"{n.value} flagged sectors do not fit in {out.numel()}")
    return out[:int(n.value)]


def confirm_matches(index: Index, scan: Scan, out: Optional[torch.Tensor] = None):
    """Confirmed (disk_sector, file_id, sector_in_file) records.

    With out=None: a numpy structured array (host). With `out` (a contiguous
    uint8 tensor of 16*cap bytes, host or device): filled in place, and the
    number of records is returned."""
    lib = load_library()
    n = ctypes.c_uint64()
    if out is None:
        cap = 1 << 16
        while True:
            buf = np.zeros(cap, dtype=MATCH_DTYPE)
            rc = _check(lib.confirm_matches(index.handle, scan.handle, buf.ctypes.data, cap, ctypes.byref(n)),
                        allow_trunc=True)
            if rc == CARVE_OK:
                return buf[:int(n.value)].copy()
            cap = int(n.value)
    if out.dtype != torch.uint8 or not out.is_contiguous() or out.numel() % 16:
        raise TypeError("out must be a contiguous uint8 tensor of 16-byte records")
    cap = out.numel() // 16
    rc = _check(lib.confirm_matches(index.handle, scan.handle, out.data_ptr() if cap else None, cap,
                                    ctypes.byref(n)), allow_trunc=True)
    if rc == CARVE_ETRUNC:
        raise CarveError(rc, f"{n.value} matches do not fit in {cap}")
    return int(n.value)


def sector_signatures(sectors: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
                      sig_kind: int = CARVE_SIG_DJB2_64) -> torch.Tensor:
    """Signature (djb2-64 by default, or CRC-64) of each whole sector of a
    device tensor, as int64 (bit pattern of the uint64)."""
    lib = load_library()
    s = _dev_u8(sectors, "sectors")
    n = s.numel() // SECTOR
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=s.device)
    _check(lib.sector_signatures_kind(int(sig_kind), s.data_ptr() if n else None, n,
                                      out.data_ptr() if n else None, _stream_ptr(stream)))
    return out


def pack_master_files(files: Sequence[torch.Tensor]):
    """Whole sectors of each file, packed file after file, and the CSR of
    their sector ranges (a trailing partial sector is not a sector)."""
    parts, offsets = [], [0]
    for f in files:
        n = f.numel() // SECTOR
        parts.append(f.reshape(-1)[:n * SECTOR])
        offsets.append(offsets[-1] + n)
    data = torch.cat(parts) if parts else torch.empty(0, dtype=torch.uint8)
    return data, offsets


def scan_batch(index: Index, images: Sequence, stream=None, batch: Optional[Batch] = None) -> Batch:
    """Flag the sectors of many device-resident images in one launch.

    images: a sequence of uint8 device tensors, or of (tensor, tau0, tau_mode)."""
    lib = load_library()
    descs = (_ImageDesc * max(1, len(images)))()
    keep = []
    for i, it in enumerate(images):
        t, tau0, mode = (it, 0, CARVE_TAU_PER_CLUSTER) if isinstance(it, torch.Tensor) else it
        t = _dev_u8(t, f"images[{i}]")
        keep.append(t)
        descs[i] = _ImageDesc(t.data_ptr() if t.numel() else None, t.numel(), int(tau0), int(mode))
    b = batch if batch is not None else Batch()
    h = ctypes.c_void_p(b.handle)
    _check(lib.scan_batch(index.handle, descs, len(images), _stream_ptr(stream), ctypes.byref(h)))
    b.handle = h.value
    b.images = keep
    b.index = index
    return b


def batch_flag_counts(batch: Batch) -> np.ndarray:
    """Flagged sectors per image (synchronizes)."""
    n = len(batch.images)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    _check(load_library().batch_flag_counts(batch.handle, out.ctypes.data, n))
    return out[:n]


def batch_flagged_sectors(batch: Batch, image: int) -> torch.Tensor:
    """Ascending flagged sector ids of one image of the batch (CPU int64 tensor)."""
    lib = load_library()
    n = ctypes.c_uint64()
    _check(lib.batch_flagged_sectors(batch.handle, image, None, 0, ctypes.byref(n)), allow_trunc=True)
    out = torch.empty(int(n.value), dtype=torch.int64)
    if out.numel():
        _check(lib.batch_flagged_sectors(batch.handle, image, out.data_ptr(), out.numel(), ctypes.byref(n)))
    return out


def batch_confirm_matches(index: Index, batch: Batch, out: Optional[torch.Tensor] = None):
    """Confirmed matches of every image, ordered by (image, disk_sector, file_id,
    sector_in_file): a numpy structured array, or the count when `out` (a
    contiguous uint8 tensor of 24-byte records, host or device) is given."""
    lib = load_library()
    n = ctypes.c_uint64()
    rec = BATCH_MATCH_DTYPE.itemsize
    if out is None:
        cap = 1 << 16
        while True:
            buf = np.zeros(cap, dtype=BATCH_MATCH_DTYPE)
            rc = _check(lib.batch_confirm_matches(index.handle, batch.handle, buf.ctypes.data, cap, ctypes.byref(n)),
                        allow_trunc=True)
            if rc == CARVE_OK:
                return buf[:int(n.value)].copy()
            cap = int(n.value)
    if out.dtype != torch.uint8 or not out.is_contiguous() or out.numel() % rec:
        raise TypeError("out must be a contiguous uint8 tensor of 24-byte records")
    cap = out.numel() // rec
    rc = _check(lib.batch_confirm_matches(index.handle, batch.handle, out.data_ptr() if cap else None, cap,
                                          ctypes.byref(n)), allow_trunc=True)
    if rc == CARVE_ETRUNC:
        raise CarveError(rc, f"{n.value} matches do not fit in {cap}")
    return int(n.value)


class Server:
    """Continuous-batching request loop over one resident index (native runtime).

    submit() queues a job; poll() makes progress without blocking and returns
    the jobs completed since the last call as (job_id, n_flagged, n_confirmed,
    status) tuples; flags()/matches() fetch a completed job's results."""

    def __init__(self, index: Index, n_streams: int = 0, max_jobs_per_batch: int = 0, budget_bytes: int = 0,
                 confirm: bool = True):
        lib = load_library()
        p = _ServerParams(n_streams, max_jobs_per_batch, budget_bytes, int(confirm))
        h = ctypes.c_void_p()
        _check(lib.server_create(index.handle, ctypes.byref(p), ctypes.byref(h)))
        self.handle = h.value
        self.index = index
        self._keep = {}
        self._done = (_JobDone * 4096)()

    def submit(self, image: torch.Tensor, tau0: int = 0, tau_mode: int = CARVE_TAU_PER_CLUSTER) -> int:
        """image: a contiguous uint8 tensor on the GPU, or in host memory
        (pinned for an asynchronous copy)."""
        t = _u8_any(image, "image")
        d = _ImageDesc(t.data_ptr() if t.numel() else None, t.numel(), int(tau0), int(tau_mode))
        jid = ctypes.c_uint64()
        _check(load_library().server_submit(self.handle, ctypes.byref(d), ctypes.byref(jid)))
        self._keep[jid.value] = t
        return int(jid.value)

    def submit_many(self, descs: np.ndarray) -> np.ndarray:
        """Queue every row of an IMAGE_DESC_DTYPE array (see image_descs) in one
        call; returns the job ids. The caller keeps the images alive until the
        jobs are released."""
        descs = np.ascontiguousarray(descs, dtype=IMAGE_DESC_DTYPE)
        ids = np.empty(len(descs), dtype=np.uint64)
        _check(load_library().server_submit_many(self.handle, descs.ctypes.data, len(descs), ids.ctypes.data))
        return ids

    def poll(self):
        n = ctypes.c_uint32()
        _check(load_library().server_poll(self.handle, self._done, len(self._done), ctypes.byref(n)))
        return [(int(r.job_id), int(r.n_flagged), int(r.n_confirmed), int(r.status))
                for r in self._done[:n.value]]

    def poll_array(self) -> np.ndarray:
        """poll() as a JOB_DONE_DTYPE array."""
        n = ctypes.c_uint32()
        _check(load_library().server_poll(self.handle, self._done, len(self._done), ctypes.byref(n)))
        return np.frombuffer(self._done, dtype=JOB_DONE_DTYPE, count=n.value).copy()

    def flags(self, job_id: int) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_uint64()
        _check(lib.server_job_flags(self.handle, job_id, None, 0, ctypes.byref(n)), allow_trunc=True)
        out = np.zeros(int(n.value), dtype=np.uint64)
        if out.size:
            _check(lib.server_job_flags(self.handle, job_id, out.ctypes.data, out.size, ctypes.byref(n)))
        return out

    def matches(self, job_id: int) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_uint64()
        _check(lib.server_job_matches(self.handle, job_id, None, 0, ctypes.byref(n)), allow_trunc=True)
        out = np.zeros(int(n.value), dtype=MATCH_DTYPE)
        if out.size:
            _check(lib.server_job_matches(self.handle, job_id, out.ctypes.data, out.size, ctypes.byref(n)))
        return out

    def release(self, job_id: int):
        _check(load_library().server_release(self.handle, job_id))
        self._keep.pop(job_id, None)

    def release_many(self, job_ids) -> None:
        ids = np.ascontiguousarray(job_ids, dtype=np.uint64)
        _check(load_library().server_release_many(self.handle, ids.ctypes.data, len(ids)))
        if self._keep:
            for j in ids.tolist():
                self._keep.pop(j, None)

    def fail_next_launches(self, n: int) -> None:
        """Tests of the failure path: the next n batch launches fail after
        enqueuing their work (their jobs are reported with CARVE_EDEVICE)."""
        _check(load_library().server_fail_next_launches(self.handle, int(n)))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(load_library().server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        h, self.handle = self.handle, None
        if h:
            load_library().server_free(h)
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def image_descs(jobs) -> np.ndarray:
    """IMAGE_DESC_DTYPE array from (uint8 GPU or host tensor, tau0, tau_mode) tuples."""
    out = np.zeros(len(jobs), dtype=IMAGE_DESC_DTYPE)
    for i, (t, tau0, mode) in enumerate(jobs):
        t = _u8_any(t, "image")
        out[i] = (t.data_ptr() if t.numel() else 0, t.numel(), int(tau0), int(mode))
    return out


class Ingest:
    """Scans of images in host memory through a pair of device buffers (the
    paper's double-buffered pipeline); see include/carve.h."""

    def __init__(self, index: Index, chunk_bytes: int = 0, confirm: bool = True, copy_threads: int = 0):
        lib = load_library()
        p = _IngestParams(int(chunk_bytes), int(confirm), int(copy_threads))
        h = ctypes.c_void_p()
        _check(lib.ingest_create(index.handle, ctypes.byref(p), ctypes.byref(h)))
        self.handle = h.value
        self.index = index

    def scan(self, image: torch.Tensor, tau0: int = 0, tau_mode: int = CARVE_TAU_PER_CLUSTER) -> None:
        """image: a contiguous uint8 CPU tensor (pinned or pageable)."""
        if image.device.type != "cpu" or image.dtype != torch.uint8 or not image.is_contiguous():
            raise TypeError("image must be a contiguous uint8 CPU tensor")
        _check(load_library().ingest_scan(self.handle, image.data_ptr() if image.numel() else None, image.numel(),
                                          int(tau0), int(tau_mode)))

    def flagged(self) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_uint64()
        _check(lib.ingest_flagged_sectors(self.handle, None, 0, ctypes.byref(n)), allow_trunc=True)
        out = np.zeros(int(n.value), dtype=np.uint64)
        if out.size:
            _check(lib.ingest_flagged_sectors(self.handle, out.ctypes.data, out.size, ctypes.byref(n)))
        return out

    def matches(self) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_uint64()
        _check(lib.ingest_matches(self.handle, None, 0, ctypes.byref(n)), allow_trunc=True)
        out = np.zeros(int(n.value), dtype=MATCH_DTYPE)
        if out.size:
            _check(lib.ingest_matches(self.handle, out.ctypes.data, out.size, ctypes.byref(n)))
        return out

    def stats(self) -> dict:
        st = _IngestStats()
        _check(load_library().ingest_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _IngestStats._fields_ if k != "reserved"}

    def close(self):
        h, self.handle = self.handle, None
        if h:
            load_library().ingest_free(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def confirm_enqueue(index: Index, scan, out: Optional[torch.Tensor] = None) -> None:
    """Enqueue the confirmation of the last scan (or batch) without waiting.
    With `out` (a contiguous device uint8 tensor of 16*cap bytes; not for
    batches) the records go straight there (confirm_enqueue_to)."""
    lib = load_library()
    if isinstance(scan, Batch):
        if out is not None:
            raise TypeError("a batch confirms into its own buffer")
        _check(lib.batch_confirm_enqueue(index.handle, scan.handle))
    elif out is None:
        _check(lib.confirm_enqueue(index.handle, scan.handle))
    else:
        if out.dtype != torch.uint8 or not out.is_contiguous() or out.numel() % 16:
            raise TypeError("out must be a contiguous uint8 tensor of 16-byte records")
        cap = out.numel() // 16
        _check(lib.confirm_enqueue_to(index.handle, scan.handle, out.data_ptr() if cap else None, cap))
        scan.pending = [t for t in scan.pending if t is not out] + [out]   # alive until the stream has run


def flagged_sectors_enqueue(scan: Scan, out: torch.Tensor) -> None:
    """Enqueue the copy of the first min(count, out.numel()) flagged ids into
    `out` (a contiguous device int64 tensor) without waiting."""
    if out.dtype != torch.int64 or not out.is_contiguous():
        raise TypeError("out must be a contiguous int64 tensor")
    _check(load_library().flagged_sectors_enqueue(scan.handle, out.data_ptr() if out.numel() else None,
                                                  out.numel()))
    scan.pending = [t for t in scan.pending if t is not out] + [out]


def scan_wait_kernel(scan, stream=None) -> None:
    """Make `stream` (default: torch's current stream) wait for the scan
    object's latest scan kernel only, not its compaction and confirmation."""
    _check(load_library().scan_wait_kernel(scan.handle, _stream_ptr(stream)))


def scan_counts(scan) -> tuple:
    """(flagged units, confirmed records or None when no confirmation ran after
    the latest scan), read in one synchronization of the scan's stream."""
    nf, nm = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().scan_counts(scan.handle, ctypes.byref(nf), ctypes.byref(nm)))
    scan.pending = []
    return int(nf.value), (None if nm.value == CARVE_NOT_CONFIRMED else int(nm.value))
