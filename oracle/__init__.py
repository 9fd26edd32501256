"""CPU oracle for hash-based sector carving -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg
may import this package. It shares no code with the GPU library
(`paper_0901_1307_amd`), and neither imports the other.

`carve_oracle.c` is the plain C implementation (djb2 of Eq. (1) with the 64-bit
accumulator of Section 4, or the 64-bit CRC of Section 2.1 read as
CRC-64/GO-ISO and computed bit by bit; per-cluster-position membership of
Section 3.1 via a sorted array and bisection, byte-for-byte confirmation of
Section 3.1, and a brute-force all-pairs byte comparison). `spec.py` holds
pure-Python forms of the signatures used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "carve_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
SECTOR = 512

MATCH_DTYPE = np.dtype([("disk_sector", "<u8"), ("file_id", "<u4"), ("sector_in_file", "<u4")])
SIG_DJB2, SIG_CRC64_GO_ISO = 0, 1


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (plain C, -O2, pthreads)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                    src, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    P, U64, U32, I32, I64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int64
    lib.oracle_djb2.restype = U64
    lib.oracle_djb2.argtypes = [P, U64]
    lib.oracle_sector_signatures.restype = None
    lib.oracle_sector_signatures.argtypes = [P, U64, P, I32]
    lib.oracle_build.restype = P
    lib.oracle_build.argtypes = [P, P, U32, I32]
    if hasattr(lib, "oracle_crc64"):   # copies of an older source (mutation tests) may lack it
        lib.oracle_crc64.restype = U64
        lib.oracle_crc64.argtypes = [P, U64]
        lib.oracle_sector_signatures_kind.restype = None
        lib.oracle_sector_signatures_kind.argtypes = [P, U64, P, I32, I32]
        lib.oracle_build_kind.restype = P
        lib.oracle_build_kind.argtypes = [P, P, U32, I32, I32]
    if hasattr(lib, "oracle_build_fragments"):
        lib.oracle_build_fragments.restype = P
        lib.oracle_build_fragments.argtypes = [P, P, U32, I32]
        lib.oracle_fragment_flags.restype = I64
        lib.oracle_fragment_flags.argtypes = [P, P, U64, P, U64, I32]
        lib.oracle_fragment_confirm.restype = I64
        lib.oracle_fragment_confirm.argtypes = [P, P, P, U64, P, U64]
        lib.oracle_fragment_bruteforce.restype = I64
        lib.oracle_fragment_bruteforce.argtypes = [P, U64, P, P, U32, P, U64]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [P]
    lib.oracle_index_size.restype = U64
    lib.oracle_index_size.argtypes = [P]
    lib.oracle_flag_sectors.restype = None
    lib.oracle_flag_sectors.argtypes = [P, P, P, U64, U32, I32, P, I32]
    lib.oracle_flag_image.restype = I64
    lib.oracle_flag_image.argtypes = [P, P, U64, U32, I32, P, U64, I32]
    lib.oracle_confirm.restype = I64
    lib.oracle_confirm.argtypes = [P, P, P, U64, U32, I32, P, U64]
    lib.oracle_bruteforce.restype = I64
    lib.oracle_bruteforce.argtypes = [P, U64, P, P, U32, U32, I32, P, U64, I32]
    return lib


_lib = None


def load(path: str = _LIB) -> ctypes.CDLL:
    """Load the compiled oracle, compiling it first only if it is not built."""
    global _lib
    if path != _LIB:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def default_threads() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def _u8(a) -> np.ndarray:
    if hasattr(a, "numpy"):
        a = a.detach().cpu().numpy()
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def djb2(data, lib=None) -> int:
    b = _u8(data).reshape(-1)
    return int((lib or load()).oracle_djb2(_ptr(b), b.size))


def crc64(data, lib=None) -> int:
    b = _u8(data).reshape(-1)
    return int((lib or load()).oracle_crc64(_ptr(b), b.size))


def sector_signatures(sectors, threads: int = 1, lib=None, sig_kind: int = SIG_DJB2) -> np.ndarray:
    s = _u8(sectors).reshape(-1)
    n = s.size // SECTOR
    out = np.empty(n, dtype=np.uint64)
    lib = lib or load()
    if sig_kind == SIG_DJB2:
        lib.oracle_sector_signatures(_ptr(s), n, _ptr(out), threads)
    else:
        lib.oracle_sector_signatures_kind(_ptr(s), n, _ptr(out), threads, sig_kind)
    return out


def pack_files(files: Sequence[bytes]) -> Tuple[np.ndarray, List[int]]:
    """Packed full sectors of each file and the CSR of their ranges.

    A file contributes floor(len/512) sectors; a trailing partial sector is not
    a sector of the file (Section 2: files of interest are stored on whole,
    512-byte aligned sectors)."""
    parts, offsets = [], [0]
    for f in files:
        b = _u8(f).reshape(-1)
        n = b.size // SECTOR
        parts.append(b[:n * SECTOR])
        offsets.append(offsets[-1] + n)
    data = np.concatenate(parts) if parts else np.empty(0, np.uint8)
    return data.reshape(-1, SECTOR), offsets


class Index:
    """Sorted (signature, master) entries of a packed master set."""

    def __init__(self, masters, file_offsets: Sequence[int], threads: int = 1, lib=None, sig_kind: int = SIG_DJB2):
        self.lib = lib or load()
        self.masters = _u8(masters).reshape(-1)
        self.offsets = np.ascontiguousarray(file_offsets, dtype=np.uint64)
        assert self.masters.size == int(self.offsets[-1]) * SECTOR
        self.n_files = len(file_offsets) - 1
        self.sig_kind = sig_kind
        if sig_kind == SIG_DJB2:
            self.h = self.lib.oracle_build(_ptr(self.masters), _ptr(self.offsets), self.n_files, threads)
        else:
            self.h = self.lib.oracle_build_kind(_ptr(self.masters), _ptr(self.offsets), self.n_files, threads,
                                                sig_kind)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h:
            self.lib.oracle_free(h)

    def __len__(self):
        return int(self.lib.oracle_index_size(self.h))

    def flag_image(self, image, tau0: int = 0, any_tau: bool = False, threads: int = 1) -> np.ndarray:
        img = _u8(image).reshape(-1)
        n = img.size // SECTOR
        out = np.empty(max(n, 1), dtype=np.uint64)
        cnt = self.lib.oracle_flag_image(self.h, _ptr(img), img.size, tau0, int(any_tau), _ptr(out), n, threads)
        return out[:cnt].copy()

    def flag_sectors(self, sectors, ids, tau0: int = 0, any_tau: bool = False, threads: int = 1) -> np.ndarray:
        s = _u8(sectors).reshape(-1)
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        assert s.size == ids.size * SECTOR
        flag = np.zeros(ids.size, dtype=np.uint8)
        self.lib.oracle_flag_sectors(self.h, _ptr(s), _ptr(ids), ids.size, tau0, int(any_tau), _ptr(flag), threads)
        return flag.astype(bool)

    def confirm(self, sectors, ids, tau0: int = 0, any_tau: bool = False) -> np.ndarray:
        s = _u8(sectors).reshape(-1)
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        assert s.size == ids.size * SECTOR
        args = (self.h, _ptr(s), _ptr(ids), ids.size, tau0, int(any_tau))
        out = np.zeros(4 * ids.size + 1024, dtype=MATCH_DTYPE)
        cnt = self.lib.oracle_confirm(*args, _ptr(out), out.size)
        if cnt > out.size:
            out = np.zeros(cnt, dtype=MATCH_DTYPE)
            self.lib.oracle_confirm(*args, _ptr(out), cnt)
        return out[:cnt].copy()

    def confirm_image(self, image, flagged, tau0: int = 0, any_tau: bool = False) -> np.ndarray:
        img = _u8(image).reshape(-1)
        ids = np.ascontiguousarray(flagged, dtype=np.uint64)
        secs = img[:(img.size // SECTOR) * SECTOR].reshape(-1, SECTOR)[ids.astype(np.int64)]
        return self.confirm(secs, ids, tau0, any_tau)


def bruteforce(image, masters, file_offsets, tau0: int = 0, any_tau: bool = False,
               threads: int = 1, lib=None) -> np.ndarray:
    lib = lib or load()
    img = _u8(image).reshape(-1)
    m = _u8(masters).reshape(-1)
    off = np.ascontiguousarray(file_offsets, dtype=np.uint64)
    args = (_ptr(img), img.size, _ptr(m), _ptr(off), len(file_offsets) - 1, tau0, int(any_tau))
    out = np.zeros(4 * (img.size // SECTOR) + 1024, dtype=MATCH_DTYPE)
    cnt = lib.oracle_bruteforce(*args, _ptr(out), out.size, threads)
    if cnt > out.size:
        out = np.zeros(cnt, dtype=MATCH_DTYPE)
        lib.oracle_bruteforce(*args, _ptr(out), cnt, threads)
    return out[:cnt].copy()


# ------------------------------------------------------ fragments (Section 5)
FRAGMENT = 64
STRIDE = 4


def n_windows(n_bytes: int) -> int:
    return 0 if n_bytes < FRAGMENT else (n_bytes - FRAGMENT) // STRIDE + 1


def pack_fragment_files(files: Sequence[bytes]) -> Tuple[np.ndarray, List[int]]:
    """Packed whole 64-byte fragments of each file and the CSR of their ranges
    (a trailing partial fragment is not a fragment)."""
    parts, offsets = [], [0]
    for f in files:
        b = _u8(f).reshape(-1)
        n = b.size // FRAGMENT
        parts.append(b[:n * FRAGMENT])
        offsets.append(offsets[-1] + n)
    data = np.concatenate(parts) if parts else np.empty(0, np.uint8)
    return data.reshape(-1, FRAGMENT), offsets


class FragmentIndex:
    """Sorted (signature, fragment) entries of packed master fragments."""

    def __init__(self, fragments, file_offsets: Sequence[int], threads: int = 1, lib=None):
        self.lib = lib or load()
        self.fragments = _u8(fragments).reshape(-1)
        self.offsets = np.ascontiguousarray(file_offsets, dtype=np.uint64)
        assert self.fragments.size == int(self.offsets[-1]) * FRAGMENT
        self.n_files = len(file_offsets) - 1
        self.h = self.lib.oracle_build_fragments(_ptr(self.fragments), _ptr(self.offsets), self.n_files, threads)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h:
            self.lib.oracle_free(h)

    def flag_windows(self, image, threads: int = 1) -> np.ndarray:
        img = _u8(image).reshape(-1)
        out = np.zeros(max(n_windows(img.size), 1), dtype=np.uint64)
        cnt = self.lib.oracle_fragment_flags(self.h, _ptr(img), img.size, _ptr(out), out.size, threads)
        return out[:cnt].copy()

    def confirm_windows(self, image, flagged) -> np.ndarray:
        img = _u8(image).reshape(-1)
        ids = np.ascontiguousarray(flagged, dtype=np.uint64)
        out = np.zeros(4 * ids.size + 1024, dtype=MATCH_DTYPE)
        args = (self.h, _ptr(img), _ptr(ids), ids.size)
        cnt = self.lib.oracle_fragment_confirm(*args, _ptr(out), out.size)
        if cnt > out.size:
            out = np.zeros(cnt, dtype=MATCH_DTYPE)
            self.lib.oracle_fragment_confirm(*args, _ptr(out), cnt)
        return out[:cnt].copy()


def fragment_bruteforce(image, fragments, file_offsets, lib=None) -> np.ndarray:
    lib = lib or load()
    img = _u8(image).reshape(-1)
    m = _u8(fragments).reshape(-1)
    off = np.ascontiguousarray(file_offsets, dtype=np.uint64)
    args = (_ptr(img), img.size, _ptr(m), _ptr(off), len(file_offsets) - 1)
    out = np.zeros(4 * n_windows(img.size) + 1024, dtype=MATCH_DTYPE)
    cnt = lib.oracle_fragment_bruteforce(*args, _ptr(out), out.size)
    if cnt > out.size:
        out = np.zeros(cnt, dtype=MATCH_DTYPE)
        lib.oracle_fragment_bruteforce(*args, _ptr(out), cnt)
    return out[:cnt].copy()
