"""Parity at the full workload sizes, through the C ABI, in the launch
configuration bench.py times: the index layout, prefilter size and launch
shape that autotune_index picks on a tuning sample (an image of the same
recipe that is not the scanned one, up to 8 GiB), one scan of the whole image. Every flag and every confirmed
record is compared with the CPU oracle over the whole image.

mid: 8 GiB image, 1,048,576 master sectors, one oracle pass.
large: 64 GiB image, 16,777,216 master sectors, in 1 GiB host chunks. A
chunk starting at sector s is flagged by the oracle with tau0 = s mod 8: under
Section 3.1's rule a sector's flag and its matches depend only on its own
bytes and its cluster position, so the chunks' results, shifted by s, are the
whole image's."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512
CHUNK = 1 << 21           # sectors per oracle chunk (1 GiB)


def _log(*a):
    print(*a, flush=True)


def _planted_ids(img) -> np.ndarray:
    ids = []
    for c, r in zip(img.planted_clusters.tolist(), img.planted_overwrite.tolist()):
        ids.extend(range(8 * c + r, 8 * c + 8))
    return np.asarray(ids, dtype=np.int64)


def oracle_chunked(ox, data, n_sectors: int, threads: int, tau0: int = 0, any_tau: bool = False,
                   chunk: int = CHUNK):
    """The oracle's flags and records of a device image, chunk by chunk."""
    flags, recs = [], []
    for s in range(0, n_sectors, chunk):
        e = min(n_sectors, s + chunk)
        host = data[s * SECTOR: e * SECTOR].cpu().numpy()
        t = (tau0 + s) % 8
        f = ox.flag_image(host, t, any_tau, threads=threads)
        m = ox.confirm_image(host, f, t, any_tau)
        m["disk_sector"] += np.uint64(s)
        flags.append(f + np.uint64(s))
        recs.append(m)
    if not flags:
        return np.empty(0, np.uint64), np.empty(0, oracle.MATCH_DTYPE)
    return np.concatenate(flags), np.concatenate(recs)


def _full_size(name: str):
    cfg = synth.CONFIGS[name]
    _log(f"[{name}] generating on the GPU")
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets,
                                     synth.tuning_sample(cfg, ms, device="cuda", max_sectors=1 << 24))
    _log(f"[{name}] index {idx.stats()}, pick {pick}")
    sc = carve.scan_image(idx, img.data)
    flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
    matches = carve.confirm_matches(idx, sc)
    del sc
    _log(f"[{name}] GPU: {len(flags)} flagged, {len(matches)} confirmed; running the oracle")
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    want_flags, want = oracle_chunked(ox, img.data, cfg.n_disk_sectors, th)
    assert np.array_equal(flags, want_flags)
    assert_same_matches(matches, want)
    planted = _planted_ids(img)
    assert np.isin(planted, flags.astype(np.int64)).all()
    _log(f"[{name}] bit-exact over the whole image: {len(flags)} flags, {len(matches)} matches")
    return flags, matches


def test_mid_full_size_exact():
    _full_size("mid")


def test_large_full_size_exact():
    flags, matches = _full_size("large")
    # the low-entropy clusters reach the flag/confirm split at this size
    assert len(flags) > 50_000 and len(matches) > 0
