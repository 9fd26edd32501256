"""Parity at the full workload sizes, through the C ABI, in the launch
configuration bench.py times (default index parameters, one scan per image).

mid (8 GiB image, 1,048,576 master sectors): every flag and every confirmed
match is compared with the CPU oracle run over the whole image.
large (64 GiB image, 16,777,216 master sectors): the oracle judges sampled
sectors one by one (random ones, every flagged one, every planted one), and
whole-image properties are checked."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_same_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512


def _log(*a):
    print(*a, flush=True)


def _planted_ids(img) -> np.ndarray:
    ids = []
    for c, r in zip(img.planted_clusters.tolist(), img.planted_overwrite.tolist()):
        ids.extend(range(8 * c + r, 8 * c + 8))
    return np.asarray(ids, dtype=np.int64)


def test_mid_full_size_exact():
    cfg = synth.CONFIGS["mid"]
    _log("[mid] generating on the GPU")
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    sc = carve.scan_image(idx, img.data)
    flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
    matches = carve.confirm_matches(idx, sc)
    _log(f"[mid] GPU: {len(flags)} flagged, {len(matches)} confirmed; running the oracle")
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    host = img.data.cpu().numpy()
    want_flags = ox.flag_image(host, threads=th)
    assert np.array_equal(flags, want_flags)
    want = ox.confirm_image(host, want_flags)
    assert_same_matches(matches, want)
    planted = _planted_ids(img)
    assert np.isin(planted, flags.astype(np.int64)).all()
    _log(f"[mid] bit-exact: {len(flags)} flags, {len(matches)} matches")


def test_large_sampled():
    cfg = synth.CONFIGS["large"]
    _log("[large] generating on the GPU")
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    _log(f"[large] index: {idx.stats()}")
    sc = carve.scan_image(idx, img.data)
    flags = carve.flagged_sectors(sc).numpy().astype(np.int64)
    matches = carve.confirm_matches(idx, sc)
    _log(f"[large] GPU: {len(flags)} flagged, {len(matches)} confirmed; building the oracle")
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    g = torch.Generator().manual_seed(11)
    rand = torch.randint(0, cfg.n_disk_sectors, (1 << 20,), generator=g).numpy()
    planted = _planted_ids(img)
    sample = np.unique(np.concatenate([rand, flags, planted, [0, cfg.n_disk_sectors - 1]]))
    _log(f"[large] oracle on {len(sample)} sampled sectors")
    secs = img.data.view(-1, SECTOR)[torch.from_numpy(sample).cuda()].cpu().numpy()
    want_flag = ox.flag_sectors(secs, sample.astype(np.uint64), threads=th)
    got_flag = np.isin(sample, flags)
    assert np.array_equal(got_flag, want_flag)
    # confirmed matches of the flagged sectors (all of them are in the sample)
    sel = np.isin(sample, flags)
    want = ox.confirm(secs[sel], sample[sel].astype(np.uint64))
    assert_same_matches(matches, want)
    # properties of the whole image
    assert np.all(np.diff(flags) > 0)
    assert np.isin(planted, flags).all()
    assert len(set(matches["disk_sector"].tolist())) <= len(flags)
    _log(f"[large] sampled parity ok: {len(flags)} flags, {len(matches)} matches")
