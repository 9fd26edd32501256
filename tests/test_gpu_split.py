"""The position-split scan (one image, per-cluster rule, an index whose
filter is 4 MiB or more): every XCD scans one cluster position and probes
that position's slice of the filter. Flags and records against the oracle,
on the whole 8 GiB mid image and on ragged slices of it at every tau0."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_same_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512


@pytest.fixture(scope="module")
def mid():
    cfg = synth.CONFIGS["mid"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    # 32 bits per signature: a 4 MiB filter, so scans of one image run split
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, bloom_bits_per_key=32)
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    return ms, img, idx, ox, th


def test_split_index_has_a_large_filter(mid):
    _, _, idx, _, _ = mid
    assert idx.stats()["bloom_bytes"] >= 4 << 20


def test_split_whole_mid_image(mid):
    ms, img, idx, ox, th = mid
    sc = carve.scan_image(idx, img.data)
    flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
    matches = carve.confirm_matches(idx, sc)
    host = img.data.cpu().numpy()
    want_flags = ox.flag_image(host, threads=th)
    assert np.array_equal(flags, want_flags)
    assert_same_matches(matches, ox.confirm_image(host, want_flags))


@pytest.mark.parametrize("n_sectors,extra", [(0, 100), (1, 0), (3, 5), (7, 511), (8, 0), (9, 0), (63, 0), (64, 0),
                                             (65, 3), (511, 0), (512, 0), (513, 0), (4096 * 3 + 77, 0)])
def test_split_ragged_slices(mid, n_sectors, extra):
    ms, img, idx, ox, th = mid
    planted = img.planted_clusters.tolist()
    start = 8 * planted[n_sectors % len(planted)] - 3 if planted else 5   # around a planted cluster
    start = max(start, 0)
    n_bytes = n_sectors * SECTOR + extra
    whole = img.data[start * SECTOR: start * SECTOR + n_bytes]
    buf = torch.zeros(max(n_bytes, 16), dtype=torch.uint8, device="cuda")
    buf[:whole.numel()] = whole
    part = buf[:n_bytes]
    host = part.cpu().numpy()
    for tau0 in range(8):
        for mode in (carve.CARVE_TAU_PER_CLUSTER, carve.CARVE_TAU_ANY):
            sc = carve.scan_image(idx, part, tau0=tau0, tau_mode=mode)
            flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
            any_tau = mode == carve.CARVE_TAU_ANY
            want = ox.flag_image(host, tau0, any_tau, threads=th)
            assert np.array_equal(flags, want), (n_sectors, tau0, mode)
            assert_same_matches(carve.confirm_matches(idx, sc), ox.confirm_image(host, want, tau0, any_tau))


@pytest.mark.parametrize("split", [carve.CARVE_SPLIT_OFF, carve.CARVE_SPLIT_ON])
@pytest.mark.parametrize("n_masters", [3, 20, 40, 70, 150, 1000, 5000])
def test_small_indexes_either_walk(n_masters, split):
    """Indexes of a few master sectors and up: no filter (under 5 distinct
    signatures), filters too small to split (fewer than 16 words), and the
    smallest split filters (2 words per position and up). Either walk,
    forced, agrees with the oracle at several tau0 and both rules."""
    cfg = synth.scaled(synth.CONFIGS["tiny"], n_master_sectors=n_masters, n_disk_sectors=4096 + 13,
                       n_files=max(1, n_masters // 8), equal_files=False, tail_bytes=100)
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda").data
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    idx.set_scan_config(0, 0, split)
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    host = img.cpu().numpy()
    for tau0 in (0, 3):
        for mode in (carve.CARVE_TAU_PER_CLUSTER, carve.CARVE_TAU_ANY):
            any_tau = mode == carve.CARVE_TAU_ANY
            sc = carve.scan_image(idx, img, tau0=tau0, tau_mode=mode)
            flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
            want = ox.flag_image(host, tau0, any_tau, threads=th)
            assert np.array_equal(flags, want), (n_masters, split, tau0, mode)
            assert_same_matches(carve.confirm_matches(idx, sc), ox.confirm_image(host, want, tau0, any_tau))
