"""The index autotuner (autotune_index), through the C ABI: every candidate it
can pick (layout x prefilter bits per signature x contiguous or
position-split walk) flags and confirms exactly what the CPU oracle does
(Section 3.1; the layouts of Eq. (3) and Section 4), the picked index scans
bit-exactly, and a pick is cached per class of master set."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    # 262,144 master sectors, a 64 MiB image and a 32 MiB tuning sample of the mid recipe
    cfg = synth.scaled(synth.CONFIGS["mid"], n_master_sectors=1 << 18, n_disk_sectors=1 << 17, n_files=200,
                       p_master_cluster=0.03)
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda").data
    sample = synth.tuning_sample(cfg, ms, device="cuda", max_sectors=1 << 16)
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    host = img.cpu().numpy()
    want = {}
    for any_tau in (False, True):
        f = ox.flag_image(host, 0, any_tau, threads=th)
        want[any_tau] = (f, ox.confirm_image(host, f, 0, any_tau))
    assert len(want[False][0]) > 1000
    return ms, img, sample, want


def _check(idx, img, want):
    for any_tau in (False, True):
        sc = carve.scan_image(idx, img, tau_mode=carve.CARVE_TAU_ANY if any_tau else carve.CARVE_TAU_PER_CLUSTER)
        flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
        assert np.array_equal(flags, want[any_tau][0])
        assert_same_matches(carve.confirm_matches(idx, sc), want[any_tau][1])


@pytest.mark.parametrize("layout", [carve.CARVE_LAYOUT_BUCKETED, carve.CARVE_LAYOUT_LINEAR, carve.CARVE_LAYOUT_SORTED])
@pytest.mark.parametrize("bits", [0, 8, 16, 32])
def test_every_candidate_exact(setup, layout, bits):
    ms, img, _, want = setup
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, layout=layout, bloom_bits_per_key=bits)
    for split in (carve.CARVE_SPLIT_OFF, carve.CARVE_SPLIT_ON):
        idx.set_scan_config(2, 1, split)
        _check(idx, img, want)


def test_pick_exact_and_cached(setup):
    ms, img, sample, want = setup
    idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets, sample, no_cache=True)
    assert pick["candidates"] == 12 and not pick["from_cache"]
    assert pick["layout"] in ("bucketed", "linear", "sorted") and pick["kernel_ms_on_sample"] > 0
    cfg = idx.scan_config()
    assert (cfg["blocks_per_cu"], cfg["tiles_per_chunk"]) == (pick["blocks_per_cu"], pick["tiles_per_chunk"])
    _check(idx, img, want)
    idx2, pick2 = carve.autotune_index(ms.sectors, ms.file_offsets, sample)
    assert pick2["from_cache"] and pick2["candidates"] == 0
    for k in ("layout", "bloom_bits_per_key", "blocks_per_cu", "tiles_per_chunk", "split"):
        assert pick2[k] == pick[k], k
    assert idx2.scan_config() == idx.scan_config()
    _check(idx2, img, want)


def test_contiguous_only_and_narrow_space(setup):
    ms, img, sample, want = setup
    idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets, sample, layouts=1 << carve.CARVE_LAYOUT_LINEAR,
                                     bloom_bits=(8, carve.CARVE_BLOOM_OFF), contiguous_only=True, no_cache=True)
    assert pick["candidates"] == 2 and pick["layout"] == "linear" and pick["split"] == "off"
    assert pick["bloom_bits_per_key"] in (8, "off")
    _check(idx, img, want)
    b = carve.scan_batch(idx, [img, img[: 4096 * 100]])
    assert carve.batch_flag_counts(b).tolist()[0] == len(want[False][0])


def test_bad_space(setup):
    ms, _, sample, _ = setup
    with pytest.raises(carve.CarveError):
        carve.autotune_index(ms.sectors, ms.file_offsets, sample, layouts=8)
    with pytest.raises(carve.CarveError):
        carve.autotune_index(ms.sectors, ms.file_offsets, sample, bloom_bits=(3,))
    with pytest.raises(carve.CarveError):
        carve.autotune_index(ms.sectors, ms.file_offsets, sample[:100])
