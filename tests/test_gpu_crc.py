"""The CRC-64 signature (Section 2.1, read as CRC-64/GO-ISO) on the GPU
against the CPU oracle: signatures, flags and confirmed matches."""
import random

import numpy as np
import pytest
import torch

import oracle
import pins
import synth
from gpu_util import assert_same_matches, dev_bytes, gpu_flags_and_matches, oracle_flags_and_matches
from oracle import spec
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512
CRC = carve.CARVE_SIG_CRC64_ISO


def _u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4097])
def test_crc_signatures_random(n):
    rng = np.random.default_rng(n)
    host = rng.integers(0, 256, size=n * SECTOR, dtype=np.uint8)
    got = _u64(carve.sector_signatures(torch.from_numpy(host).cuda(), sig_kind=CRC))
    want = oracle.sector_signatures(host, threads=4, sig_kind=oracle.SIG_CRC64_GO_ISO)
    assert np.array_equal(got, want)


def test_crc_signatures_special_sectors():
    secs = [bytes(SECTOR), b"\xff" * SECTOR, bytes(i & 255 for i in range(SECTOR))]
    secs.append(spec.crc_collide(secs[2], 100))          # same CRC as the ramp
    got = _u64(carve.sector_signatures(dev_bytes(b"".join(secs)), sig_kind=CRC))
    want = [spec.crc_polydiv(s) for s in secs]
    assert [int(x) for x in got] == want
    assert want[0] == 0x7CD9900000000000 and want[3] == want[2]


def test_crc_signatures_differ_from_djb2():
    host = np.random.default_rng(3).integers(0, 256, size=8 * SECTOR, dtype=np.uint8)
    t = torch.from_numpy(host).cuda()
    assert not np.array_equal(_u64(carve.sector_signatures(t, sig_kind=CRC)), _u64(carve.sector_signatures(t)))


@pytest.mark.parametrize("bloom", [0, carve.CARVE_BLOOM_OFF])
@pytest.mark.parametrize("tau0,any_tau", [(0, False), (5, False), (0, True)])
def test_crc_small_case(bloom, tau0, any_tau):
    image, masters, offsets, truth = pins.crc_small_case()
    mflat = b"".join(masters)
    idx = carve.build_master_index(dev_bytes(mflat), offsets, bloom_bits_per_key=bloom, sig_kind=CRC)
    f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), tau0, any_tau)
    wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets, np.frombuffer(image, np.uint8),
                                      tau0, any_tau, sig_kind=oracle.SIG_CRC64_GO_ISO)
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    if tau0 == 0 and not any_tau:
        assert len(set(f.tolist()) - set(m["disk_sector"].tolist())) > 0   # CRC collisions: flagged only


@pytest.fixture(scope="module")
def tiny_crc():
    cfg = synth.CONFIGS["tiny"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, sig_kind=CRC)
    return cfg, ms, img, idx


@pytest.mark.parametrize("tau0,any_tau", [(0, False), (3, False), (0, True)])
def test_crc_tiny_config(tiny_crc, tau0, any_tau):
    cfg, ms, img, idx = tiny_crc
    f, m, _ = gpu_flags_and_matches(idx, img.data, tau0, any_tau)
    wf, wm = oracle_flags_and_matches(ms.sectors.cpu().numpy(), ms.file_offsets, img.data.cpu().numpy(), tau0,
                                      any_tau, sig_kind=oracle.SIG_CRC64_GO_ISO)
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_crc_and_djb2_confirm_the_same_bytes(tiny_crc):
    """Confirmation is a byte comparison: both signatures confirm exactly the
    brute-force set (they may flag different collisions)."""
    cfg, ms, img, idx = tiny_crc
    _, m_crc, _ = gpu_flags_and_matches(idx, img.data)
    djb = carve.build_master_index(ms.sectors, ms.file_offsets)
    _, m_djb, _ = gpu_flags_and_matches(djb, img.data)
    assert_same_matches(m_crc, m_djb)
    brute = oracle.bruteforce(img.data.cpu().numpy(), ms.sectors.cpu().numpy(), ms.file_offsets,
                              threads=oracle.default_threads())
    assert_same_matches(m_crc, brute)


def test_crc_batch_equals_alone(tiny_crc):
    cfg, ms, img, idx = tiny_crc
    data = img.data
    images = [(data[: 512 * 777 + 5], 0, 0), (data[512 * 1000: 512 * 9000], 0, 0),
              (data[512 * 20000: 512 * 20100], 4, carve.CARVE_TAU_ANY), (data[:0], 0, 0)]
    b = carve.scan_batch(idx, images)
    counts = carve.batch_flag_counts(b)
    bm = carve.batch_confirm_matches(idx, b)
    at = 0
    for i, (t, tau0, mode) in enumerate(images):
        f, m, _ = gpu_flags_and_matches(idx, t, tau0, mode == carve.CARVE_TAU_ANY)
        assert counts[i] == len(f)
        assert np.array_equal(carve.batch_flagged_sectors(b, i).numpy().astype(np.uint64), f)
        sel = bm[bm["image"] == i]
        assert np.array_equal(sel["disk_sector"], m["disk_sector"]) and np.array_equal(sel["file_id"], m["file_id"])
        at += len(m)
    assert at == len(bm)


def test_crc_mid_scaled():
    """Several thousand tiles, a ragged tail, Bloom on, against the oracle."""
    cfg = synth.scaled(synth.CONFIGS["mid"], n_master_sectors=60000, n_disk_sectors=(1 << 20) + 37, n_files=70,
                       tail_bytes=300)
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, sig_kind=CRC)
    f, m, _ = gpu_flags_and_matches(idx, img.data)      # the image's clusters start at sector 0
    wf, wm = oracle_flags_and_matches(ms.sectors.cpu().numpy(), ms.file_offsets, img.data.cpu().numpy(),
                                      sig_kind=oracle.SIG_CRC64_GO_ISO)
    assert len(wf) > 1000
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_crc_kind_rejected_when_unknown():
    with pytest.raises(carve.CarveError):
        carve.sector_signatures(torch.zeros(512, dtype=torch.uint8, device="cuda"), sig_kind=7)
    with pytest.raises(carve.CarveError) as e:
        carve.build_master_index(torch.zeros(512, dtype=torch.uint8, device="cuda"), [0, 1], sig_kind=7)
    assert e.value.code == carve.CARVE_EUNSUPPORTED
