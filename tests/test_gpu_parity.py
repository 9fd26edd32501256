"""HIP path vs the CPU oracle, element by element, through the C ABI.

Integer work throughout: the bar is bit-exact equality of signatures, of the
ascending flagged-sector list and of the ordered match records."""
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
MOD = 1 << 64
K_BUCKET = 0x9E3779B97F4A7C15


def _u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


# ---------------------------------------------------------------- signatures
@pytest.mark.parametrize("n", [1, 63, 64, 65, 64 * 37 + 13, 4096])
def test_signatures_random(n):
    g = torch.Generator().manual_seed(n)
    host = torch.randint(0, 256, (n, SECTOR), dtype=torch.uint8, generator=g)
    got = _u64(carve.sector_signatures(host.cuda()))
    want = oracle.sector_signatures(host.numpy(), threads=4)
    assert np.array_equal(got, want)


def test_signatures_special_sectors():
    rng = random.Random(5)
    secs = [bytes(SECTOR), b"\xff" * SECTOR, bytes(i & 255 for i in range(SECTOR))]
    secs += [bytes([c]) * SECTOR for c in (1, 0x21, 0x80)]
    secs += [spec.craft_sector(bytes(rng.getrandbits(8) for _ in range(100)), t)
             for t in (0, 1, MOD - 1, 5381, rng.getrandbits(64))]
    host = np.frombuffer(b"".join(secs), np.uint8)
    got = _u64(carve.sector_signatures(torch.from_numpy(host.copy()).cuda()))
    assert [int(x) for x in got] == [spec.djb2_closed(s) for s in secs]


def test_signatures_ignore_trailing_bytes():
    g = torch.Generator().manual_seed(1)
    host = torch.randint(0, 256, (3 * SECTOR + 100,), dtype=torch.uint8, generator=g)
    got = _u64(carve.sector_signatures(host.cuda()))
    assert got.size == 3
    assert np.array_equal(got, oracle.sector_signatures(host[:3 * SECTOR].numpy()))


# ------------------------------------------------------- small adversarial
BLOOMS = [0, carve.CARVE_BLOOM_OFF, 4]   # automatic, none, a deliberately weak filter


@pytest.mark.parametrize("bloom", BLOOMS)
@pytest.mark.parametrize("tau0,any_tau", [(0, False), (3, False), (7, False), (0, True), (5, True)])
def test_small_case(tau0, any_tau, bloom):
    image, masters, offsets, truth = pins.small_case(seed=3)
    mflat = b"".join(masters)
    idx = carve.build_master_index(dev_bytes(mflat), offsets, bloom_bits_per_key=bloom)
    img = dev_bytes(image)
    flags, matches, _ = gpu_flags_and_matches(idx, img, tau0, any_tau)
    wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets, np.frombuffer(image, np.uint8),
                                      tau0, any_tau)
    assert np.array_equal(flags, wf)
    assert_same_matches(matches, wm)


def test_index_stats_small():
    _, masters, offsets, _ = pins.small_case(seed=3)
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets)
    st = idx.stats()
    assert st["n_master_sectors"] == len(masters)
    assert st["n_unique_signatures"] == len(set(masters))
    assert st["bloom_bytes"] > 0
    off = carve.build_master_index(dev_bytes(b"".join(masters)), offsets, bloom_bits_per_key=carve.CARVE_BLOOM_OFF)
    assert off.stats()["bloom_bytes"] == 0


@pytest.mark.parametrize("bloom", BLOOMS)
def test_tiny_config_bloom_invariance(tiny_gpu, bloom):
    """The prefilter is an optimisation only: flags and matches do not depend on it."""
    cfg, ms, img, idx = tiny_gpu
    alt = carve.build_master_index(ms.sectors, ms.file_offsets, bloom_bits_per_key=bloom)
    for tau0, any_tau in ((0, False), (0, True)):
        f1, m1, _ = gpu_flags_and_matches(idx, img.data, tau0, any_tau)
        f2, m2, _ = gpu_flags_and_matches(alt, img.data, tau0, any_tau)
        assert np.array_equal(f1, f2)
        assert_same_matches(m2, m1)


# ------------------------------------------------------- tiny configuration
@pytest.fixture(scope="module")
def tiny_gpu():
    cfg = synth.CONFIGS["tiny"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    return cfg, ms, img, idx


@pytest.mark.parametrize("tau0,any_tau", [(0, False), (6, False), (0, True)])
def test_tiny_config(tiny_gpu, tau0, any_tau):
    cfg, ms, img, idx = tiny_gpu
    flags, matches, _ = gpu_flags_and_matches(idx, img.data, tau0, any_tau)
    wf, wm = oracle_flags_and_matches(ms.sectors.cpu().numpy(), ms.file_offsets, img.data.cpu().numpy(), tau0, any_tau)
    assert np.array_equal(flags, wf)
    assert_same_matches(matches, wm)
    if tau0 == 0 and not any_tau:
        assert len(flags) > 5000


def test_tiny_config_bruteforce(tiny_gpu):
    """GPU confirmed set == all-pairs byte comparison (no signatures at all)."""
    cfg, ms, img, idx = tiny_gpu
    _, matches, _ = gpu_flags_and_matches(idx, img.data)
    brute = oracle.bruteforce(img.data.cpu().numpy(), ms.sectors.cpu().numpy(), ms.file_offsets,
                              threads=oracle.default_threads())
    assert_same_matches(matches, brute)


def test_deterministic_and_reusable_scan(tiny_gpu):
    cfg, ms, img, idx = tiny_gpu
    f1, m1, sc = gpu_flags_and_matches(idx, img.data)
    f2, m2, _ = gpu_flags_and_matches(idx, img.data, scan=sc)       # reuse the scan object
    assert np.array_equal(f1, f2)
    assert_same_matches(m1, m2)
    # a shorter image through the same scan object
    f3, _, _ = gpu_flags_and_matches(idx, img.data[:1000 * SECTOR + 7], scan=sc)
    assert np.array_equal(f3, f1[f1 < 1000])


def test_chunked_scan_with_tau0(tiny_gpu):
    """Scanning an image in chunks that start mid-cluster, with tau0 = start mod 8,
    gives the same flags as one scan."""
    cfg, ms, img, idx = tiny_gpu
    full, _, _ = gpu_flags_and_matches(idx, img.data)
    got = []
    bounds = [0, 5, 4099, 77777, cfg.n_disk_sectors]
    for a, b in zip(bounds, bounds[1:]):
        f, _, _ = gpu_flags_and_matches(idx, img.data[a * SECTOR:b * SECTOR].clone(), tau0=a % 8)
        got.append(f + np.uint64(a))
    assert np.array_equal(np.concatenate(got), full)


# ---------------------------------------------------------------- edge cases
def test_empty_and_subsector_images(tiny_gpu):
    cfg, ms, img, idx = tiny_gpu
    for nbytes in (0, 1, 511):
        t = img.data[:max(nbytes, 1)].clone()
        sc = carve.scan_image(idx, t, n_bytes=nbytes)
        assert carve.flagged_sectors(sc).numel() == 0
        assert len(carve.confirm_matches(idx, sc)) == 0


def test_single_sector_image(tiny_gpu):
    cfg, ms, img, idx = tiny_gpu
    one = ms.sectors[8].clone().reshape(-1)           # master sector k = 8 (tau 0)
    f, m, _ = gpu_flags_and_matches(idx, one)
    assert f.tolist() == [0]
    assert (int(m["file_id"][0]), int(m["sector_in_file"][0])) == (0, 8)
    f, _, _ = gpu_flags_and_matches(idx, one, tau0=1)
    assert f.tolist() == []


def test_empty_master_set():
    idx = carve.build_master_index(torch.empty(0, dtype=torch.uint8, device="cuda"), [0])
    img = torch.zeros(64 * SECTOR, dtype=torch.uint8, device="cuda")
    f, m, _ = gpu_flags_and_matches(idx, img)
    assert f.size == 0 and len(m) == 0


def test_zero_disk_against_zero_master():
    rng = random.Random(4)
    masters = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(20)]
    masters[3] = bytes(SECTOR)
    masters[13] = bytes(SECTOR)                        # second file, k = 3 as well
    offsets = [0, 10, 20]
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets)
    img = torch.zeros(1000 * SECTOR, dtype=torch.uint8, device="cuda")
    for any_tau in (False, True):
        f, m, _ = gpu_flags_and_matches(idx, img, any_tau=any_tau)
        wf, wm = oracle_flags_and_matches(np.frombuffer(b"".join(masters), np.uint8), offsets,
                                          np.zeros(1000 * SECTOR, np.uint8), any_tau=any_tau)
        assert np.array_equal(f, wf)
        assert_same_matches(m, wm)
    assert len(m) == 2000


def test_master_with_signature_zero():
    """Signature 0 is the empty-slot marker of the table; it must still match."""
    rng = random.Random(6)
    masters = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(16)]
    z = spec.craft_sector(b"zero", 0)
    z2 = spec.craft_sector(b"zero-2", 0)               # same signature, other bytes
    masters[5] = z
    offsets = [0, 16]
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets)
    disk = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(64)]
    disk[13] = z          # tau 5: flagged and confirmed
    disk[21] = z2         # tau 5: flagged, not confirmed
    disk[22] = z          # tau 6: not flagged
    f, m, _ = gpu_flags_and_matches(idx, dev_bytes(b"".join(disk)))
    assert f.tolist() == [13, 21]
    assert m["disk_sector"].tolist() == [13]
    f, m, _ = gpu_flags_and_matches(idx, dev_bytes(b"".join(disk)), any_tau=True)
    assert f.tolist() == [13, 21, 22]


def _inv(a: int) -> int:
    return pow(a, -1, MOD)


def _crafted_batch(prefix: bytes, targets):
    """Sectors with given signatures: shared prefix, 13 base-33 digits at the end."""
    body = prefix + bytes(SECTOR - 13 - len(prefix))
    base = spec.djb2_closed(body + bytes(13))
    out = []
    for t in targets:
        need = (t - base) % MOD
        d = []
        for _ in range(13):
            d.append(need % 33)
            need //= 33
        out.append(body + bytes(d[12 - i] for i in range(13)))
    return out


@pytest.mark.parametrize("bloom", BLOOMS)
def test_long_probe_chains(bloom):
    """Thousands of master signatures whose home bucket is bucket 0 (so they
    overflow into many later buckets), probed by present and absent sectors."""
    rng = random.Random(7)
    kinv = _inv(K_BUCKET)
    n_same = 3000
    vals = rng.sample(range(1, 1 << 30), 2 * n_same)
    targets = [(v * kinv) % MOD for v in vals]          # target*K < 2^30: home bucket 0
    crafted = _crafted_batch(b"chain", targets)
    masters = crafted[:n_same] + [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(5000)]
    offsets = [0, 4000, len(masters)]
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets, bloom_bits_per_key=bloom)
    st = idx.stats()
    assert st["n_overflow_keys"] > 2000
    disk = []
    for i in range(4096):
        r = rng.random()
        if r < 0.3:
            disk.append(crafted[rng.randrange(n_same)])          # present
        elif r < 0.6:
            disk.append(crafted[n_same + rng.randrange(n_same)])  # absent, same home bucket
        else:
            disk.append(bytes(rng.getrandbits(8) for _ in range(SECTOR)))
    image = b"".join(disk)
    for any_tau in (False, True):
        f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), any_tau=any_tau)
        wf, wm = oracle_flags_and_matches(np.frombuffer(b"".join(masters), np.uint8), offsets,
                                          np.frombuffer(image, np.uint8), any_tau=any_tau)
        assert np.array_equal(f, wf)
        assert_same_matches(m, wm)


def test_many_duplicates_of_one_sector():
    """A sector repeated in many master files: every copy is reported, ordered."""
    rng = random.Random(8)
    dup = bytes(rng.getrandbits(8) for _ in range(SECTOR))
    masters, offsets = [], [0]
    for f in range(300):
        n = 8 + f % 5
        sec = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(n)]
        sec[f % n] = dup
        masters += sec
        offsets.append(len(masters))
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets)
    disk = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(256)]
    for j in (3, 64, 65, 200):
        disk[j] = dup
    image = b"".join(disk)
    for any_tau in (False, True):
        f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), any_tau=any_tau)
        wf, wm = oracle_flags_and_matches(np.frombuffer(b"".join(masters), np.uint8), offsets,
                                          np.frombuffer(image, np.uint8), any_tau=any_tau)
        assert np.array_equal(f, wf)
        assert_same_matches(m, wm)
    assert len(m) == 4 * 300


@pytest.mark.parametrize("n_planted", [1023, 1024, 1025, 2047, 2048, 2049, 4097])
def test_compaction_chunk_edges(n_planted):
    """The compaction works in chunks of 1024 items: hit words (64 sectors
    each) for the flagged ids, then one count per flagged sector for the
    record offsets. Flags on both sides of word-chunk edges and flagged counts
    around multiples of 1024 give the oracle's lists exactly."""
    gen = torch.Generator().manual_seed(n_planted)
    masters = torch.randint(0, 256, (4096 * SECTOR,), dtype=torch.uint8, generator=gen)
    n_sec = 2048 * 64 * 2 + 37                         # 4096 hit words and a ragged one
    image = torch.randint(0, 256, (n_sec * SECTOR,), dtype=torch.uint8, generator=gen)
    edges = [0, 1024 * 64 - 1, 1024 * 64, 2048 * 64 - 1, 2048 * 64, 2048 * 64 + 1, 4096 * 64 - 1, 4096 * 64,
             n_sec - 1]
    rng = random.Random(n_planted)
    rest = rng.sample(sorted(set(range(n_sec)) - set(edges)), n_planted - len(edges))
    img2 = image.view(n_sec, SECTOR)
    m2 = masters.view(4096, SECTOR)
    for p in edges + rest:
        img2[p] = m2[8 * rng.randrange(512) + p % 8]      # a master at the sector's own cluster position
    idx = carve.build_master_index(masters.cuda(), [0, 4096])
    f, m, _ = gpu_flags_and_matches(idx, image.cuda())
    wf, wm = oracle_flags_and_matches(masters.numpy(), [0, 4096], image.numpy())
    assert len(wf) == n_planted
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_kernel_timing_series(tiny_gpu):
    """Every timed launch's kernel duration can be read after the loop."""
    cfg, ms, img, idx = tiny_gpu
    sc = carve.scan_image(idx, img.data)
    sc.set_timing(True)
    for _ in range(3):
        carve.scan_image(idx, img.data, scan=sc)
    got = sc.kernel_ms_recent(8)
    assert len(got) == 3 and all(t > 0 for t in got)
    assert got[-1] == sc.kernel_ms()
    assert sc.kernel_ms_recent(2) == got[1:]
    sc.set_timing(False)
    carve.scan_image(idx, img.data, scan=sc)           # untimed: the series stays
    assert sc.kernel_ms_recent(8) == got
    sc.set_timing(True)                                # a new series
    assert sc.kernel_ms_recent(8) == []
    carve.scan_image(idx, img.data, scan=sc)
    assert len(sc.kernel_ms_recent(8)) == 1


def test_invalid_arguments():
    img = torch.zeros(4 * SECTOR + 16, dtype=torch.uint8, device="cuda")
    idx = carve.build_master_index(torch.zeros(SECTOR, dtype=torch.uint8, device="cuda"), [0, 1])
    with pytest.raises(carve.CarveError) as e:
        carve.scan_image(idx, img[1:])                          # misaligned
    assert e.value.code == carve.CARVE_EINVAL
    with pytest.raises(carve.CarveError):
        carve.scan_image(idx, img, tau0=8)
    with pytest.raises(carve.CarveError):
        carve.scan_image(idx, img, tau_mode=7)
    with pytest.raises(carve.CarveError):
        carve.build_master_index(torch.zeros(2 * SECTOR, dtype=torch.uint8, device="cuda"), [1, 2])
    # a zero master sector: with any position, all 4 zero disk sectors are flagged
    sc = carve.scan_image(idx, img, tau_mode=carve.CARVE_TAU_ANY)
    out = torch.empty(2, dtype=torch.int64)
    with pytest.raises(carve.CarveError) as e:
        carve.flagged_sectors(sc, out)
    assert e.value.code == carve.CARVE_ETRUNC
    assert out.tolist() == [0, 1]                               # the first cap ids were copied
    assert carve.flagged_sectors(sc).tolist() == [0, 1, 2, 3]   # retry with room
    rec = torch.empty(16 * 3, dtype=torch.uint8)
    with pytest.raises(carve.CarveError) as e:
        carve.confirm_matches(idx, sc, rec)
    assert e.value.code == carve.CARVE_ETRUNC
    assert len(carve.confirm_matches(idx, sc)) == 4


def test_confirm_enqueue_then_copy(tiny_gpu):
    """Confirmation enqueued right after the scan, copied later, equals the direct path."""
    cfg, ms, img, idx = tiny_gpu
    f, m, sc = gpu_flags_and_matches(idx, img.data)
    carve.scan_image(idx, img.data, scan=sc)
    carve.confirm_enqueue(idx, sc)
    assert_same_matches(carve.confirm_matches(idx, sc), m)
    assert np.array_equal(carve.flagged_sectors(sc).numpy().astype(np.uint64), f)


@pytest.mark.parametrize("any_tau", [False, True])
def test_more_matches_than_enqueued_room(any_tau):
    """Records beyond the room reserved at enqueue time are produced again on copy."""
    rng = random.Random(13)
    masters, offsets = [], [0]
    for f in range(100):
        sec = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(10)]
        sec[3] = bytes(SECTOR)
        masters += sec
        offsets.append(len(masters))
    idx = carve.build_master_index(dev_bytes(b"".join(masters)), offsets)
    img = torch.zeros(1000 * SECTOR, dtype=torch.uint8, device="cuda")
    sc = carve.scan_image(idx, img, tau_mode=carve.CARVE_TAU_ANY if any_tau else 0)
    carve.confirm_enqueue(idx, sc)
    got = carve.confirm_matches(idx, sc)
    wf, wm = oracle_flags_and_matches(np.frombuffer(b"".join(masters), np.uint8), offsets,
                                      np.zeros(1000 * SECTOR, np.uint8), any_tau=any_tau)
    assert len(wm) == (100_000 if any_tau else 12_500)
    assert_same_matches(got, wm)


def test_confirm_into_device_memory(tiny_gpu):
    """Records emitted straight into a device buffer equal the host copy-out;
    a later host copy of the same scan produces them again; a short device
    buffer gets the first records and ETRUNC with the full count."""
    cfg, ms, img, idx = tiny_gpu
    f, m, _ = gpu_flags_and_matches(idx, img.data)
    assert len(m) > 10
    sc = carve.scan_image(idx, img.data)
    out = torch.zeros(16 * (len(m) + 5), dtype=torch.uint8, device="cuda")
    assert carve.confirm_matches(idx, sc, out) == len(m)
    got = np.frombuffer(out.cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)[: len(m)]
    assert_same_matches(got, m)
    assert_same_matches(carve.confirm_matches(idx, sc), m)       # host copy after a direct emit
    carve.scan_image(idx, img.data, scan=sc)
    short = torch.zeros(16 * 7, dtype=torch.uint8, device="cuda")
    with pytest.raises(carve.CarveError) as e:
        carve.confirm_matches(idx, sc, short)
    assert e.value.code == carve.CARVE_ETRUNC and str(len(m)) in str(e.value)
    first = np.frombuffer(short.cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)
    assert_same_matches(first, m[:7])


def test_one_wait_step(tiny_gpu):
    """The step that waits once: scan_image, the confirmation enqueued into a
    device buffer, the ids copy enqueued, then scan_counts. Ids and records
    equal the oracle's on every repetition; confirm_matches with the same
    buffer only reads the count; a short id buffer gets the first ids; a host
    copy-out afterwards produces the records again; host buffers are refused."""
    cfg, ms, img, idx = tiny_gpu
    wf, wm = oracle_flags_and_matches(ms.sectors.cpu().numpy(), ms.file_offsets, img.data.cpu().numpy())
    assert len(wf) > 5000 and len(wm) > 5000
    ids = torch.full((len(wf) + 9,), -1, dtype=torch.int64, device="cuda")
    rec = torch.zeros(16 * (len(wm) + 3), dtype=torch.uint8, device="cuda")
    sc = None
    for rep in range(3):
        sc = carve.scan_image(idx, img.data, scan=sc)
        if rep == 0:
            assert carve.scan_counts(sc) == (len(wf), None)
        carve.confirm_enqueue(idx, sc, rec)
        carve.flagged_sectors_enqueue(sc, ids)
        assert carve.scan_counts(sc) == (len(wf), len(wm))
        assert np.array_equal(ids[: len(wf)].cpu().numpy().astype(np.uint64), wf)
        assert bool((ids[len(wf):] == -1).all())
        got = np.frombuffer(rec.cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)[: len(wm)]
        assert_same_matches(got, wm)
        assert carve.confirm_matches(idx, sc, rec) == len(wm)
    short = torch.zeros(5, dtype=torch.int64, device="cuda")
    carve.flagged_sectors_enqueue(sc, short)
    assert carve.scan_counts(sc)[0] == len(wf)
    assert np.array_equal(short.cpu().numpy().astype(np.uint64), wf[:5])
    assert_same_matches(carve.confirm_matches(idx, sc), wm)
    with pytest.raises(carve.CarveError) as e:
        carve.flagged_sectors_enqueue(sc, torch.zeros(4, dtype=torch.int64))
    assert e.value.code == carve.CARVE_EINVAL
    with pytest.raises(carve.CarveError) as e:
        carve.confirm_enqueue(idx, sc, torch.zeros(64, dtype=torch.uint8))
    assert e.value.code == carve.CARVE_EINVAL
    empty = carve.scan_image(idx, img.data[:100])
    assert carve.scan_counts(empty) == (0, None)
    carve.confirm_enqueue(idx, empty, rec)
    assert carve.scan_counts(empty) == (0, 0)


def test_host_memory_image_rejected(tiny_gpu):
    """scan_image takes device memory: a pinned or pageable host image is refused
    on the host (EINVAL), before any kernel runs."""
    cfg, ms, img, idx = tiny_gpu
    lib = carve.load_library()
    pinned = torch.zeros(4096, dtype=torch.uint8, pin_memory=True)
    pageable = torch.zeros(4096, dtype=torch.uint8)
    for t in (pinned, pageable):
        h = carve.ctypes.c_void_p()
        rc = lib.scan_image(idx.handle, t.data_ptr(), t.numel(), 0, 0, None, carve.ctypes.byref(h))
        assert rc == carve.CARVE_EINVAL and not h.value
        assert b"device memory" in lib.carve_last_error()


def test_plain_steps_in_flight(tiny_gpu):
    """Two scan objects on two streams over one index, each step's scan
    waiting only for the previous step's scan kernel (scan_wait_kernel) while
    that step's compaction, confirmation and ids copy run on its own stream;
    steps alternate tau0 and the image prefix, so consecutive steps differ.
    Every step's ids and records equal the oracle's."""
    cfg, ms, img, idx = tiny_gpu
    host = img.data.cpu().numpy()
    masters = ms.sectors.cpu().numpy()
    plan = [(0, img.data.numel()), (5, img.data.numel() - 512 * 77), (3, img.data.numel() // 1024 * 512 + 512 * 3),
            (0, img.data.numel() - 512), (7, img.data.numel())]
    expect = [oracle_flags_and_matches(masters, ms.file_offsets, host[:n], tau0) for tau0, n in plan]
    most_f = max(len(f) for f, _ in expect)
    most_m = max(len(m) for _, m in expect)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    scans = [None, None]
    ids = [torch.full((most_f + 5,), -1, dtype=torch.int64, device="cuda") for _ in range(2)]
    rec = [torch.zeros(16 * (most_m + 5), dtype=torch.uint8, device="cuda") for _ in range(2)]

    def check(i):
        k = i % 2
        wf, wm = expect[i]
        assert carve.scan_counts(scans[k]) == (len(wf), len(wm))
        assert np.array_equal(ids[k][: len(wf)].cpu().numpy().astype(np.uint64), wf)
        got = np.frombuffer(rec[k].cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)[: len(wm)]
        assert_same_matches(got, wm)

    for i, (tau0, n) in enumerate(plan):
        k = i % 2
        with torch.cuda.stream(streams[k]):
            if i > 0:
                carve.scan_wait_kernel(scans[1 - k], streams[k])
            scans[k] = carve.scan_image(idx, img.data[:n], tau0=tau0, scan=scans[k])
            carve.confirm_enqueue(idx, scans[k], rec[k])
            carve.flagged_sectors_enqueue(scans[k], ids[k])
        if i > 0:
            check(i - 1)
    check(len(plan) - 1)
