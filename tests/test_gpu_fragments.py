"""Fragment scanning (Section 5): every 64-byte window at a 4-byte boundary of
an image against the 64-byte fragments of master files, on the GPU, against
the CPU oracle (flags and confirmed matches, element by element)."""
import random

import numpy as np
import pytest
import torch

import oracle
import pins
from gpu_util import assert_same_matches, dev_bytes
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu


def _gpu(idx, image: torch.Tensor, scan=None):
    sc = carve.scan_fragments(idx, image, scan=scan)
    return carve.flagged_sectors(sc).numpy().astype(np.uint64), carve.confirm_matches(idx, sc), sc


def _oracle(frag_data, offsets, image: bytes):
    ox = oracle.FragmentIndex(frag_data, offsets, threads=oracle.default_threads())
    img = np.frombuffer(image, np.uint8)
    f = ox.flag_windows(img, threads=oracle.default_threads())
    return f, ox.confirm_windows(img, f)


@pytest.mark.parametrize("bloom", [0, carve.CARVE_BLOOM_OFF])
def test_fragments_small_case(bloom):
    image, fragments, frag_data, offsets, truth = pins.fragment_small_case()
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets, bloom_bits_per_key=bloom)
    f, m, _ = _gpu(idx, dev_bytes(image))
    wf, wm = _oracle(frag_data, offsets, image)
    assert len(wf) > 100
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    got = {(int(r["disk_sector"]), int(r["file_id"]), int(r["sector_in_file"])) for r in m}
    assert truth <= got


def _files(rng, n, lo=64, hi=4096):
    return [bytes(rng.getrandbits(8) for _ in range(rng.randrange(lo, hi))) for _ in range(n)]


@pytest.mark.parametrize("n_bytes", [0, 63, 64, 67, 68, 100, 124, 128, 4096, 4096 + 60, 4096 + 64, 8191,
                                     8192 + 59, 8192 + 60, 8192 + 64, 8192 + 67, 3 * 8192 + 1000, 5 * 8192])
def test_fragment_sizes(n_bytes):
    """Every window up to the last one (4j + 64 <= n), across whole and partial
    lanes (16 windows each) and wave tasks (1024 windows, 4 KiB of image each:
    4096 + 60 bytes is exactly one task, 4096 + 64 one window more), with a
    fragment planted at the very end."""
    rng = random.Random(n_bytes)
    files = _files(rng, 6)
    frag_data, offsets = oracle.pack_fragment_files(files)
    img = bytearray(rng.getrandbits(8) for _ in range(n_bytes))
    if n_bytes >= 64:
        last = (n_bytes - 64) // 4 * 4
        if last >= 64:
            img[0:64] = frag_data[-1].tobytes()               # the first window
        img[last:last + 64] = frag_data[0].tobytes()          # the last window
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    buf = torch.zeros(max(n_bytes, 16) + 16, dtype=torch.uint8, device="cuda")
    if n_bytes:
        buf[:n_bytes] = torch.frombuffer(bytearray(img), dtype=torch.uint8).cuda()
    f, m, _ = _gpu(idx, buf[:n_bytes])
    wf, wm = _oracle(frag_data, offsets, bytes(img))
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    if n_bytes >= 64:
        assert int(wf[-1]) == (n_bytes - 64) // 4
        if n_bytes >= 128:
            assert int(wf[0]) == 0


def test_fragment_many_candidates():
    """One fragment shared by 70 files (more than the 64 candidates a match
    mask holds) inside a repeated run: every copy confirmed, in order."""
    rng = random.Random(3)
    common = bytes(rng.getrandbits(8) for _ in range(64))
    files = [bytes(rng.getrandbits(8) for _ in range(64 * (i % 3))) + common for i in range(70)]
    frag_data, offsets = oracle.pack_fragment_files(files)
    img = bytearray(rng.getrandbits(8) for _ in range(20000))
    for o in (400, 1200, 1264, 9000):
        img[o:o + 64] = common
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    f, m, _ = _gpu(idx, dev_bytes(bytes(img)))
    wf, wm = _oracle(frag_data, offsets, bytes(img))
    assert len(wm) == 4 * 70
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


@pytest.mark.parametrize("n_list", [31, 32, 33, 63, 64])
def test_fragment_candidate_lists(n_list):
    """A candidate list of n_list fragments with one signature, every third a
    crafted collision (same signature, other bytes): windows equal to the
    common fragment match only the equal ones, a window equal to a collision
    only its copies (lists up to 32 and longer ones are recorded differently)."""
    from oracle import spec
    rng = random.Random(n_list)
    common = bytes(rng.getrandbits(8) for _ in range(64))
    spots = [i for i in range(63) if common[i] <= 254 and common[i + 1] >= 33]
    variants = [spec.collide(common, i) for i in spots[:3]]
    assert all(spec.djb2_closed(v) == spec.djb2_closed(common) and v != common for v in variants)
    files = [variants[(k // 3) % len(variants)] if k % 3 == 2 else common for k in range(n_list)]
    frag_data, offsets = oracle.pack_fragment_files(files)
    img = bytearray(rng.getrandbits(8) for _ in range(16384))
    for o in (0, 1000, 5000, 16384 - 64):
        img[o:o + 64] = common
    img[9000:9064] = variants[0]
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    f, m, _ = _gpu(idx, dev_bytes(bytes(img)))
    wf, wm = _oracle(frag_data, offsets, bytes(img))
    n_common = sum(1 for x in files if x == common)
    assert len(wm) == 4 * n_common + sum(1 for x in files if x == variants[0])
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_fragment_mixed_large():
    """A 4 MiB image with logos embedded at aligned and unaligned offsets,
    zero runs and random bytes, 300 master files; also confirmation enqueued
    and emitted into device memory."""
    rng = random.Random(9)
    files = _files(rng, 300, 256, 8192)
    files[7] = bytes(2048)                                    # a file of zeros
    frag_data, offsets = oracle.pack_fragment_files(files)
    n = 4 << 20
    img = bytearray(np.random.default_rng(9).integers(0, 256, size=n, dtype=np.uint8).tobytes())
    o = 0
    while o < n - 10000:
        data = files[rng.randrange(len(files))]
        o += rng.randrange(100, 20000)
        o -= o % 4 if rng.random() < 0.8 else 0
        img[o:o + len(data)] = data
        o += len(data)
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    image = dev_bytes(bytes(img))
    f, m, sc = _gpu(idx, image)
    wf, wm = _oracle(frag_data, offsets, bytes(img))
    assert len(wf) > 1000
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    carve.scan_fragments(idx, image, scan=sc)
    carve.confirm_enqueue(idx, sc)
    assert_same_matches(carve.confirm_matches(idx, sc), wm)
    carve.scan_fragments(idx, image, scan=sc)
    out = torch.zeros(16 * (len(wm) + 3), dtype=torch.uint8, device="cuda")
    assert carve.confirm_matches(idx, sc, out) == len(wm)
    assert_same_matches(np.frombuffer(out.cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)[: len(wm)], wm)


def test_fragment_index_guards():
    rng = random.Random(4)
    frag_data, offsets = oracle.pack_fragment_files(_files(rng, 3))
    fidx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    sectors = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    sidx = carve.build_master_index(sectors, [0, 8])
    with pytest.raises(carve.CarveError):
        carve.scan_image(fidx, sectors)
    with pytest.raises(carve.CarveError):
        carve.scan_fragments(sidx, sectors)
    with pytest.raises(carve.CarveError):
        carve.scan_batch(fidx, [(sectors, 0, 0)])
    with pytest.raises(carve.CarveError):
        carve.Server(fidx)
    with pytest.raises(carve.CarveError):
        carve.scan_fragments(fidx, sectors[1:])                # misaligned
    # fragments use djb2-64: a CRC index of fragments is refused
    lib = carve.load_library()
    h = carve.ctypes.c_void_p()
    p = carve._IndexParams(carve.CARVE_SIG_CRC64_ISO, 0.0, 0, 0)
    off = np.array([0, 8], np.uint64)
    rc = lib.build_fragment_index(sectors.data_ptr(), off.ctypes.data, 1, carve.ctypes.byref(p), None,
                                  carve.ctypes.byref(h))
    assert rc == carve.CARVE_EUNSUPPORTED and not h.value


def test_fragment_workload_scaled():
    """The benchmark's recipe (logo files embedded in random bytes) at 32 MiB."""
    import dataclasses

    import synth
    cfg = dataclasses.replace(synth.FRAGMENT_CONFIGS["logos"], n_files=200, image_bytes=(32 << 20) + 50,
                              n_embedded=1500)
    files = synth.fragment_files(cfg, device="cuda")
    frags, offsets = carve.pack_fragment_files(files)
    img = synth.fragment_image(cfg, files, device="cuda")
    idx = carve.build_fragment_index(frags, offsets)
    f, m, _ = _gpu(idx, img)
    wf, wm = _oracle(frags.cpu().numpy(), offsets, img.cpu().numpy().tobytes())
    assert len(wm) > 10000
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_fragment_workload_full():
    """The benchmark's workload at its full size (2 GiB image, 346,577
    fragments of 2,000 files, the 160 KiB LDS filter and the 2 MiB Bloom
    filter), scanned as bench.py times it: every window's flag and every
    confirmed record equal the oracle's over the whole image."""
    import synth
    cfg = synth.FRAGMENT_CONFIGS["logos"]
    files = synth.fragment_files(cfg, device="cuda")
    frags, offsets = carve.pack_fragment_files(files)
    img = synth.fragment_image(cfg, files, device="cuda")
    idx = carve.build_fragment_index(frags, offsets)
    f, m, _ = _gpu(idx, img)
    host = img.cpu().numpy()
    del img
    ox = oracle.FragmentIndex(frags.cpu().numpy(), offsets, threads=oracle.default_threads())
    wf = ox.flag_windows(host, threads=oracle.default_threads())
    wm = ox.confirm_windows(host, wf)
    assert len(wf) > 3_000_000
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


def test_fragment_workload_chunk_boundary():
    """The benchmark's recipe on an image of 2^30 + 132 bytes: 268,435,474
    windows, so the compaction's hit words make 4,097 chunks of 1,024 and the
    one-block scan of their sums takes a second pass of a single sum (passes
    of 4,096). Every flag and record against the oracle."""
    import dataclasses

    import synth
    cfg = dataclasses.replace(synth.FRAGMENT_CONFIGS["logos"], image_bytes=(1 << 30) + 132, n_embedded=12500)
    n_words = -(-((cfg.image_bytes - 64) // 4 + 1) // 64)   # hit words of 64 windows
    assert -(-n_words // 1024) == 4097
    files = synth.fragment_files(cfg, device="cuda")
    frags, offsets = carve.pack_fragment_files(files)
    img = synth.fragment_image(cfg, files, device="cuda")
    idx = carve.build_fragment_index(frags, offsets)
    f, m, _ = _gpu(idx, img)
    host = img.cpu().numpy()
    del img
    ox = oracle.FragmentIndex(frags.cpu().numpy(), offsets, threads=oracle.default_threads())
    wf = ox.flag_windows(host, threads=oracle.default_threads())
    wm = ox.confirm_windows(host, wf)
    assert len(wf) > 1_000_000
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)


@pytest.mark.parametrize("bloom", [0, carve.CARVE_BLOOM_OFF])
@pytest.mark.parametrize("zero_master", [True, False])
def test_fragment_signature_low_halves(bloom, zero_master):
    """The scan filters windows on a 32-bit key taken from their signature
    (the low half of the signature's data part: the signature minus
    5381 * 33^64, modulo 2^32) and takes the exact 64-bit test only for those
    that pass: master fragments whose signature is 0 (it lives beside the
    table), whose low half is 0, 1 or 2^32 - 1, or whose key is 0, 1 or
    2^32 - 1, with other high halves; windows equal to them, windows crafted
    to their signatures with other bytes (flagged, not confirmed), and windows
    that share only a low half (not flagged); against the oracle."""
    from oracle import spec
    rng = random.Random(77 + zero_master)
    key0 = (5381 * pow(33, 64, 1 << 64)) & 0xFFFFFFFF   # the low half whose key is 0
    targets = [(1 << 32) * 5, (1 << 32) * 12345 + 1, (1 << 64) - 1, ((1 << 31) + 7) << 32 | 0xFFFFFFFF,
               (1 << 32) * 777 + key0, (1 << 32) * 31 + key0 + 1, (1 << 32) * 90001 + key0 - 1]
    if zero_master:
        targets.append(0)
    crafted = [spec.craft_sector(bytes([65 + i]) * 8, t, n=64) for i, t in enumerate(targets)]
    assert [spec.djb2_closed(c) for c in crafted] == targets
    files = _files(rng, 5, 128, 1024)
    files.append(b"".join(crafted) + bytes(rng.getrandbits(8) for _ in range(64)))
    frag_data, offsets = oracle.pack_fragment_files(files)
    # same low half, another high half: never flagged
    others = [spec.craft_sector(b"other" + bytes([i]), (t ^ (0xDEAD << 40)) & ((1 << 64) - 1), n=64)
              for i, t in enumerate(targets)]
    collisions = [spec.craft_sector(b"collide" + bytes([i]), t, n=64) for i, t in enumerate(targets)]
    img = bytearray(rng.getrandbits(8) for _ in range(64 * 1024))
    pieces = crafted + others + collisions
    for k, p in enumerate(pieces):
        o = 4096 + 1024 * k + 4 * (k % 7)
        img[o:o + 64] = p
    image = bytes(img)
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets, bloom_bits_per_key=bloom)
    f, m, _ = _gpu(idx, dev_bytes(image))
    wf, wm = _oracle(frag_data, offsets, image)
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    flagged = set(f.tolist())
    for k in range(len(pieces)):
        j = (4096 + 1024 * k + 4 * (k % 7)) // 4
        if k < len(crafted):
            assert j in flagged and j in set(m["disk_sector"].tolist())
        elif k < 2 * len(crafted):
            assert j not in flagged
        else:
            assert j in flagged and j not in set(m["disk_sector"].tolist())


@pytest.mark.parametrize("after", ["scan", "kernel"])
def test_two_steps_in_flight(after):
    """Two scan objects on two streams sharing one index, as bench.py runs the
    fragment step: step i runs wholly on stream i % 2 (scan, records into a
    device buffer, ids copy, count readback), its scan ordered after step
    i-1's scan, either by an event after scan_fragments (its kernel and
    compaction) or by scan_wait_kernel (its kernel alone), so step i-1's
    confirmation (and compaction) run beside step i's scan; the host reads
    step i-1's counts after enqueuing step i. Each step scans other bytes;
    ids and records equal the oracle's for that step."""
    rng = random.Random(21)
    files = _files(rng, 200, 256, 8192)
    frag_data, offsets = oracle.pack_fragment_files(files)
    idx = carve.build_fragment_index(dev_bytes(frag_data.tobytes()), offsets)
    images, expect = [], []
    for k in range(6):
        n = (2 << 20) + 4 * k + (k % 3)                      # ragged lengths
        img = bytearray(np.random.default_rng(100 + k).integers(0, 256, size=n, dtype=np.uint8).tobytes())
        o = 0
        while o < n - 10000:
            data = files[rng.randrange(len(files))]
            o += rng.randrange(100, 9000)
            o -= o % 4 if rng.random() < 0.7 else 0
            img[o:o + len(data)] = data
            o += len(data)
        images.append(dev_bytes(bytes(img)))
        expect.append(_oracle(frag_data, offsets, bytes(img)))
    most_f = max(len(f) for f, _ in expect)
    most_m = max(len(m) for _, m in expect)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    scans, events = [None, None], [torch.cuda.Event(), torch.cuda.Event()]
    ids = [torch.full((most_f + 7,), -1, dtype=torch.int64, device="cuda") for _ in range(2)]
    rec = [torch.zeros(16 * (most_m + 7), dtype=torch.uint8, device="cuda") for _ in range(2)]

    def check(i):
        k = i % 2
        wf, wm = expect[i]
        assert carve.scan_counts(scans[k]) == (len(wf), len(wm))
        assert np.array_equal(ids[k][: len(wf)].cpu().numpy().astype(np.uint64), wf)
        got = np.frombuffer(rec[k].cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)[: len(wm)]
        assert_same_matches(got, wm)

    for i in range(len(images)):
        k = i % 2
        with torch.cuda.stream(streams[k]):
            if i > 0:
                if after == "kernel":
                    carve.scan_wait_kernel(scans[1 - k], streams[k])
                else:
                    streams[k].wait_event(events[1 - k])
            scans[k] = carve.scan_fragments(idx, images[i], scan=scans[k])
            events[k].record(streams[k])
            carve.confirm_enqueue(idx, scans[k], rec[k])
            carve.flagged_sectors_enqueue(scans[k], ids[k])
        if i > 0:
            check(i - 1)
    check(len(images) - 1)
