"""Batched scans: many uneven images in one launch give exactly the results of
scanning each image alone (and of the CPU oracle)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_same_matches, gpu_flags_and_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512


@pytest.fixture(scope="module")
def setup():
    cfg = synth.scaled(synth.CONFIGS["mid"], n_master_sectors=20000, n_disk_sectors=1, n_files=40)
    ms = synth.master_set(cfg, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    # uneven images: empty, sub-sector, one sector, ragged tails, a few thousand tiles
    sizes = [0, 100, 512, 511 + 512 * 3, 64 * 512, 64 * 512 + 7, 1 << 20, 5 * (1 << 20) + 4096 + 13, 3 << 20]
    images = []
    for i, nb in enumerate(sizes):
        n = max(nb // SECTOR, 1)
        c = synth.scaled(cfg, n_master_sectors=cfg.n_master_sectors, n_disk_sectors=n,
                         p_master_cluster=0.05 * (i % 3), tail_bytes=0)
        img = synth.disk_image(c, ms, device="cuda", image_id=i).data
        buf = torch.zeros(max(nb, 16), dtype=torch.uint8, device="cuda")
        k = min(nb, img.numel())
        buf[:k] = img[:k]
        images.append((buf[:nb] if nb else buf[:0], i % 8, carve.CARVE_TAU_ANY if i % 4 == 3 else 0))
    return ms, idx, images


def _alone(idx, images):
    out = []
    for t, tau0, mode in images:
        f, m, _ = gpu_flags_and_matches(idx, t, tau0, mode == carve.CARVE_TAU_ANY)
        out.append((f, m))
    return out


def _check_batch(idx, b, alone):
    counts = carve.batch_flag_counts(b)
    assert counts.tolist() == [len(f) for f, _ in alone]
    for i, (f, _) in enumerate(alone):
        assert np.array_equal(carve.batch_flagged_sectors(b, i).numpy().astype(np.uint64), f)
    bm = carve.batch_confirm_matches(idx, b)
    want = [(i, int(r["disk_sector"]), int(r["file_id"]), int(r["sector_in_file"]))
            for i, (_, m) in enumerate(alone) for r in m]
    got = list(zip(bm["image"].tolist(), bm["disk_sector"].tolist(), bm["file_id"].tolist(),
                   bm["sector_in_file"].tolist()))
    assert got == want


def test_batch_equals_images_alone(setup):
    ms, idx, images = setup
    alone = _alone(idx, images)
    assert sum(len(f) for f, _ in alone) > 100
    b = carve.scan_batch(idx, images)
    _check_batch(idx, b, alone)
    # and the oracle agrees with the images alone
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=oracle.default_threads())
    for (t, tau0, mode), (f, m) in zip(images, alone):
        host = t.cpu().numpy()
        wf = ox.flag_image(host, tau0, mode == carve.CARVE_TAU_ANY, threads=4)
        assert np.array_equal(f, wf)
        assert_same_matches(m, ox.confirm_image(host, wf, tau0, mode == carve.CARVE_TAU_ANY))


@pytest.mark.parametrize("blocks_per_cu,tiles_per_chunk", [(0, 1), (1, 1), (2, 4), (3, 16), (0, 64)])
def test_batch_launch_shapes(setup, blocks_per_cu, tiles_per_chunk):
    """The launch shape never changes a result."""
    ms, idx, images = setup
    base = idx.scan_config()
    alone = _alone(idx, images)
    try:
        idx.set_scan_config(blocks_per_cu, tiles_per_chunk)
        _check_batch(idx, carve.scan_batch(idx, images), alone)
        for (t, tau0, mode), (f, _) in zip(images, alone):
            g, _, _ = gpu_flags_and_matches(idx, t, tau0, mode == carve.CARVE_TAU_ANY)
            assert np.array_equal(g, f)
    finally:
        idx.set_scan_config(base["blocks_per_cu"], base["tiles_per_chunk"])


def test_autotune_keeps_results(setup):
    ms, idx, images = setup
    alone = _alone(idx, images)
    best = idx.autotune(images[-1][0])
    assert idx.scan_config() == best
    _check_batch(idx, carve.scan_batch(idx, images), alone)


def test_batch_reuse_and_graph_replay(setup):
    """A reused batch with unchanged descriptors enqueues only kernels, so it can
    be captured in a HIP graph; every replay equals the eager result."""
    ms, idx, images = setup
    alone = _alone(idx, images)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = carve.scan_batch(idx, images)
        torch.cuda.synchronize()
        carve.confirm_enqueue(idx, b)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):   # the whole hot path: scan and confirmation
            carve.scan_batch(idx, images, batch=b)
            carve.confirm_enqueue(idx, b)
    for rep in range(4):
        # eager work between replays, then the replay and its check
        carve.scan_batch(idx, images[::-1] if rep % 2 else images[:3], batch=carve.Batch())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_batch(idx, b, alone)


def _plant(ms, image, rep, tau0):
    """New bytes in place: the first 16 sectors of master file 0 at a sector
    of the image whose cluster position is 0 (a different one each time)."""
    p = 64 * (rep + 1) + (-tau0) % 8
    image[p * 512:(p + 16) * 512] = ms.sectors.reshape(-1)[:16 * 512]


def test_graph_of_scan_only_confirms_each_replay(setup):
    """A graph that captures only the scan: the confirmation asked for after a
    replay is that of the bytes the replay scanned, also when the batch object
    was confirmed before (a replay runs no host code)."""
    ms, idx, images = setup
    imgs = [(t.clone(), tau0, mode) for t, tau0, mode in images]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = carve.scan_batch(idx, imgs)
        carve.batch_confirm_matches(idx, b)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            carve.scan_batch(idx, imgs, batch=b)
    big, tau0, _ = imgs[6]
    for rep in range(4):
        _plant(ms, big, rep, tau0)
        if rep == 3:
            with torch.cuda.stream(stream):
                carve.confirm_enqueue(idx, b)      # confirmed before the replay
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_batch(idx, b, _alone(idx, imgs))


def test_graph_of_scan_image_confirms_each_replay(setup):
    """The same for one image: scan_image captured alone, confirm_matches after
    each replay over new bytes equals a fresh scan of them."""
    ms, idx, images = setup
    t, tau0, mode = images[6]
    img = t.clone()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sc = carve.scan_image(idx, img, tau0=tau0, tau_mode=mode)
        carve.confirm_matches(idx, sc)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            carve.scan_image(idx, img, tau0=tau0, tau_mode=mode, scan=sc)
    for rep in range(3):
        _plant(ms, img, rep, tau0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        f, m, _ = gpu_flags_and_matches(idx, img, tau0, mode == carve.CARVE_TAU_ANY)
        assert np.array_equal(carve.flagged_sectors(sc).numpy().astype(np.uint64), f)
        assert_same_matches(carve.confirm_matches(idx, sc), m)
        assert len(m) >= 16


def test_graph_of_one_wait_step(setup):
    """scan_image, the confirmation into a device buffer and the ids copy
    captured in one graph: every replay over new bytes gives the oracle's ids
    and records (read with one scan_counts). The single-pass kernels leave
    their state clean on every replay; eager scans of other sizes run between
    the replays."""
    ms, idx, images = setup
    t, tau0, mode = images[7]
    img = t.clone()
    any_tau = mode == carve.CARVE_TAU_ANY
    n_units = img.numel() // SECTOR
    ids = torch.empty(n_units, dtype=torch.int64, device="cuda")
    rec = torch.empty(16 * (4 * n_units + 1024), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sc = carve.scan_image(idx, img, tau0=tau0, tau_mode=mode)
        carve.confirm_enqueue(idx, sc, rec)
        carve.flagged_sectors_enqueue(sc, ids)
        carve.scan_counts(sc)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            carve.scan_image(idx, img, tau0=tau0, tau_mode=mode, scan=sc)
            carve.confirm_enqueue(idx, sc, rec)
            carve.flagged_sectors_enqueue(sc, ids)
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets)
    for rep in range(4):
        _plant(ms, img, rep, tau0)
        other, o_tau0, o_mode = images[(5, 8, 6, 4)[rep]]
        gpu_flags_and_matches(idx, other, o_tau0, o_mode == carve.CARVE_TAU_ANY)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        nf, nm = carve.scan_counts(sc)
        host = img.cpu().numpy()
        wf = ox.flag_image(host, tau0, any_tau)
        wm = ox.confirm_image(host, wf, tau0, any_tau)
        assert (nf, nm) == (len(wf), len(wm)) and nm >= 16
        assert np.array_equal(ids[:nf].cpu().numpy().astype(np.uint64), wf)
        got = np.frombuffer(rec[: 16 * nm].cpu().numpy().tobytes(), dtype=carve.MATCH_DTYPE)
        assert_same_matches(got, wm)


def test_batch_rejects_bad_descriptor(setup):
    ms, idx, images = setup
    bad = list(images)
    t = bad[6][0]
    bad[6] = (t[1:], 0, 0)                     # misaligned
    with pytest.raises(carve.CarveError) as e:
        carve.scan_batch(idx, bad)
    assert e.value.code == carve.CARVE_EINVAL and "image 6" in str(e.value)
    bad[6] = (images[6][0], 9, 0)              # tau0 out of range
    with pytest.raises(carve.CarveError):
        carve.scan_batch(idx, bad)
    # a good batch still works afterwards
    _check_batch(idx, carve.scan_batch(idx, images), _alone(idx, images))


def test_empty_batch(setup):
    ms, idx, images = setup
    b = carve.scan_batch(idx, [])
    assert carve.batch_flag_counts(b).size == 0
    assert len(carve.batch_confirm_matches(idx, b)) == 0
