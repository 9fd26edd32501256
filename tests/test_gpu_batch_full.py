"""The batched workload at its full size, in the launch configuration bench.py
times: the 256 images of log-uniform sizes 1 MiB-1 GiB (about 47 GiB) against
the mid master set, the index and launch shape autotune_index picks (for
contiguous scans) on a tuning sample,
one persistent scan_batch launch replayed from a HIP graph, then the per-image
counts, ids and confirmation. Every image's flags and records are compared
with the CPU oracle run on that image (Section 3.1: flag by the signature sets
S_tau, then confirm byte for byte)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512


def _log(*a):
    print(*a, flush=True)


def test_batched_full_size_exact():
    cfg = synth.CONFIGS["mid"]
    _log("[batched] generating 256 images on the GPU")
    ms = synth.master_set(cfg, device="cuda")
    images = synth.batch_images(cfg, ms, device="cuda")
    total = sum(t.numel() for t in images)
    assert len(images) == 256 and total > 40 << 30
    idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets,
                                     synth.tuning_sample(cfg, ms, device="cuda", max_sectors=1 << 24),
                                     contiguous_only=True)
    _log(f"[batched] {total / 2**30:.1f} GiB, pick {pick}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = carve.scan_batch(idx, images)
        carve.batch_flag_counts(b)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            carve.scan_batch(idx, images, batch=b)
        graph.replay()
        counts = carve.batch_flag_counts(b).astype(np.int64)
        ids = carve.batch_flagged_sectors(b, carve.CARVE_ALL_IMAGES).numpy().astype(np.uint64)
        bm = carve.batch_confirm_matches(idx, b)
    torch.cuda.synchronize()
    assert len(ids) == counts.sum()
    _log(f"[batched] GPU: {len(ids)} flagged, {len(bm)} confirmed; running the oracle image by image")
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    starts = np.concatenate([[0], np.cumsum(counts)])
    mstart = np.searchsorted(bm["image"], np.arange(len(images) + 1), side="left")
    n_flag = n_match = 0
    for i, t in enumerate(images):
        host = t.cpu().numpy()
        wf = ox.flag_image(host, 0, False, threads=th)
        wm = ox.confirm_image(host, wf, 0, False)
        got_f = ids[starts[i]: starts[i + 1]]
        assert np.array_equal(got_f, wf), i
        got_m = bm[mstart[i]: mstart[i + 1]]
        assert len(got_m) == len(wm), i
        for f in ("disk_sector", "file_id", "sector_in_file"):
            assert np.array_equal(got_m[f], wm[f]), (i, f)
        n_flag += len(wf)
        n_match += len(wm)
    assert n_flag == len(ids) and n_match == len(bm)
    assert np.all(np.diff(bm["image"].astype(np.int64)) >= 0)
    _log(f"[batched] bit-exact on every image: {n_flag} flags, {n_match} matches")
