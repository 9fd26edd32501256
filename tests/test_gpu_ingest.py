"""Host ingest (the paper's double-buffered pipeline): an image in host memory,
pinned or pageable, scanned chunk by chunk gives exactly the flags and matches
of the same image scanned in device memory, and of the CPU oracle."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import assert_same_matches, gpu_flags_and_matches, oracle_flags_and_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["tiny"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    return ms, img.data, idx


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("chunk,n_bytes", [(1 << 20, (7 << 20) + 4096 * 3 + 700), (4 << 20, 64 << 20),
                                           (64 << 20, (64 << 20) - 5), (4096, 40960 + 512)])
def test_ingest_equals_device_scan(tiny, pinned, chunk, n_bytes):
    ms, dev, idx = tiny
    host = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=pinned)
    host.copy_(dev[:n_bytes].cpu())
    ing = carve.Ingest(idx, chunk_bytes=chunk)
    for tau0, mode in ((0, carve.CARVE_TAU_PER_CLUSTER), (5, carve.CARVE_TAU_PER_CLUSTER), (0, carve.CARVE_TAU_ANY)):
        ing.scan(host, tau0, mode)
        st = ing.stats()
        assert st["pinned_source"] == int(pinned) and st["bytes"] == n_bytes // 512 * 512
        assert st["chunks"] == -(-(n_bytes // 512 * 512) // chunk)
        f, m, _ = gpu_flags_and_matches(idx, dev[:n_bytes], tau0, mode == carve.CARVE_TAU_ANY)
        assert np.array_equal(ing.flagged(), f)
        assert_same_matches(ing.matches(), m)
    ing.close()


def test_ingest_against_oracle(tiny):
    ms, dev, idx = tiny
    n = (3 << 20) + 1000
    host = dev[:n].cpu()
    ing = carve.Ingest(idx, chunk_bytes=1 << 18)
    ing.scan(host)
    wf, wm = oracle_flags_and_matches(ms.sectors.cpu().numpy(), ms.file_offsets, host.numpy())
    assert len(wf) > 100
    assert np.array_equal(ing.flagged(), wf)
    assert_same_matches(ing.matches(), wm)
    ing.close()


def test_ingest_edges_and_errors(tiny):
    ms, dev, idx = tiny
    ing = carve.Ingest(idx, chunk_bytes=8192, confirm=False)
    ing.scan(torch.empty(0, dtype=torch.uint8))
    assert ing.flagged().size == 0 and ing.stats()["chunks"] == 0
    ing.scan(dev[:511].cpu())
    assert ing.flagged().size == 0
    ing.scan(dev[: 1 << 20].cpu())
    f, _, _ = gpu_flags_and_matches(idx, dev[: 1 << 20])
    assert np.array_equal(ing.flagged(), f) and ing.matches().size == 0      # confirmation off
    ing.close()
    with pytest.raises(carve.CarveError):
        carve.Ingest(idx, chunk_bytes=5000)                                  # not a multiple of 4096
    with pytest.raises(carve.CarveError):
        carve.Ingest(idx, copy_threads=65)
    ing = carve.Ingest(idx, chunk_bytes=1 << 16)
    with pytest.raises(carve.CarveError):
        ing.scan(dev[: 1 << 16].cpu(), tau0=8)
    ing.close()
