"""The oracle on the synthetic workloads: brute force at the tiny configuration's
full size, and the generator's planted ground truth."""
import numpy as np
import pytest
import torch

import oracle
import synth


def _tuples(arr):
    return set(zip(arr["disk_sector"].tolist(), arr["file_id"].tolist(), arr["sector_in_file"].tolist()))


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["tiny"]
    ms = synth.master_set(cfg)
    img = synth.disk_image(cfg, ms)
    return cfg, ms, img


def _planted(ms, img):
    """(disk sector, file, sector in file) of every planted, non-overwritten sector."""
    off = ms.file_offsets
    out = set()
    for c, src, r in zip(img.planted_clusters.tolist(), img.planted_src.tolist(), img.planted_overwrite.tolist()):
        f = max(i for i in range(len(off) - 1) if off[i] <= src)
        for i in range(r, 8):
            out.add((8 * c + i, f, src - off[f] + i))
    return out


@pytest.mark.slow
def test_tiny_full_size_bruteforce(tiny):
    """Confirmed set == all-pairs byte comparison of 131072 x 4096 sectors; every
    byte-equal sector is flagged; the planted sectors are found."""
    cfg, ms, img = tiny
    th = oracle.default_threads()
    ix = oracle.Index(ms.sectors, ms.file_offsets, threads=th)
    flags = ix.flag_image(img.data, threads=th)
    conf = ix.confirm_image(img.data, flags)
    brute = oracle.bruteforce(img.data, ms.sectors, ms.file_offsets, threads=th)
    assert np.array_equal(conf, brute)
    assert set(brute["disk_sector"].tolist()) <= set(flags.tolist())
    assert _planted(ms, img) <= _tuples(conf)
    # duplicated master sectors produce multi-hit matches
    assert len(conf) > len(set(conf["disk_sector"].tolist()))


def test_generator_regenerates_sectors(tiny):
    cfg, ms, img = tiny
    ids = torch.tensor([0, 1, 7, 8, 4095, 65536, 131071], dtype=torch.int64)
    assert torch.equal(synth.disk_sectors(cfg, ms, ids), img.data.view(-1, 512)[ids])
    mids = torch.tensor([0, 511, 512, 4095], dtype=torch.int64)
    assert torch.equal(synth.master_sectors(ms, mids), ms.sectors[mids])


def test_generator_recipe(tiny):
    cfg, ms, img = tiny
    n_cl = cfg.n_disk_sectors // 8
    assert sum(img.kind_counts.values()) == n_cl
    assert abs(img.kind_counts[synth.workloads.KIND_MASTER] / n_cl - 0.05) < 0.01
    assert abs(img.kind_counts[synth.workloads.KIND_ZERO] / n_cl - 0.02) < 0.005
    ow = img.planted_overwrite
    assert abs(float((ow > 0).float().mean()) - 0.5) < 0.08
    assert set(ow.tolist()) <= {0, 1, 2, 3}
    assert len(ms.dup_dst) == 16
    # 8 duplicates at the same cluster position, 8 at another one
    off = ms.file_offsets
    tau = lambda s: (s - off[max(i for i in range(len(off) - 1) if off[i] <= s)]) % 8  # noqa: E731
    same = sum(tau(d) == tau(s) for d, s in zip(ms.dup_dst.tolist(), ms.dup_src.tolist()))
    assert same == 8


def test_oracle_sampled_flags_match_full(tiny):
    """Flags of sampled sectors given one by one equal the full-image flags."""
    cfg, ms, img = tiny
    ix = oracle.Index(ms.sectors, ms.file_offsets, threads=2)
    flags = set(ix.flag_image(img.data, threads=2).tolist())
    g = torch.Generator().manual_seed(0)
    ids = torch.randint(0, cfg.n_disk_sectors, (2000,), generator=g)
    ids = torch.cat([ids, torch.tensor(sorted(flags)[:200])])
    secs = synth.disk_sectors(cfg, ms, ids)
    got = ix.flag_sectors(secs, ids.numpy().astype(np.uint64))
    assert got.tolist() == [int(j) in flags for j in ids.tolist()]
