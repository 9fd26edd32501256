"""Helpers shared by the GPU tests (not collected)."""
import numpy as np
import torch

import oracle
from paper_0901_1307_amd import carve

SECTOR = 512


def dev_bytes(b: bytes) -> torch.Tensor:
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda() if b else torch.empty(0, dtype=torch.uint8,
                                                                                         device="cuda")


def gpu_flags_and_matches(index, image: torch.Tensor, tau0=0, any_tau=False, scan=None):
    mode = carve.CARVE_TAU_ANY if any_tau else carve.CARVE_TAU_PER_CLUSTER
    sc = carve.scan_image(index, image, tau0=tau0, tau_mode=mode, scan=scan)
    flags = carve.flagged_sectors(sc).numpy().astype(np.uint64)
    matches = carve.confirm_matches(index, sc)
    return flags, matches, sc


def oracle_flags_and_matches(masters_host, offsets, image_host, tau0=0, any_tau=False, threads=None,
                             sig_kind=oracle.SIG_DJB2):
    th = threads or oracle.default_threads()
    ix = oracle.Index(masters_host, offsets, threads=th, sig_kind=sig_kind)
    flags = ix.flag_image(image_host, tau0, any_tau, threads=th)
    matches = ix.confirm_image(image_host, flags, tau0, any_tau)
    return flags, matches


def assert_same_matches(got, want):
    assert got.dtype == want.dtype or got.dtype.names == want.dtype.names
    assert len(got) == len(want), (len(got), len(want))
    for f in ("disk_sector", "file_id", "sector_in_file"):
        assert np.array_equal(got[f], want[f]), f
