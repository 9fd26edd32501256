"""The served workload at its full size, through the server in the
configuration bench.py times (2 stream lanes, a 32 GiB admission budget,
confirmation on, the index's default launch shape): every job of the
60-second Poisson stream at 2000 jobs/s (about 120,000 jobs, 64 KiB-256 MiB,
flow buffers under 1 MiB matched at any position) is submitted at once, the
server batches them as lanes free up, and each job's flags and records are
compared with the CPU oracle.

Jobs are slices of one 2 GiB device pool. Under Section 3.1's rule a
sector's flag and its matches depend only on its bytes and its cluster
position, and a job starting at pool sector `first` with tau0 = first mod 8
gives its sector j the pool sector first + j's position. So the oracle flags
and confirms the pool once per rule, and each job's expected results are the
pool's restricted to [first, first + n) and shifted by first. That identity
is pinned on a sample of jobs by running the oracle on their own bytes."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_same_matches
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512


def _log(*a):
    print(*a, flush=True)


def _restrict(flags, recs, first, n):
    lo, hi = np.searchsorted(flags, [first, first + n])
    f = flags[lo:hi] - np.uint64(first)
    mlo, mhi = np.searchsorted(recs["disk_sector"], [first, first + n])
    m = recs[mlo:mhi].copy()
    m["disk_sector"] -= np.uint64(first)
    return f, m


def test_served_workload_every_job_exact():
    cfg = synth.CONFIGS["served"]
    _log("[served] generating the master set and the 2 GiB pool on the GPU")
    ms = synth.master_set(cfg, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    pool = synth.disk_image(cfg, ms, device="cuda").data
    pool_sectors = pool.numel() // SECTOR
    specs = synth.served_job_specs(cfg.seed, rate=2000.0, duration=60.0)
    firsts = synth.served_job_slices(specs, pool_sectors, cfg.seed)
    jobs = []
    for (_, size, flow), first in zip(specs, firsts):
        jobs.append((pool[first * SECTOR: first * SECTOR + size], 0 if flow else first % 8,
                     carve.CARVE_TAU_ANY if flow else carve.CARVE_TAU_PER_CLUSTER))
    assert len(jobs) > 100_000 and any(m == carve.CARVE_TAU_ANY for _, _, m in jobs)
    _log(f"[served] {len(jobs)} jobs, {sum(t.numel() for t, _, _ in jobs) / 1e12:.2f} TB; oracle over the pool")
    th = oracle.default_threads()
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=th)
    host = pool.cpu().numpy()
    want = {}
    for mode in (carve.CARVE_TAU_PER_CLUSTER, carve.CARVE_TAU_ANY):
        f = ox.flag_image(host, 0, mode == carve.CARVE_TAU_ANY, threads=th)
        want[mode] = (f, ox.confirm_image(host, f, 0, mode == carve.CARVE_TAU_ANY))
    # the restriction identity, pinned on the smallest, the largest and random jobs
    order = np.argsort([t.numel() for t, _, _ in jobs])
    sample = set(order[:16].tolist()) | set(order[-8:].tolist()) | set(
        np.random.default_rng(5).choice(len(jobs), 40, replace=False).tolist())
    for k in sorted(sample):
        t, tau0, mode = jobs[k]
        jh = t.cpu().numpy()
        f = ox.flag_image(jh, tau0, mode == carve.CARVE_TAU_ANY, threads=th)
        rf, rm = _restrict(*want[mode], firsts[k], t.numel() // SECTOR)
        assert np.array_equal(f, rf), k
        assert_same_matches(ox.confirm_image(jh, f, tau0, mode == carve.CARVE_TAU_ANY), rm)
    _log("[served] submitting every job to the server")
    srv = carve.Server(idx, n_streams=2, budget_bytes=32 << 30, confirm=True)
    ids = srv.submit_many(carve.image_descs(jobs))
    job_of = {int(j): k for k, j in enumerate(ids.tolist())}
    n_done = n_flag = n_match = 0
    while n_done < len(jobs):
        d = srv.poll_array()
        for r in d:
            assert r["status"] == carve.CARVE_OK
            jid = int(r["job_id"])
            k = job_of[jid]
            t, tau0, mode = jobs[k]
            wf, wm = _restrict(*want[mode], firsts[k], t.numel() // SECTOR)
            assert int(r["n_flagged"]) == len(wf) and int(r["n_confirmed"]) == len(wm), k
            assert np.array_equal(srv.flags(jid), wf), k
            assert_same_matches(srv.matches(jid), wm)
            n_flag += len(wf)
            n_match += len(wm)
        if len(d):
            srv.release_many(d["job_id"])
            n_done += len(d)
    st = srv.stats()
    srv.close()
    assert st["jobs_completed"] == len(jobs) and st["batches_launched"] > 1
    assert n_flag > 0 and n_match > 0
    _log(f"[served] every job bit-exact: {n_flag} flags, {n_match} matches in {st['batches_launched']} batches")
