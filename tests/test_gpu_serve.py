"""The serving loop: every job's flags and records in the mix equal the CPU
oracle's on that job's own bytes (Section 3.1: flag by S_tau, confirm byte for
byte) and the job scanned and confirmed alone; admission respects the byte
budget."""
import random

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
def pool():
    cfg = synth.scaled(synth.CONFIGS["served"], n_master_sectors=100_000, n_disk_sectors=1 << 19, n_files=300)
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda").data        # 256 MiB pool
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    ox = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=oracle.default_threads())
    return ms, idx, img, ox


def _check_job(srv, jid, done_counts, ox, idx, t, tau0, mode, given=None):
    """A served job against the oracle on its own bytes (`given`: the host
    tensor the server was handed, else the device tensor t) and against the
    job scanned alone on the GPU (t)."""
    any_tau = mode == carve.CARVE_TAU_ANY
    host = (t if given is None else given).cpu().numpy()
    wf = ox.flag_image(host, tau0, any_tau, threads=oracle.default_threads())
    wm = ox.confirm_image(host, wf, tau0, any_tau)
    assert done_counts == (len(wf), len(wm))
    assert np.array_equal(srv.flags(jid), wf)
    assert_same_matches(srv.matches(jid), wm)
    f, m, _ = gpu_flags_and_matches(idx, t, tau0, any_tau)
    assert np.array_equal(f, wf)
    assert_same_matches(m, wm)
    return len(wf)


def _jobs(img, n, seed, max_bytes=8 << 20):
    rng = random.Random(seed)
    jobs = []
    for _ in range(n):
        size = int(np.exp(rng.uniform(np.log(64 << 10), np.log(max_bytes)))) // SECTOR * SECTOR + rng.choice([0, 77])
        flow = size < (1 << 20)
        first = rng.randrange(0, img.numel() // SECTOR - size // SECTOR - 1)
        if not flow and rng.random() < 0.5:
            first -= first % 8                                    # cluster-aligned chunk
        t = img[first * SECTOR: first * SECTOR + size]
        jobs.append((t, 0 if flow else first % 8, carve.CARVE_TAU_ANY if flow else carve.CARVE_TAU_PER_CLUSTER))
    return jobs


def _drain(srv, ids):
    done = {}
    while len(done) < len(ids):
        for jid, nf, nc, st in srv.poll():
            assert st == carve.CARVE_OK
            done[jid] = (nf, nc)
    return done


@pytest.mark.parametrize("n_streams,budget", [(4, 0), (2, 24 << 20), (1, 0)])
def test_served_equals_alone(pool, n_streams, budget):
    ms, idx, img, ox = pool
    jobs = _jobs(img, 60, seed=n_streams)
    srv = carve.Server(idx, n_streams=n_streams, budget_bytes=budget)
    ids = [srv.submit(t, tau0, mode) for t, tau0, mode in jobs]
    done = _drain(srv, ids)
    st = srv.stats()
    assert st["jobs_completed"] == len(jobs) and st["in_flight_bytes"] == 0
    assert st["batches_launched"] >= 1
    total_flags = 0
    for jid, (t, tau0, mode) in zip(ids, jobs):
        total_flags += _check_job(srv, jid, done[jid], ox, idx, t, tau0, mode)
        srv.release(jid)
    assert total_flags > 0
    srv.close()


def test_jobs_arriving_while_others_run(pool):
    """Jobs submitted between polls join later batches; results are unchanged."""
    ms, idx, img, ox = pool
    jobs = _jobs(img, 80, seed=9)
    srv = carve.Server(idx, n_streams=3)
    ids, done = [], {}
    for k, (t, tau0, mode) in enumerate(jobs):
        ids.append(srv.submit(t, tau0, mode))
        if k % 3 == 0:
            for jid, nf, nc, st in srv.poll():
                done[jid] = (nf, nc)
    done.update(_drain(srv, [i for i in ids if i not in done]))
    assert srv.stats()["batches_launched"] > 1
    for jid, (t, tau0, mode) in zip(ids, jobs):
        _check_job(srv, jid, done[jid], ox, idx, t, tau0, mode)
    srv.close()


def test_budget_and_errors(pool):
    ms, idx, img, ox = pool
    srv = carve.Server(idx, n_streams=2, budget_bytes=1 << 20)
    with pytest.raises(carve.CarveError) as e:
        srv.submit(img[: 2 << 20])                               # larger than the whole budget
    assert e.value.code == carve.CARVE_EUNSUPPORTED
    with pytest.raises(carve.CarveError):
        srv.submit(img[1: 1 + 4096])                             # misaligned
    with pytest.raises(carve.CarveError):
        srv.flags(12345)                                         # no such job
    ids = [srv.submit(img[k << 19: (k + 1) << 19]) for k in range(6)]   # 512 KiB each: 2 fit the budget
    polls = 0
    done = {}
    while len(done) < len(ids):
        st = srv.stats()
        assert st["in_flight_bytes"] <= 1 << 20
        for jid, nf, nc, s_ in srv.poll():
            done[jid] = nf
        polls += 1
    assert srv.stats()["batches_launched"] >= 3
    srv.close()


def test_results_beyond_staged_room():
    """Every sector flagged, many matches each: more than the room staged at
    launch, so retirement fetches the rest; results still equal the jobs alone."""
    rng = random.Random(5)
    masters, offsets = [], [0]
    for f in range(40):
        sec = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(10)]
        sec[3] = bytes(SECTOR)
        masters += sec
        offsets.append(len(masters))
    ms = torch.tensor(list(b"".join(masters)), dtype=torch.uint8, device="cuda")
    idx = carve.build_master_index(ms, offsets)
    ox = oracle.Index(ms.cpu().numpy(), offsets, threads=4)
    zeros = torch.zeros(4 << 20, dtype=torch.uint8, device="cuda")
    jobs = [(zeros[: n * SECTOR], n % 8, carve.CARVE_TAU_ANY if n % 2 else carve.CARVE_TAU_PER_CLUSTER)
            for n in (1, 7, 64, 999, 4096, 8191)]
    srv = carve.Server(idx, n_streams=2, budget_bytes=64 << 20)
    ids = [srv.submit(t, tau0, mode) for t, tau0, mode in jobs]
    done = _drain(srv, ids)
    for jid, (t, tau0, mode) in zip(ids, jobs):
        n_f = _check_job(srv, jid, done[jid], ox, idx, t, tau0, mode)
        if mode == carve.CARVE_TAU_ANY:
            assert n_f == t.numel() // SECTOR
    srv.close()


def test_bulk_submit_poll_release(pool):
    ms, idx, img, ox = pool
    jobs = _jobs(img, 50, seed=21)
    srv = carve.Server(idx, n_streams=3)
    bad = carve.image_descs(jobs[:5])
    bad[3]["tau0"] = 9
    with pytest.raises(carve.CarveError) as e:
        srv.submit_many(bad)                                     # all or nothing
    assert e.value.code == carve.CARVE_EINVAL and "job 3" in str(e.value)
    assert srv.stats()["queued_jobs"] == 0
    ids = srv.submit_many(carve.image_descs(jobs))
    assert len(ids) == len(jobs) and (np.diff(ids.astype(np.int64)) == 1).all()
    done = {}
    while len(done) < len(jobs):
        d = srv.poll_array()
        for r in d:
            assert r["status"] == carve.CARVE_OK
            done[int(r["job_id"])] = (int(r["n_flagged"]), int(r["n_confirmed"]))
    for jid, (t, tau0, mode) in zip(ids.tolist(), jobs):
        _check_job(srv, jid, done[jid], ox, idx, t, tau0, mode)
    with pytest.raises(carve.CarveError):
        srv.release_many(np.array([ids[0], 987654321], dtype=np.uint64))   # stops at the unknown id
    srv.release_many(ids[1:])
    with pytest.raises(carve.CarveError):
        srv.flags(int(ids[0]))                                   # released by the first call
    assert srv.stats()["done_jobs"] == 0
    srv.close()


def test_host_memory_jobs(pool):
    """Jobs in host memory (pinned and pageable) beside device jobs: each is
    copied to its lane's device arena at launch, and every result equals the
    same bytes scanned alone on the GPU."""
    ms, idx, img, ox = pool
    part = img[: 64 << 20]
    pinned = torch.empty(part.numel(), dtype=torch.uint8, pin_memory=True)
    pinned.copy_(part.cpu())
    pageable = pinned.clone()
    jobs = _jobs(part, 60, seed=31, max_bytes=4 << 20)
    srv = carve.Server(idx, n_streams=3, budget_bytes=48 << 20)
    ids, where = [], []
    for k, (t, tau0, mode) in enumerate(jobs):
        off = t.data_ptr() - part.data_ptr()
        src = (t, pinned, pageable)[k % 3]
        if k % 3:
            src = src[off: off + t.numel()]
        ids.append(srv.submit(src, tau0, mode))
        where.append(k % 3)
    done = _drain(srv, ids)
    assert srv.stats()["batches_launched"] > 1
    for jid, (t, tau0, mode), w in zip(ids, jobs, where):
        # the oracle reads the bytes the server was given (device, pinned or pageable)
        off = t.data_ptr() - part.data_ptr()
        src = (t, pinned[off: off + t.numel()], pageable[off: off + t.numel()])[w]
        _check_job(srv, jid, done[jid], ox, idx, t, tau0, mode, given=src if w else None)
    assert sum(done[j][0] for j, w in zip(ids, where) if w) > 0     # host jobs found something
    srv.close()


@pytest.mark.parametrize("n_streams", [1, 2])
def test_failed_launch_reports_and_recovers(pool, n_streams):
    """A batch launch that fails after its work was enqueued (forced from the
    host with server_fail_next_launches; every kernel runs normally): the
    server waits for the lane, reports the batch's jobs with the error, frees
    their budget and keeps serving. The failed jobs have no results; submitted
    again they complete, and every completed job equals the oracle."""
    ms, idx, img, ox = pool
    jobs = _jobs(img, 12, seed=40 + n_streams, max_bytes=4 << 20)
    srv = carve.Server(idx, n_streams=n_streams)
    srv.fail_next_launches(1)
    ids = {srv.submit(t, tau0, mode): k for k, (t, tau0, mode) in enumerate(jobs)}
    status, counts = {}, {}
    while len(status) < len(ids):
        for jid, nf, nc, st in srv.poll():
            status[jid], counts[jid] = st, (nf, nc)
    failed = [j for j, st in status.items() if st != carve.CARVE_OK]
    assert failed and all(status[j] == carve.CARVE_EDEVICE for j in failed)
    assert srv.stats()["in_flight_bytes"] == 0
    for j in failed:
        with pytest.raises(carve.CarveError) as e:
            srv.flags(j)
        assert e.value.code == carve.CARVE_EDEVICE
    for j, k in ids.items():
        if status[j] == carve.CARVE_OK:
            t, tau0, mode = jobs[k]
            _check_job(srv, j, counts[j], ox, idx, t, tau0, mode)
    again = {srv.submit(*jobs[ids[j]]): ids[j] for j in failed}
    done = _drain(srv, list(again))
    for j, k in again.items():
        t, tau0, mode = jobs[k]
        _check_job(srv, j, done[j], ox, idx, t, tau0, mode)
    assert srv.stats()["in_flight_bytes"] == 0
    srv.close()
