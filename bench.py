#!/usr/bin/env python3
"""Disk-scan throughput of the carving path on one MI355X.

A step is one pass of the whole hot path over a device-resident disk image,
enqueued whole and then waited for once: scan_image (sector loads, djb2-64
signatures, cluster positions, index probe, ordered compaction of the flagged
ids), confirm_enqueue_to (byte comparison of every flagged sector with its
candidate master sectors, ordered records into a device buffer),
flagged_sectors_enqueue (ids into a device buffer) and scan_counts (the one
readback: both counts). The fragment workload keeps two steps in flight by
default (--inflight), on two streams with a scan object and output buffers
each: the scan kernels run in step order (each waits for the previous scan
kernel, scan_wait_kernel), and each step's compaction, confirmation, ids copy
and readback run beside the next step's scan; its line also reports the same
steps one at a time (`ms_per_step_one_in_flight`). The plain workloads run
one step at a time by default (--inflight 2 --overlap kernel is 0.4-2%
faster, measured, but its kernel shares the chip with the confirmation); the
report's `mid` object also times the same steps two in flight
(`in_flight_comparison`). The
master index is built once, before timing, and the launch shape is picked by
the library's autotuner on a tuning sample (an image of the same recipe that
is not the timed one).

With no --workload, prints one JSON line for the whole metric: the headline
is the large workload (64 GiB image, 16M master sectors), with `roofline`
(the scan kernel's algorithmic bytes over its HIP-event duration, against
8 TB/s of HBM3E and against a measured streaming-read ceiling) and
`cpu_baseline` (the CPU oracle on a bounded sample of the same image); the
sub-objects `mid`, `batched` and `served` carry the other workloads (the served
one with p50/p99 latency). `--workload X` runs one workload alone.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "disk GB/s scanned (bit-exact flags) and % HBM roofline; p99 latency served"
HBM_PEAK_GBS = 8000.0
# the arithmetic of the path: djb2-64 (or the CRC-64) modulo 2^64 over the image's unsigned bytes
DTYPE = "u64 mod 2^64 over u8"
BYTES_PER_SECTOR_ALG = 512 + 1.0 / 8.0   # read the sector once, write one flag bit
TUNING_SAMPLE_SECTORS = 1 << 24          # the autotuners' sample: at most 8 GiB
# a kernel's code and its compiler flags: its traffic counters stay valid while these are unchanged
KERNEL_SOURCES = ("paper_0901_1307_amd/csrc/carve_scan_kernel.h", "paper_0901_1307_amd/csrc/carve_device.h",
                  "paper_0901_1307_amd/build.py")
FRAG_KERNEL_SOURCES = ("paper_0901_1307_amd/csrc/carve_fragment_kernel.h", "paper_0901_1307_amd/csrc/carve_device.h",
                       "paper_0901_1307_amd/build.py")
FRAG_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_frag_scan_logos.json")


def traffic_file(kernel: str, config: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{config}.json")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(config: str, kernel_ms: float, path: str, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from its committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a copy of
    known size), as a rate over this run's kernel duration; None if there is
    no summary for this workload or the kernel changed since."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None, None
    if t.get("config") != config or t.get("kernel_source_sha256_16") != kernel_source_hash(sources):
        return None, None
    b = float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])
    return round(b / (kernel_ms * 1e-3) / 1e9, 1), t


def calibrate_copy(nbytes: int = 4 << 30, reps: int = 4):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE
    and WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def free_gpu_memory():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def cpu_baseline(ms, img, n_sectors: int, target_s: float, sig_kind: int = 0):
    """The oracle, as it is, on the host cores: signatures + membership + flag
    list over the first sectors of the same image (the master sort is timed
    apart and excluded)."""
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    ix = oracle.Index(ms.sectors.cpu().numpy(), ms.file_offsets, threads=threads, sig_kind=sig_kind)
    t_sort = time.perf_counter() - t0
    probe = min(n_sectors, 1 << 17)               # 64 MiB to size the sample
    host = img.data[:probe * 512].cpu().numpy()
    t0 = time.perf_counter()
    ix.flag_image(host, threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-6)
    n = int(min(n_sectors, max(probe, rate * target_s)))
    n -= n % 8
    host = img.data[:n * 512].cpu().numpy()
    # passes over the sample until about target_s of CPU work (the whole image
    # can take well under that on many cores)
    passes, dt = 0, 0.0
    while passes == 0 or (dt < target_s and passes < 64):
        t0 = time.perf_counter()
        flags = ix.flag_image(host, threads=threads)
        dt += time.perf_counter() - t0
        passes += 1
    # one thread, on about a quarter of that CPU time
    n1 = 1 << 14
    t0 = time.perf_counter()
    ix.flag_image(host[:n1 * 512], threads=1)
    n1 = int(min(n, max(n1, n1 / max(time.perf_counter() - t0, 1e-6) * target_s / 4)))
    n1 -= n1 % 8
    t0 = time.perf_counter()
    ix.flag_image(host[:n1 * 512], threads=1)
    dt1 = time.perf_counter() - t0
    del host, ix
    return {
        "value": round(passes * n * 512 / dt / 1e9, 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "single_thread_value": round(n1 * 512 / dt1 / 1e9, 4),
        "single_thread_sample": f"first {n1} sectors ({n1 * 512 / 2**30:.2f} GiB) once, {dt1:.2f} s",
        "sample": (f"first {n} sectors ({n * 512 / 2**30:.2f} GiB) of the benchmark image, {len(flags)} flagged, "
                   f"scanned {passes} times; signatures + sorted-array membership + flag list in {dt:.2f} s on "
                   f"{threads} threads ({cpu_model()}); master sort {t_sort:.2f} s excluded"),
    }


def read_ceiling(image, split: bool, reps: int = 3) -> dict:
    """The library's streaming-read probe over the image with the scan's access
    pattern: the best rate over resident grids of 1-4 work-groups per CU and
    all that fit (each the median of `reps` runs)."""
    from paper_0901_1307_amd import carve
    n_bytes = image.numel() // 512 * 512
    rows = []
    for bpc in (0, 1, 2, 3, 4):
        ms = sorted(carve.read_ceiling_probe(image, split=split, blocks_per_cu=bpc) for _ in range(reps))
        rows.append((n_bytes / (ms[len(ms) // 2] * 1e-3) / 1e9, bpc, ms[len(ms) // 2]))
    best = max(rows)
    return {"pattern": "split by cluster position" if split else "contiguous", "GBps": round(best[0], 1),
            "blocks_per_cu": best[1], "ms": round(best[2], 4),
            "sweep_GBps": {str(b): round(r, 1) for r, b, _ in rows}}


def scan_kernel_name(idx) -> str:
    """The kernel a per-cluster scan of one image runs with this index."""
    from paper_0901_1307_amd import carve
    split = idx.scan_config()["split"]
    big = idx.stats()["bloom_bytes"] >= (4 << 20)
    on = split == carve.CARVE_SPLIT_ON or (split == carve.CARVE_SPLIT_AUTO and big)
    return "k_scan_tau" if on and idx.stats()["bloom_bytes"] else "k_scan"


class StepLanes:
    """Steps of one workload kept in flight on `depth` streams. Step i runs
    wholly on stream i % depth with that stream's scan object and output
    buffers: the scan, the confirmation into the records buffer, the ids copy
    and the one count readback. The host waits for step i - depth + 1's counts
    after enqueuing step i, so the GPU never waits for the host. Step i's scan
    waits on the other stream for step i-1's whole step (overlap None), for
    step i-1's scan_image or scan_fragments call, its kernel and compaction
    ("scan"), or for its scan kernel alone ("kernel", scan_wait_kernel); the
    rest of step i-1 then runs beside step i's scan. depth 1 is the plain
    loop: enqueue a step, wait for its counts."""

    def __init__(self, index, depth, first_scan, scan_again, ids_len, rec_bytes, overlap=None):
        import torch
        from paper_0901_1307_amd import carve
        self.carve, self.index, self.depth = carve, index, depth
        self.scan_again, self.overlap = scan_again, overlap
        self.lanes = []
        for k in range(depth):
            s = torch.cuda.current_stream() if k == 0 else torch.cuda.Stream()
            with torch.cuda.stream(s):
                sc = first_scan()
            self.lanes.append({"stream": s, "scan": sc, "event": torch.cuda.Event(),
                               "ids": torch.empty(ids_len, dtype=torch.int64, device="cuda"),
                               "rec": torch.empty(rec_bytes, dtype=torch.uint8, device="cuda")})
        torch.cuda.synchronize()

    def _enqueue(self, i):
        import torch
        lane, prev = self.lanes[i % self.depth], self.lanes[(i - 1) % self.depth]
        with torch.cuda.stream(lane["stream"]):
            if self.depth > 1 and i > 0:   # in step order
                if self.overlap == "kernel":
                    self.carve.scan_wait_kernel(prev["scan"], lane["stream"])
                else:
                    lane["stream"].wait_event(prev["event"])
            self.scan_again(lane["scan"])
            if self.overlap == "scan":
                lane["event"].record(lane["stream"])
            self.carve.confirm_enqueue(self.index, lane["scan"], lane["rec"])
            self.carve.flagged_sectors_enqueue(lane["scan"], lane["ids"])
            if not self.overlap:
                lane["event"].record(lane["stream"])

    def run(self, n, check):
        """n steps; check(counts) on each step's (n_flagged, n_confirmed)."""
        for i in range(n):
            self._enqueue(i)
            if i >= self.depth - 1:
                check(self.carve.scan_counts(self.lanes[(i - self.depth + 1) % self.depth]["scan"]))
        for i in range(max(0, n - self.depth + 1), n):
            check(self.carve.scan_counts(self.lanes[i % self.depth]["scan"]))

    def set_timing(self, on):
        for lane in self.lanes:
            lane["scan"].set_timing(on)

    def kernel_ms(self, n):
        """The kernel durations of the last n steps (each lane's share)."""
        out = []
        for k, lane in enumerate(self.lanes):
            mine = sum(1 for i in range(n) if i % self.depth == k)
            out += lane["scan"].kernel_ms_recent(mine) if mine else []
        return out

    def release(self):
        self.lanes = []


def timed_lanes(lanes, steps, warmup, expect):
    """warmup, then `steps` timed steps between HIP events on the default
    stream (the host has waited for every step's counts before the closing
    event); returns (ms_per_step, wall ms per step, kernel ms of every timed
    launch)."""
    import torch

    def check(c):
        assert c == expect, (c, expect)

    lanes.run(warmup, check)
    lanes.set_timing(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record()
    lanes.run(steps, check)
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - wall0) * 1e3 / steps
    kms = lanes.kernel_ms(steps)
    assert len(kms) == steps
    lanes.set_timing(False)
    return ev0.elapsed_time(ev1) / steps, wall, kms


def run_plain(args, config: str, with_cpu: bool, with_ceiling: bool, also_in_flight: int = 0) -> dict:
    """One image: K timed steps of scan + ids + confirmation. also_in_flight > 1:
    the same steps timed again with that many in flight (each step's scan after
    the previous scan kernel), reported beside the line's own figures."""
    import torch

    import synth
    from paper_0901_1307_amd import carve

    cfg = synth.CONFIGS[config]
    if args.seed is not None:
        import dataclasses
        cfg = dataclasses.replace(cfg, seed=args.seed)
    t0 = time.perf_counter()
    log(f"[bench] generating {cfg.name}: {cfg.n_master_sectors} master sectors, {cfg.n_disk_sectors} disk sectors")
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s; building the index")
    t0 = time.perf_counter()
    sig_kind = carve.CARVE_SIG_CRC64_ISO if args.sig == "crc64" else carve.CARVE_SIG_DJB2_64
    sig_name = "CRC-64/GO-ISO" if args.sig == "crc64" else "djb2-64"
    pick = None
    if args.split is not None:   # a fixed index, kernel and launch shape (profiling runs)
        idx = carve.build_master_index(ms.sectors, ms.file_offsets, sig_kind=sig_kind,
                                       bloom_bits_per_key=args.bloom_bits)
        split = {"auto": carve.CARVE_SPLIT_AUTO, "off": carve.CARVE_SPLIT_OFF, "on": carve.CARVE_SPLIT_ON}[args.split]
        idx.set_scan_config(args.blocks_per_cu, args.tiles_per_chunk, split)
        log(f"[bench] index built in {time.perf_counter() - t0:.2f} s: {idx.stats()}; fixed launch shape")
    else:
        # the library's autotuner (index layout, prefilter size, launch shape)
        # on a tuning sample of the same recipe, not on the timed image
        sample = synth.tuning_sample(cfg, ms, device="cuda", max_sectors=TUNING_SAMPLE_SECTORS)
        idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets, sample, sig_kind=sig_kind)
        del sample
        log(f"[bench] autotuned in {time.perf_counter() - t0:.2f} s: {pick}; index {idx.stats()}")
    shape = idx.scan_config()
    kernel = scan_kernel_name(idx)

    n_sectors = cfg.n_disk_sectors
    image_bytes = img.data.numel()
    flag_out = torch.empty(n_sectors, dtype=torch.int64, device="cuda")
    sc = carve.scan_image(idx, img.data)
    n_flag = carve.flagged_sectors(sc, flag_out).numel()
    n_match = carve.confirm_matches(idx, sc, torch.empty(16 * max(1, 4 * n_flag), dtype=torch.uint8, device="cuda"))
    del flag_out
    log(f"[bench] {n_flag} flagged, {n_match} confirmed")

    # the whole path enqueued per step (scan, records into a device buffer, ids
    # copy), one wait for both counts; steps in flight on `inflight` streams
    inflight = args.inflight or 1
    reuse = [sc]   # the first lane takes the scan object above (no extra scan before the warm-up)

    def lanes_of(depth):
        return StepLanes(idx, depth, lambda: reuse.pop() if reuse else carve.scan_image(idx, img.data),
                         lambda s: carve.scan_image(idx, img.data, scan=s), n_sectors, 16 * max(1, 2 * n_match + 1024),
                         overlap=None if args.overlap in ("auto", "off") else args.overlap)

    serial = None
    if inflight > 1:   # the same steps one at a time, for comparison
        lanes = lanes_of(1)
        ms1, _, _ = timed_lanes(lanes, args.steps, args.warmup, (n_flag, n_match))
        lanes.release()
        serial = round(ms1, 4)
    lanes = lanes_of(inflight)
    ms_per_step, wall, kernel_ms = timed_lanes(lanes, args.steps, args.warmup, (n_flag, n_match))
    lanes.release()
    log(f"[bench] {args.steps} steps, {inflight} in flight: {ms_per_step:.3f} ms/step (event), "
        f"wall {wall:.3f} ms/step; one at a time {serial} ms/step")
    extra = None
    if also_in_flight > 1 and also_in_flight != inflight:
        lanes = StepLanes(idx, also_in_flight, lambda: carve.scan_image(idx, img.data),
                          lambda s: carve.scan_image(idx, img.data, scan=s), n_sectors,
                          16 * max(1, 2 * n_match + 1024), overlap="kernel")
        ms_x, _, kms_x = timed_lanes(lanes, args.steps, args.warmup, (n_flag, n_match))
        lanes.release()
        extra = {"steps_in_flight": also_in_flight, "ms_per_step": round(ms_x, 4),
                 "value": round(image_bytes / (ms_x * 1e-3) / 1e9, 2),
                 "kernel_ms": round(sum(kms_x) / len(kms_x), 4) if kms_x else None}
        log(f"[bench] the same steps, {also_in_flight} in flight: {ms_x:.3f} ms/step")
    # apart from the timed steps: the same step with ids and records copied to
    # pinned host memory (end to end including device-to-host)
    flag_h = torch.empty(n_flag + 1024, dtype=torch.int64, pin_memory=True)
    match_h = torch.empty(16 * (n_match + 1024), dtype=torch.uint8, pin_memory=True)

    def step_host():
        carve.scan_image(idx, img.data, scan=sc)
        nf = carve.flagged_sectors(sc, flag_h).numel()
        nm = carve.confirm_matches(idx, sc, match_h)
        return nf, nm

    step_host()
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    for _ in range(5):
        assert step_host() == (n_flag, n_match)
    ms_host = (time.perf_counter() - t_h) * 1e3 / 5
    del sc, flag_h, match_h

    value = image_bytes / (ms_per_step * 1e-3) / 1e9
    k_avg = sum(kernel_ms) / len(kernel_ms)
    achieved = n_sectors * BYTES_PER_SECTOR_ALG / (k_avg * 1e-3) / 1e9
    tkey = cfg.name if args.sig == "djb2" else f"{cfg.name}-{args.sig}"
    traffic, traffic_src = measured_traffic(tkey, k_avg, traffic_file(kernel, cfg.name))
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg.name}: {image_bytes / 2**30:.0f} GiB device-resident disk image "
                         f"({n_sectors} sectors of 512 B) against {cfg.n_master_sectors} master sectors "
                         f"in {len(ms.file_offsets) - 1} files, {sig_name}, per-cluster positions"),
            "signature": sig_name,
            "image_bytes": image_bytes,
            "n_sectors": n_sectors,
            "n_master_sectors": cfg.n_master_sectors,
            "seed": cfg.seed,
            "launch_shape": shape,
            "index_pick": pick,
            "prefilter_bytes": idx.stats()["bloom_bytes"],
        },
        "sectors_per_s": round(n_sectors / (ms_per_step * 1e-3)),
        "steps_in_flight": inflight,
        "ms_per_step_one_in_flight": serial,
        "in_flight_comparison": extra,
        "ms_per_step_host_outputs": round(ms_host, 4),
        "hbm_frac_of_value": round(value / HBM_PEAK_GBS, 4),
        "flagged": n_flag,
        "confirmed": n_match,
        "roofline": {
            "bound": "hbm",
            "kernel": (f"{kernel} (signature + probe"
                       + (", split by cluster position over the 8 XCDs)" if kernel == "k_scan_tau" else ")")),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel_ms": round(k_avg, 4),
            "kernel_ms_median": round(sorted(kernel_ms)[len(kernel_ms) // 2], 4),
            "kernel_ms_min": round(min(kernel_ms), 4),
            "algorithmic_bytes_per_launch": round(n_sectors * BYTES_PER_SECTOR_ALG),
            "traffic_bytes_per_launch": (None if traffic_src is None else
                                         round(traffic_src["fetch_bytes_per_launch"] +
                                               traffic_src["write_bytes_per_launch"])),
        },
    }
    if with_ceiling:
        ceil = read_ceiling(img.data, split=kernel == "k_scan_tau")
        other = read_ceiling(img.data, split=kernel != "k_scan_tau")
        log(f"[bench] streaming-read ceiling ({ceil['pattern']}): {ceil['GBps']:.0f} GB/s; "
            f"{other['pattern']}: {other['GBps']:.0f} GB/s")
        out["roofline"]["read_ceiling"] = ceil
        out["roofline"]["read_ceiling_other_pattern"] = other
        out["roofline"]["frac_of_read_ceiling"] = round(achieved / ceil["GBps"], 4)
    if with_cpu:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(ms, img, n_sectors, args.cpu_seconds, sig_kind)
    del img, ms, idx
    free_gpu_memory()
    return out


def run_batched(args) -> dict:
    """Many uneven images against the mid master set: one persistent launch per
    step, replayed from a HIP graph, then per-image counts and confirmation."""
    import torch

    import synth
    from paper_0901_1307_amd import carve

    cfg = synth.CONFIGS["mid"]
    t0 = time.perf_counter()
    ms = synth.master_set(cfg, device="cuda")
    images = synth.batch_images(cfg, ms, device="cuda", n_images=args.images)
    total = sum(t.numel() for t in images)
    n_sectors = total // 512
    torch.cuda.synchronize()
    log(f"[bench] {len(images)} images, {total / 2**30:.1f} GiB, generated in {time.perf_counter() - t0:.1f} s")
    # batches scan contiguously: the autotuner times that walk only
    sample = synth.tuning_sample(cfg, ms, device="cuda", max_sectors=TUNING_SAMPLE_SECTORS)
    idx, pick = carve.autotune_index(ms.sectors, ms.file_offsets, sample, contiguous_only=True)
    del sample
    tuned = idx.scan_config()
    log(f"[bench] autotuned: {pick}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = carve.scan_batch(idx, images)
        counts = carve.batch_flag_counts(b)
        n_match = carve.batch_confirm_matches(idx, b, torch.empty(24 * max(1, 4 * int(counts.sum())),
                                                                  dtype=torch.uint8, device="cuda"))
        match_out = torch.empty(24 * (2 * n_match + 1024), dtype=torch.uint8, device="cuda")
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):   # scan, compaction and confirmation
            carve.scan_batch(idx, images, batch=b)
            carve.confirm_enqueue(idx, b)
    n_flag = int(counts.sum())
    log(f"[bench] {n_flag} flagged, {n_match} confirmed")

    def step():
        graph.replay()
        c = carve.batch_flag_counts(b)
        m = carve.batch_confirm_matches(idx, b, match_out)
        return int(c.sum()), m

    # replays, readbacks and events all on the batch's stream
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            assert step() == (n_flag, n_match)
        ev1.record()
        torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    # the scan kernel alone, eager, HIP events on its stream
    kb = carve.Batch()
    with torch.cuda.stream(stream):
        carve.scan_batch(idx, images, batch=kb)
        kb.set_timing(True)
        for _ in range(5):
            carve.scan_batch(idx, images, batch=kb)
        kms = kb.kernel_ms_recent(5)
    k_avg = sum(kms) / len(kms)
    achieved = n_sectors * BYTES_PER_SECTOR_ALG / (k_avg * 1e-3) / 1e9
    value = total / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": (f"batched: {len(images)} device-resident images, sizes log-uniform 1 MiB-1 GiB "
                                f"({total / 2**30:.1f} GiB), hit rate 0-5% each, against the mid master set "
                                f"({cfg.n_master_sectors} sectors); one persistent launch replayed from a HIP graph"),
                   "image_bytes": total, "n_images": len(images), "launch_shape": tuned, "index_pick": pick},
        "flagged": n_flag, "confirmed": n_match,
        "roofline": {"bound": "hbm", "kernel": "k_scan<kFlags, ManyImages>", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel_ms": round(k_avg, 4)},
    }
    del graph, b, kb, images, match_out, idx, ms
    free_gpu_memory()
    return out


def run_served(args) -> dict:
    """Open loop: jobs arrive on a Poisson clock and go through the native
    server (admission by a 32 GiB budget, continuous batching over stream
    lanes, confirmation); latency = completion seen by the loop - arrival.
    Then a closed loop of the same jobs (all queued at once), twice: the first
    pass after the lightly loaded open loop, then the steady state."""
    import numpy as np
    import torch

    import synth
    from paper_0901_1307_amd import carve

    cfg = synth.CONFIGS["served"]
    ms = synth.master_set(cfg, device="cuda")
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    pool = synth.disk_image(cfg, ms, device="cuda").data
    pool_sectors = pool.numel() // 512
    rate = args.rate if args.rate is not None else (1500.0 if args.host_jobs else 2000.0)
    src = pool
    h2d = None
    if args.host_jobs:   # jobs arrive in (pinned) host memory and cross PCIe
        src = torch.empty(pool.numel(), dtype=torch.uint8, pin_memory=True)
        src.copy_(pool.cpu())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            pool.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        h2d = 3 * pool.numel() / (time.perf_counter() - t1) / 1e9
    specs = synth.served_job_specs(cfg.seed, rate=rate, duration=args.duration)
    firsts = synth.served_job_slices(specs, pool_sectors, cfg.seed)
    jobs = []
    for (t, size, flow), first in zip(specs, firsts):
        view = src[first * 512: first * 512 + size]
        jobs.append((t, view, first % 8 if not flow else 0,
                     carve.CARVE_TAU_ANY if flow else carve.CARVE_TAU_PER_CLUSTER))
    log(f"[bench] served: {len(jobs)} jobs over {args.duration:.0f} s, "
        f"{sum(j[1].numel() for j in jobs) / 1e9:.1f} GB, pool {pool.numel() / 2**30:.1f} GiB, "
        f"index {idx.stats()['n_master_sectors']} master sectors")
    idx.set_scan_config(blocks_per_cu=args.blocks_per_cu, tiles_per_chunk=0)
    srv = carve.Server(idx, n_streams=args.lanes, budget_bytes=32 << 30, confirm=True)

    def drain(n_jobs):
        """Poll until n_jobs complete, releasing each batch of completions at once."""
        while n_jobs:
            done = srv.poll_array()
            if len(done):
                assert (done["status"] == carve.CARVE_OK).all()
                srv.release_many(done["job_id"])
                n_jobs -= len(done)

    warm = carve.image_descs([(v, tau0, mode) for _, v, tau0, mode in jobs[:64]])
    drain(len(srv.submit_many(warm)))   # warm-up

    # open loop
    arrival, size_of, lat, done_at = {}, {}, [], []
    nxt, n, n_done, bytes_done = 0, len(jobs), 0, 0
    flags = confirmed = 0
    t0 = time.perf_counter()
    while n_done < n:
        now = time.perf_counter() - t0
        while nxt < n and jobs[nxt][0] <= now:
            t, v, tau0, mode = jobs[nxt]
            jid = srv.submit(v, tau0, mode)
            arrival[jid], size_of[jid] = t, v.numel()
            nxt += 1
        done = srv.poll_array()
        if len(done):
            tc = time.perf_counter() - t0
            assert (done["status"] == carve.CARVE_OK).all()
            for jid in done["job_id"].tolist():
                lat.append((arrival[jid], tc - arrival.pop(jid)))
                bytes_done += size_of.pop(jid)
            done_at.append(tc)
            flags += int(done["n_flagged"].sum())
            confirmed += int(done["n_confirmed"].sum())
            n_done += len(done)
            srv.release_many(done["job_id"])
    elapsed = max(done_at)
    warm_s = 5.0 if args.duration > 10 else 0.0
    steady = np.array([l for a, l in lat if a >= warm_s]) * 1e3
    p50, p99, pmax = (float(np.percentile(steady, q)) for q in (50, 99, 100))
    sustained = bytes_done / elapsed / 1e9
    log(f"[bench] open loop: {n} jobs in {elapsed:.1f} s, p50 {p50:.3f} ms, p99 {p99:.3f} ms, "
        f"{sustained:.1f} GB/s, {srv.stats()['batches_launched']} batches")

    # closed loop: the server's saturation throughput on the same jobs, handed
    # over in one call (descriptors built beforehand, as a native client would)
    sub = jobs[: min(n, 20000)]
    sub_bytes = sum(j[1].numel() for j in sub)
    descs = carve.image_descs([(v, tau0, mode) for _, v, tau0, mode in sub])
    first_pass = None
    if not args.host_jobs:
        # the first pass after the lightly loaded open loop, then the steady state
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        drain(len(srv.submit_many(descs)))
        first_pass = sub_bytes / (time.perf_counter() - t1) / 1e9
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    drain(len(srv.submit_many(descs)))
    t_closed = time.perf_counter() - t1
    capacity = sub_bytes / t_closed / 1e9
    log(f"[bench] closed loop: {len(sub)} jobs, {sub_bytes / 1e9:.1f} GB in {t_closed:.2f} s = {capacity:.0f} GB/s"
        + ("" if first_pass is None else f" (first pass: {first_pass:.0f} GB/s)"))
    after_idle = after_busy = None
    if not args.host_jobs:
        # What slows the first pass: the same pass after 2 s of an idle GPU,
        # then after 2 s idle and about 100 ms of streaming reads just before it.
        def closed_pass():
            torch.cuda.synchronize()
            t = time.perf_counter()
            drain(len(srv.submit_many(descs)))
            return sub_bytes / (time.perf_counter() - t) / 1e9

        time.sleep(2.0)
        after_idle = closed_pass()
        time.sleep(2.0)
        t = time.perf_counter()
        while time.perf_counter() - t < 0.1:
            carve.read_ceiling_probe(pool)
        after_busy = closed_pass()
        log(f"[bench] closed loop after 2 s idle: {after_idle:.0f} GB/s; after 2 s idle and 100 ms of load: "
            f"{after_busy:.0f} GB/s")
    st = srv.stats()
    srv.close()
    idx.set_scan_config(blocks_per_cu=0, tiles_per_chunk=0)   # the references below use the default launch shape
    workload = (f"served: Poisson arrivals at {rate:.0f}/s for {args.duration:.0f} s, sizes "
                f"log-uniform 64 KiB-256 MiB (flow buffers < 1 MiB matched at any position), "
                f"{'pinned host-memory' if args.host_jobs else 'device-resident'} pool, resident index of "
                f"{cfg.n_master_sectors} master sectors, 32 GiB admission budget, {args.lanes} stream lanes"
                f"{f' of {args.blocks_per_cu} scan blocks per CU' if args.blocks_per_cu else ''}, confirmation on")
    common = {
        "metric": METRIC, "value": round(sustained, 2), "unit": "GB/s", "n_gpus": 1, "steps": n,
        "warmup": 64, "ms_per_step": round(elapsed * 1e3 / n, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": workload, "jobs": n, "bytes": bytes_done, "host_jobs": bool(args.host_jobs)},
        "latency_ms": {"p50": round(p50, 4), "p99": round(p99, 4), "max": round(pmax, 4),
                       "excluded_warmup_s": warm_s},
        "offered_GBps": round(bytes_done / args.duration / 1e9, 2),
        "saturation_GBps": round(capacity, 1),
        "saturation_first_pass_GBps": None if first_pass is None else round(first_pass, 1),
        "saturation_after_idle_GBps": None if after_idle is None else round(after_idle, 1),
        "saturation_after_idle_and_load_GBps": None if after_busy is None else round(after_busy, 1),
        "closed_loop_jobs": len(sub),
        "flagged": flags, "confirmed": confirmed,
    }
    if args.host_jobs:   # PCIe-bound: compare with a plain host-to-device copy
        log(f"[bench] plain pinned host-to-device copy: {h2d:.1f} GB/s")
        common.update({"h2d_copy_GBps": round(h2d, 2), "saturation_vs_copy": round(capacity / h2d, 3)})
        del jobs, descs, src, pool, idx, ms
        free_gpu_memory()
        return common
    # reference: the same closed-loop jobs as one batch through the plain
    # batch path (scan, every image's ids and confirmed matches to the host)
    ref_jobs = [(v, tau0, mode) for _, v, tau0, mode in sub]
    b = carve.scan_batch(idx, ref_jobs)
    total_flags = int(carve.batch_flag_counts(b).sum())
    ids_h = torch.empty(max(total_flags, 1), dtype=torch.int64, pin_memory=True)
    rec_h = torch.empty(24 * (2 * total_flags + 1024), dtype=torch.uint8, pin_memory=True)

    def one_batch():
        carve.scan_batch(idx, ref_jobs, batch=b)
        n_ids = int(carve.batch_flag_counts(b).sum())
        lib = carve.load_library()
        got = carve.ctypes.c_uint64()
        carve._check(lib.batch_flagged_sectors(b.handle, carve.CARVE_ALL_IMAGES, ids_h.data_ptr(), ids_h.numel(),
                                               carve.ctypes.byref(got)))
        return n_ids, carve.batch_confirm_matches(idx, b, rec_h)

    one_batch()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        one_batch()
    ref_gbps = sub_bytes * reps / (time.perf_counter() - t2) / 1e9
    # context: the per-cluster plain path over the whole pool
    sc = carve.scan_image(idx, pool)
    fo = torch.empty(pool_sectors, dtype=torch.int64, device="cuda")
    mo = torch.empty(16 * pool_sectors, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        carve.scan_image(idx, pool, scan=sc)
        carve.flagged_sectors(sc, fo)
        carve.confirm_matches(idx, sc, mo)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(10):
        carve.scan_image(idx, pool, scan=sc)
        carve.flagged_sectors(sc, fo)
        carve.confirm_matches(idx, sc, mo)
    plain = pool.numel() * 10 / (time.perf_counter() - t3) / 1e9
    log(f"[bench] same jobs as one batch: {ref_gbps:.0f} GB/s; plain path over the pool: {plain:.0f} GB/s; "
        f"server host time: launch {st['host_launch_s']:.2f} s, retire {st['host_retire_s']:.2f} s")
    common.update({"same_jobs_one_batch_GBps": round(ref_gbps, 1),
                   "saturation_vs_one_batch": round(capacity / ref_gbps, 3),
                   "plain_path_whole_pool_GBps": round(plain, 1),
                   "saturation_vs_plain_pool": round(capacity / plain, 3),
                   "first_pass_vs_plain_pool": None if first_pass is None else round(first_pass / plain, 3)})
    del sc, fo, mo, b, ids_h, rec_h, jobs, descs, sub, ref_jobs, pool, src, idx, ms
    free_gpu_memory()
    return common


def run_layouts(args):
    """Occupancy sweep over the probe layouts (Section 4's study of hash table
    occupancy): the scan kernel's GB/s on the mid workload for the bucketed
    table, the paper's per-slot linear probing from the low signature bits
    (Eq. (3)) and a sorted array with binary search, at table loads 0.1-0.9,
    with and without the Bloom prefilter. Every configuration's flagged ids are
    checked against the default layout's, bit for bit."""
    import torch

    import synth
    from paper_0901_1307_amd import carve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = synth.CONFIGS["mid"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda").data
    n_sectors = img.numel() // 512
    ref = None
    rows = []
    names = {carve.CARVE_LAYOUT_BUCKETED: "bucketed", carve.CARVE_LAYOUT_LINEAR: "linear",
             carve.CARVE_LAYOUT_SORTED: "sorted"}
    loads = [0.1, 0.3, 0.5, 0.7, 0.9]
    for bloom in (0, carve.CARVE_BLOOM_OFF):
        for layout in (carve.CARVE_LAYOUT_BUCKETED, carve.CARVE_LAYOUT_LINEAR, carve.CARVE_LAYOUT_SORTED):
            for load in (loads if layout != carve.CARVE_LAYOUT_SORTED else [0.5]):
                idx = carve.build_master_index(ms.sectors, ms.file_offsets, max_load=load, layout=layout,
                                               bloom_bits_per_key=bloom)
                sc = carve.scan_image(idx, img)
                ids = carve.flagged_sectors(sc, torch.empty(n_sectors, dtype=torch.int64, device="cuda")).clone()
                if ref is None:
                    ref = ids
                assert torch.equal(ids, ref), (names[layout], load, bloom)
                sc.set_timing(True)
                kms = []
                for _ in range(7):
                    carve.scan_image(idx, img, scan=sc)
                    kms.append(sc.kernel_ms())
                kms = sorted(kms[2:])
                k = kms[len(kms) // 2]
                gbs = n_sectors * BYTES_PER_SECTOR_ALG / (k * 1e-3) / 1e9
                st = idx.stats()
                rows.append({"layout": names[layout], "load": load if layout != carve.CARVE_LAYOUT_SORTED else None,
                             "bloom": "off" if bloom == carve.CARVE_BLOOM_OFF else "auto",
                             "bloom_bytes": st["bloom_bytes"], "kernel_ms": round(k, 4), "GBps": round(gbs, 1),
                             "frac": round(gbs / HBM_PEAK_GBS, 4)})
                log(f"[bench] {names[layout]:9s} load {load:.1f} bloom {rows[-1]['bloom']:4s}: "
                    f"{k:.3f} ms, {gbs:.0f} GB/s")
                del idx, sc
    best = max(rows, key=lambda r: r["GBps"])
    out = {"metric": METRIC, "value": best["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": 5, "warmup": 2,
           "ms_per_step": best["kernel_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE, "data": "synthetic",
           "config": {"workload": ("layouts: scan kernel on the mid workload (8 GiB image, 1048576 master sectors) "
                                   "per probe layout, table load and prefilter; value = the best configuration"),
                      "n_sectors": n_sectors, "flagged": int(ref.numel())},
           "sweep": rows}
    print(json.dumps(out), flush=True)


def run_fragments(args):
    """Section 5's fragment scan: every 64-byte window at a 4-byte boundary of a
    device-resident image against the 64-byte fragments of master "logo"
    files. A step = scan_fragments + flagged window ids + confirmed records,
    both into device buffers."""
    import torch

    import synth
    from paper_0901_1307_amd import carve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = synth.FRAGMENT_CONFIGS["logos"]
    t0 = time.perf_counter()
    files = synth.fragment_files(cfg, device="cuda")
    frags, offsets = carve.pack_fragment_files(files)
    img = synth.fragment_image(cfg, files, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] fragments: {len(files)} files, {len(frags) // 64} fragments, image {img.numel() / 2**30:.1f} GiB, "
        f"generated in {time.perf_counter() - t0:.1f} s")
    idx = carve.build_fragment_index(frags, offsets)
    n_bytes = img.numel()
    n_windows = (n_bytes - 64) // 4 + 1
    sc = carve.scan_fragments(idx, img)
    n_flag = carve.flagged_sectors(sc).numel()
    n_match = carve.confirm_matches(idx, sc, torch.empty(16 * (2 * n_flag + 1024), dtype=torch.uint8, device="cuda"))
    del sc
    log(f"[bench] {n_flag} windows flagged, {n_match} confirmed")

    # the whole path enqueued per step (scan, records into a device buffer, ids
    # copy), one wait for both counts; steps in flight on `inflight` streams
    inflight = args.inflight or 2

    def lanes_of(depth):
        return StepLanes(idx, depth, lambda: carve.scan_fragments(idx, img),
                         lambda s: carve.scan_fragments(idx, img, scan=s), n_flag + 1024, 16 * (n_match + 1024),
                         overlap=None if args.overlap == "off" else ("kernel" if args.overlap == "auto" else args.overlap))

    serial, serial_kms = None, None
    if inflight > 1:   # the same steps one at a time, for comparison
        lanes = lanes_of(1)
        ms1, _, serial_kms = timed_lanes(lanes, args.steps, args.warmup, (n_flag, n_match))
        lanes.release()
        serial = round(ms1, 4)
    lanes = lanes_of(inflight)
    ms, _, kms = timed_lanes(lanes, args.steps, args.warmup, (n_flag, n_match))
    lanes.release()
    ms_per_step = ms
    k_avg = sum(kms) / len(kms)
    alg = n_bytes + n_windows / 8            # the image read once, one flag bit per window
    achieved = alg / (k_avg * 1e-3) / 1e9
    value = n_bytes / (ms_per_step * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic("logos", k_avg, FRAG_TRAFFIC_FILE, FRAG_KERNEL_SOURCES)
    log(f"[bench] {args.steps} steps, {inflight} in flight: {ms_per_step:.3f} ms/step, kernel {k_avg:.3f} ms; "
        f"one at a time {serial} ms/step")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": (f"fragments: every 64-byte window at a 4-byte boundary of a {n_bytes / 2**30:.0f} GiB "
                                f"device-resident image ({n_windows} windows) against {len(frags) // 64} fragments of "
                                f"{len(files)} master files of 2-32 KiB, {cfg.n_embedded} copies embedded "
                                f"({cfg.p_aligned:.0%} 4-byte aligned), djb2-64"),
                   "image_bytes": n_bytes, "n_windows": n_windows, "n_fragments": len(frags) // 64},
        "windows_per_s": round(n_windows / (ms_per_step * 1e-3)),
        "steps_in_flight": inflight, "ms_per_step_one_in_flight": serial,
        "flagged": n_flag, "confirmed": n_match,
        "roofline": {"bound": "hbm", "kernel": "k_frag_scan (rolling signatures + filter/table probe)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel_ms": round(k_avg, 4),
                     # the kernel alone: the same kernel in the steps run one at a time
                     "kernel_ms_one_in_flight": (None if not serial_kms else
                                                 round(sum(serial_kms) / len(serial_kms), 4)),
                     "frac_one_in_flight": (None if not serial_kms else
                                            round(alg / (sum(serial_kms) / len(serial_kms) * 1e-3) / 1e9
                                                  / HBM_PEAK_GBS, 4)),
                     "traffic_bytes_per_launch": (None if traffic_src is None else
                                                  round(traffic_src["fetch_bytes_per_launch"] +
                                                        traffic_src["write_bytes_per_launch"])),
                     # from the same committed counters (SQ_INSTS_VALU): VALU issue, the other limit
                     "valu_instructions_per_window": (None if traffic_src is None else
                                                      traffic_src.get("valu_instructions_per_window")),
                     "valu_busy": None if traffic_src is None else traffic_src.get("valu_busy")},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.default_threads()
        ox = oracle.FragmentIndex(frags.cpu().numpy(), offsets, threads=threads)
        host = img[: 1 << 28].cpu().numpy()
        passes, dt = 0, 0.0
        while passes == 0 or (dt < args.cpu_seconds and passes < 64):
            t1 = time.perf_counter()
            ox.flag_windows(host, threads=threads)
            dt += time.perf_counter() - t1
            passes += 1
        out["cpu_baseline"] = {"value": round(passes * host.size / dt / 1e9, 4), "unit": "GB/s", "cores": threads,
                               "kind": "oracle",
                               "sample": (f"first 256 MiB of the benchmark image scanned {passes} times: every "
                                          f"window hashed and looked up, {dt:.2f} s on {threads} threads "
                                          f"({cpu_model()})")}
    print(json.dumps(out), flush=True)


def run_ingest(args):
    """Section 3.1's pipeline: the mid image (8 GiB) scanned from host memory
    through two device buffers while the other is scanned, from a pinned and a
    pageable copy, beside a plain pinned host-to-device copy of the same bytes
    (the transfer's own ceiling). Flags and matches are checked against the
    device-resident scan."""
    import torch

    import synth
    from paper_0901_1307_amd import carve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = synth.CONFIGS["mid"]
    ms = synth.master_set(cfg, device="cuda")
    dev = synth.disk_image(cfg, ms, device="cuda").data
    idx = carve.build_master_index(ms.sectors, ms.file_offsets)
    sc = carve.scan_image(idx, dev)
    n_flag = carve.flagged_sectors(sc).numel()
    n_match = len(carve.confirm_matches(idx, sc))
    del sc
    n = dev.numel()
    t0 = time.perf_counter()
    pinned = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    pinned.copy_(dev.cpu())
    pageable = pinned.clone()
    log(f"[bench] ingest: {n / 2**30:.0f} GiB image in host memory (pinned and pageable), "
        f"prepared in {time.perf_counter() - t0:.1f} s")
    # the transfer alone: pinned host -> device, same bytes
    torch.cuda.synchronize()
    reps = 3
    t1 = time.perf_counter()
    for _ in range(reps):
        dev.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    h2d = n * reps / (time.perf_counter() - t1) / 1e9
    ing = carve.Ingest(idx)
    res = {}
    for name, host in (("pinned", pinned), ("pageable", pageable)):
        ing.scan(host)                           # warm-up, and the check
        assert ing.flagged().size == n_flag and ing.matches().size == n_match
        rates = []
        for _ in range(max(1, min(args.steps, 5))):
            ing.scan(host)
            st = ing.stats()
            rates.append(st["bytes"] / st["seconds"] / 1e9)
        res[name] = {"GBps": round(sorted(rates)[len(rates) // 2], 2), "chunks": st["chunks"]}
        log(f"[bench] ingest from {name} memory: {res[name]['GBps']:.1f} GB/s ({st['chunks']} chunks of 256 MiB)")
    ing.close()
    log(f"[bench] plain pinned host-to-device copy: {h2d:.1f} GB/s")
    value = res["pinned"]["GBps"]
    out = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": min(args.steps, 5), "warmup": 1,
        "ms_per_step": round(n / (value * 1e9) * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": (f"ingest: the mid workload's {n / 2**30:.0f} GiB image scanned and confirmed from "
                                f"host memory (PCIe included) in 256 MiB chunks through two device buffers; value = "
                                f"pinned source"),
                   "image_bytes": n},
        "pinned_GBps": res["pinned"]["GBps"], "pageable_GBps": res["pageable"]["GBps"],
        "h2d_copy_GBps": round(h2d, 2), "pinned_vs_copy": round(res["pinned"]["GBps"] / h2d, 3),
        "flagged": n_flag, "confirmed": n_match,
    }
    print(json.dumps(out), flush=True)


def run_report(args):
    """The whole metric in one line: the large workload as the headline, the
    mid, batched and served workloads as sub-objects."""
    t_start = time.perf_counter()
    head = run_plain(args, "large", with_cpu=not args.no_cpu_baseline, with_ceiling=True)
    mid = run_plain(args, "mid", with_cpu=False, with_ceiling=False, also_in_flight=2)
    batched = run_batched(args)
    served = run_served(args)
    mid_rate = mid["value"]
    head["mid"] = {"workload": mid["config"]["workload"], "value": mid["value"], "unit": "GB/s",
                   "ms_per_step": mid["ms_per_step"], "steps_in_flight": mid["steps_in_flight"],
                   "ms_per_step_one_in_flight": mid["ms_per_step_one_in_flight"],
                   "in_flight_comparison": mid["in_flight_comparison"],
                   "hbm_frac_of_value": mid["hbm_frac_of_value"],
                   "kernel": mid["roofline"]["kernel"], "kernel_ms": mid["roofline"]["kernel_ms"],
                   "achieved": mid["roofline"]["achieved"], "frac": mid["roofline"]["frac"],
                   "traffic": mid["roofline"]["traffic"], "launch_shape": mid["config"]["launch_shape"],
                   "index_pick": mid["config"]["index_pick"],
                   "flagged": mid["flagged"], "confirmed": mid["confirmed"]}
    head["batched"] = {"workload": batched["config"]["workload"], "value": batched["value"], "unit": "GB/s",
                       "ms_per_step": batched["ms_per_step"], "kernel_ms": batched["roofline"]["kernel_ms"],
                       "achieved": batched["roofline"]["achieved"], "frac": batched["roofline"]["frac"],
                       "vs_plain_mid": round(batched["value"] / mid_rate, 3),
                       "kernel_vs_plain_mid_kernel": round(batched["roofline"]["achieved"] /
                                                           mid["roofline"]["achieved"], 3),
                       "launch_shape": batched["config"]["launch_shape"],
                       "index_pick": batched["config"]["index_pick"],
                       "flagged": batched["flagged"], "confirmed": batched["confirmed"]}
    head["served"] = {"workload": served["config"]["workload"], "jobs": served["config"]["jobs"],
                      "offered_GBps": served["offered_GBps"], "sustained_GBps": served["value"],
                      "latency_ms": served["latency_ms"],
                      "saturation_steady_GBps": served["saturation_GBps"],
                      "saturation_first_pass_GBps": served["saturation_first_pass_GBps"],
                      "saturation_after_idle_GBps": served["saturation_after_idle_GBps"],
                      "saturation_after_idle_and_load_GBps": served["saturation_after_idle_and_load_GBps"],
                      "steady_vs_plain_mid": round(served["saturation_GBps"] / mid_rate, 3),
                      "first_pass_vs_plain_mid": (None if served["saturation_first_pass_GBps"] is None else
                                                  round(served["saturation_first_pass_GBps"] / mid_rate, 3)),
                      "plain_path_whole_pool_GBps": served.get("plain_path_whole_pool_GBps"),
                      "steady_vs_plain_pool": served.get("saturation_vs_plain_pool"),
                      "first_pass_vs_plain_pool": served.get("first_pass_vs_plain_pool"),
                      "same_jobs_one_batch_GBps": served.get("same_jobs_one_batch_GBps"),
                      "closed_loop_jobs": served["closed_loop_jobs"],
                      "flagged": served["flagged"], "confirmed": served["confirmed"]}
    head["elapsed_s"] = round(time.perf_counter() - t_start, 1)
    log(f"[bench] report done in {head['elapsed_s']:.0f} s")
    return head


def arg_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="report",
                    choices=["report", "plain", "batched", "served", "layouts", "fragments", "ingest"],
                    help="report (default): the large workload as the headline with mid, batched and served "
                         "as sub-objects; plain: one image (--config); batched: 256 uneven images in one "
                         "launch; served: Poisson stream of scan jobs through the continuous-batching server; "
                         "layouts: occupancy sweep over the index's probe layouts; "
                         "fragments: every 64-byte window at a 4-byte boundary (Section 5); "
                         "ingest: images in host memory through double-buffered transfers (Section 3.1)")
    ap.add_argument("--config", default="large", choices=["tiny", "mid", "large"], help="plain: the workload")
    ap.add_argument("--sig", default="djb2", choices=["djb2", "crc64"],
                    help="plain: sector signature (djb2-64 of Eq. (1), or the CRC-64 of Section 2.1)")
    ap.add_argument("--bloom-bits", type=int, default=0,
                    help="plain: prefilter bits per signature (0: automatic, 4294967295: none)")
    ap.add_argument("--split", choices=["auto", "off", "on"], default=None,
                    help="plain: fix the scan walk (and --blocks-per-cu / --tiles-per-chunk) instead of autotuning")
    ap.add_argument("--tiles-per-chunk", type=int, default=0, help="plain with --split: tiles per chunk")
    ap.add_argument("--images", type=int, default=256, help="batched: number of images")
    ap.add_argument("--rate", type=float, default=None,
                    help="served: arrivals per second (2000; 1500 with --host-jobs, under the PCIe rate)")
    ap.add_argument("--host-jobs", action="store_true",
                    help="served: jobs arrive in pinned host memory and cross PCIe")
    ap.add_argument("--duration", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--lanes", type=int, default=2, help="served: stream lanes (the server's default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="served: scan blocks per CU of each lane's launches; plain with --split: of the scan "
                         "(0: as many as fit)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--seed", type=int, default=None, help="plain: workload seed (default: the configuration's)")
    ap.add_argument("--inflight", type=int, default=None,
                    help="plain, fragments: steps in flight on as many streams (1: enqueue a step, wait for it; "
                         "default 1 for plain, 2 for fragments)")
    ap.add_argument("--overlap", choices=["auto", "kernel", "scan", "off"], default="auto",
                    help="with --inflight 2 or more: what of a step the next step's scan waits for: its scan kernel "
                         "(kernel: the compaction, confirmation and ids copy run beside the next scan), its scan "
                         "and compaction (scan), or the whole step (off); auto: kernel for fragments, off for plain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true", help="plain: skip the streaming-read ceiling")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a 4 GiB device copy (counter scaling)")
    return ap


def main():
    args = arg_parser().parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the scan has no cross-GPU step, and only --gpus 1 is supported "
              "(sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy()
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "report":
        out = run_report(args)
    elif args.workload == "plain":
        out = run_plain(args, args.config, with_cpu=not args.no_cpu_baseline, with_ceiling=not args.no_ceiling)
    elif args.workload == "batched":
        out = run_batched(args)
    elif args.workload == "served":
        out = run_served(args)
    else:
        {"layouts": run_layouts, "fragments": run_fragments, "ingest": run_ingest}[args.workload](args)
        return
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
