"""Counter-based synthetic master sets and disk images.

Every byte is a pure function of (seed, stream name, counter), computed with
int64 torch operations that never overflow, so the same call yields the same
bytes on the CPU and on a GPU, and any sector can be regenerated alone (the
oracle's sampled checks at full size rely on that).

Data model (paper, Section 2 and Section 3.1): a sector is 512 bytes, a cluster
is 8 consecutive sectors, master files start on a cluster boundary, and a
deleted file's cluster may survive whole or with its first few sectors
overwritten by a newer file.

Disk image recipe (one seeded Bernoulli draw per 4 KiB cluster):
  * master cluster: the 8 sectors of a random full cluster of a random master
    file, copied cluster-aligned; a fraction of those get their first 1-3
    sectors replaced by random bytes (partial overwrite);
  * zero cluster: 4096 zero bytes;
  * low-entropy cluster: one 4-byte pattern, drawn from a small pool, repeated;
  * otherwise uniform random bytes (the paper's corpus was random data).
Master files are uniform random sectors, plus duplicated sectors (the same
bytes at the same or at another cluster position in another file) and, when
configured, low-entropy sectors from the same pattern pool.
"""
from __future__ import annotations

import bisect
import hashlib
import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import torch

SECTOR = 512
WORDS_PER_SECTOR = SECTOR // 4
CLUSTER = 8
_M32 = 0xFFFFFFFF
_TWO32 = 1 << 32

KIND_RANDOM, KIND_MASTER, KIND_ZERO, KIND_LOW = 0, 1, 2, 3


# --------------------------------------------------------------------------
# counter-based word generator
# --------------------------------------------------------------------------
def _key(*parts) -> tuple:
    d = hashlib.sha256(repr(parts).encode()).digest()
    return tuple(int.from_bytes(d[4 * i:4 * i + 4], "little") for i in range(3))


def _mix32(x: torch.Tensor) -> torch.Tensor:
    # 32-bit integer finaliser (xorshift-multiply, multiplier 0x45d9f3b); the
    # operand stays below 2^32 and the multiplier below 2^27, so every product
    # fits in int64 without wrapping.
    x = x ^ (x >> 16)
    x = (x * 0x45D9F3B) & _M32
    x = x ^ (x >> 16)
    x = (x * 0x45D9F3B) & _M32
    return x ^ (x >> 16)


def words(key: tuple, idx: torch.Tensor) -> torch.Tensor:
    """Pseudo-random 32-bit words (int64 values in [0, 2^32)) at counters idx >= 0."""
    k0, k1, k2 = key
    a = _mix32((idx & _M32) ^ k0)
    b = _mix32((idx >> 32) ^ k1)
    return _mix32(a ^ b ^ k2)


def _words_to_bytes(w: torch.Tensor) -> torch.Tensor:
    """int64 words in [0, 2^32), last dim k -> uint8 with last dim 4k (little-endian)."""
    w32 = torch.where(w >= (1 << 31), w - _TWO32, w).to(torch.int32)
    return w32.contiguous().view(torch.uint8)


def _scalar_words(key: tuple, idx: int, n: int = 1) -> List[int]:
    t = torch.arange(idx, idx + n, dtype=torch.int64)
    return [int(v) for v in words(key, t)]


def _threshold(p: float) -> int:
    return int(round(p * _TWO32))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class CarveConfig:
    name: str
    seed: int
    n_master_sectors: int
    n_files: int
    equal_files: bool           # equal file sizes, else random cut points
    n_disk_sectors: int
    p_master_cluster: float
    p_overwrite: float          # share of copied clusters with 1-3 sectors overwritten
    p_zero: float
    p_low_entropy: float
    n_dup_same_tau: int
    n_dup_other_tau: int
    tail_bytes: int = 0         # bytes after the last full sector
    low_pattern_pool: int = 4096
    n_low_masters: int = 0      # master sectors holding a low-entropy pattern

    @property
    def image_bytes(self) -> int:
        return self.n_disk_sectors * SECTOR + self.tail_bytes


CONFIGS = {
    # 8 files x 256 KiB, 64 MiB image (131072 sectors)
    "tiny": CarveConfig("tiny", 1, 4096, 8, True, 131072, 0.05, 0.5, 0.02, 0.0, 8, 8),
    # 1M master sectors (512 MiB), 8 GiB image (16M sectors)
    "mid": CarveConfig("mid", 1, 1 << 20, 1000, False, 1 << 24, 0.01, 0.3, 0.05, 0.0, 524, 525),
    # 16M master sectors (8 GiB), 64 GiB image (128M sectors)
    "large": CarveConfig("large", 1, 1 << 24, 10000, False, 1 << 27, 0.001, 0.3, 0.0, 0.10,
                         1024, 1024, n_low_masters=64),
    # resident index of the served workload: 4M master sectors
    "served": CarveConfig("served", 1, 1 << 22, 4000, False, 1 << 22, 0.02, 0.3, 0.02, 0.02,
                          512, 512, n_low_masters=16),
}


def scaled(cfg: CarveConfig, n_master_sectors: int, n_disk_sectors: int, **kw) -> CarveConfig:
    """A smaller copy of a configuration with the same recipe."""
    n_files = kw.pop("n_files", max(1, min(cfg.n_files, n_master_sectors // 64)))
    return replace(cfg, n_master_sectors=n_master_sectors, n_disk_sectors=n_disk_sectors,
                   n_files=n_files, **kw)


# --------------------------------------------------------------------------
# master set
# --------------------------------------------------------------------------
@dataclass
class MasterSet:
    cfg: CarveConfig
    sectors: torch.Tensor               # uint8 [M, 512]
    file_offsets: List[int]             # CSR of sector ranges per file, len n_files+1
    full_cluster_starts: torch.Tensor   # int64, first sector of every full master cluster
    dup_dst: torch.Tensor               # int64, sorted; master sectors that copy another
    dup_src: torch.Tensor               # int64, aligned with dup_dst
    low_ids: torch.Tensor               # int64, sorted; low-entropy master sectors
    low_pattern: torch.Tensor           # int64 pattern word per low_ids entry

    @property
    def n_files(self) -> int:
        return len(self.file_offsets) - 1


def _file_offsets(cfg: CarveConfig) -> List[int]:
    m = cfg.n_master_sectors
    if cfg.equal_files or cfg.n_files <= 1:
        nf = max(1, cfg.n_files)
        return [f * m // nf for f in range(nf + 1)]
    k = _key(cfg.seed, cfg.name, "file-cuts")
    cuts = words(k, torch.arange(cfg.n_files - 1, dtype=torch.int64)) % (m - 1) + 1
    cuts = sorted(set(int(c) for c in cuts))
    return [0] + cuts + [m]


def _file_of(offsets: List[int], s: int) -> int:
    lo, hi = 0, len(offsets) - 2
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if offsets[mid] <= s:
            lo = mid
        else:
            hi = mid - 1
    return lo


def _pick_dups(cfg: CarveConfig, offsets: List[int]):
    """Sector pairs (dst, src): dst in another file gets src's bytes."""
    m = cfg.n_master_sectors
    nf = len(offsets) - 1
    dst_set, src_set, pairs = set(), set(), []
    if nf < 2:
        return pairs
    for which, count in (("same", cfg.n_dup_same_tau), ("other", cfg.n_dup_other_tau)):
        k = _key(cfg.seed, cfg.name, "dup", which)
        ctr = 0
        made = 0
        while made < count and ctr < 64 * (count + 16):
            w = _scalar_words(k, 4 * ctr, 4)
            ctr += 1
            src = w[0] % m
            fs = _file_of(offsets, src)
            tau = (src - offsets[fs]) % CLUSTER
            if which == "other":
                tau = (tau + 1 + w[1] % (CLUSTER - 1)) % CLUSTER
            fd = w[2] % nf
            if fd == fs:
                continue
            ln = offsets[fd + 1] - offsets[fd]
            if ln <= tau:
                continue
            q = w[3] % ((ln - tau + CLUSTER - 1) // CLUSTER)
            dst = offsets[fd] + CLUSTER * q + tau
            if dst in dst_set or dst in src_set or src in dst_set:
                continue
            dst_set.add(dst)
            src_set.add(src)
            pairs.append((dst, src))
            made += 1
    return pairs


def _pattern_pool_word(cfg: CarveConfig, p: torch.Tensor) -> torch.Tensor:
    return words(_key(cfg.seed, cfg.name, "pattern-pool"), p)


def master_words(ms: MasterSet, ids: torch.Tensor) -> torch.Tensor:
    """Content words [n, 128] of master sectors ids (int64 tensor on any device)."""
    cfg = ms.cfg
    dev = ids.device
    base = ids
    if ms.dup_dst.numel():
        dd, dsrc = ms.dup_dst.to(dev), ms.dup_src.to(dev)
        pos = torch.searchsorted(dd, ids).clamp(max=dd.numel() - 1)
        hit = dd[pos] == ids
        base = torch.where(hit, dsrc[pos], ids)
    ar = torch.arange(WORDS_PER_SECTOR, dtype=torch.int64, device=dev)
    w = words(_key(cfg.seed, cfg.name, "master"), base[:, None] * WORDS_PER_SECTOR + ar[None, :])
    if ms.low_ids.numel():
        li, lp = ms.low_ids.to(dev), ms.low_pattern.to(dev)
        pos = torch.searchsorted(li, ids).clamp(max=li.numel() - 1)
        hit = li[pos] == ids
        w = torch.where(hit[:, None], lp[pos][:, None], w)
    return w


def master_sectors(ms: MasterSet, ids: torch.Tensor) -> torch.Tensor:
    """Bytes [n, 512] of master sectors ids."""
    return _words_to_bytes(master_words(ms, ids))


def master_set(cfg: CarveConfig, device="cpu", chunk: int = 1 << 18) -> MasterSet:
    offsets = _file_offsets(cfg)
    off = torch.tensor(offsets, dtype=torch.int64)
    lens = off[1:] - off[:-1]
    ncl = lens // CLUSTER
    total = int(ncl.sum())
    first = torch.cumsum(ncl, 0) - ncl
    starts = (torch.repeat_interleave(off[:-1], ncl)
              + CLUSTER * (torch.arange(total, dtype=torch.int64) - torch.repeat_interleave(first, ncl)))
    pairs = sorted(_pick_dups(cfg, offsets))
    dup_dst = torch.tensor([p[0] for p in pairs], dtype=torch.int64)
    dup_src = torch.tensor([p[1] for p in pairs], dtype=torch.int64)
    low_ids = torch.empty(0, dtype=torch.int64)
    low_pat = torch.empty(0, dtype=torch.int64)
    if cfg.n_low_masters:
        k = _key(cfg.seed, cfg.name, "low-masters")
        taken = set(int(v) for v in dup_dst) | set(int(v) for v in dup_src)
        ids, ctr = [], 0
        while len(ids) < cfg.n_low_masters and ctr < 64 * cfg.n_low_masters:
            s = _scalar_words(k, ctr)[0] % cfg.n_master_sectors
            ctr += 1
            if s not in taken:
                taken.add(s)
                ids.append(s)
        ids.sort()
        low_ids = torch.tensor(ids, dtype=torch.int64)
        sel = words(_key(cfg.seed, cfg.name, "low-master-pick"), low_ids) % cfg.low_pattern_pool
        low_pat = _pattern_pool_word(cfg, sel)
    ms = MasterSet(cfg, torch.empty(0), offsets, starts, dup_dst, dup_src, low_ids, low_pat)
    m = cfg.n_master_sectors
    out = torch.empty((m, SECTOR), dtype=torch.uint8, device=device)
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        out[s:e] = master_sectors(ms, torch.arange(s, e, dtype=torch.int64, device=device))
    ms.sectors = out
    return ms


# --------------------------------------------------------------------------
# disk images
# --------------------------------------------------------------------------
@dataclass
class DiskImage:
    cfg: CarveConfig
    image_id: int
    data: torch.Tensor                  # uint8 [n_disk_sectors*512 + tail_bytes]
    planted_clusters: torch.Tensor      # int64 disk cluster ids holding a master cluster
    planted_src: torch.Tensor           # int64 first master sector of the copied cluster
    planted_overwrite: torch.Tensor     # int64 number of leading sectors overwritten (0-3)
    kind_counts: dict = field(default_factory=dict)


def _cluster_plan(cfg: CarveConfig, ms: MasterSet, c: torch.Tensor, image_id: int):
    """Kind, source master sector and overwrite count for disk clusters c."""
    kk = lambda name: _key(cfg.seed, cfg.name, image_id, name)  # noqa: E731
    u = words(kk("kind"), c)
    t_m = _threshold(cfg.p_master_cluster)
    t_z = t_m + _threshold(cfg.p_zero)
    t_l = t_z + _threshold(cfg.p_low_entropy)
    kind = torch.full_like(c, KIND_RANDOM)
    kind = torch.where(u < t_l, torch.full_like(c, KIND_LOW), kind)
    kind = torch.where(u < t_z, torch.full_like(c, KIND_ZERO), kind)
    n_full = ms.full_cluster_starts.numel()
    if n_full:
        kind = torch.where(u < t_m, torch.full_like(c, KIND_MASTER), kind)
    fcs = ms.full_cluster_starts.to(c.device)
    src = fcs[words(kk("src"), c) % max(n_full, 1)] if n_full else torch.zeros_like(c)
    ow = words(kk("overwrite"), c) < _threshold(cfg.p_overwrite)
    r = torch.where(ow, 1 + words(kk("overwrite-count"), c) % 3, torch.zeros_like(c))
    pat = _pattern_pool_word(cfg, words(kk("pattern"), c) % cfg.low_pattern_pool)
    return kind, src, r, pat


def disk_sectors(cfg: CarveConfig, ms: MasterSet, ids: torch.Tensor, image_id: int = 0) -> torch.Tensor:
    """Bytes [n, 512] of disk sectors ids of image image_id (any device)."""
    dev = ids.device
    c = ids // CLUSTER
    i = ids % CLUSTER
    kind, src, r, pat = _cluster_plan(cfg, ms, c, image_id)
    ar = torch.arange(WORDS_PER_SECTOR, dtype=torch.int64, device=dev)
    w = words(_key(cfg.seed, cfg.name, image_id, "random"), ids[:, None] * WORDS_PER_SECTOR + ar[None, :])
    w = torch.where((kind == KIND_ZERO)[:, None], torch.zeros_like(w), w)
    w = torch.where((kind == KIND_LOW)[:, None], pat[:, None].expand_as(w), w)
    use = (kind == KIND_MASTER) & (i >= r)
    if bool(use.any()):
        w[use] = master_words(ms, (src + i)[use])
    return _words_to_bytes(w)


def disk_image(cfg: CarveConfig, ms: MasterSet, device="cpu", image_id: int = 0,
               chunk: int = 1 << 18, out: Optional[torch.Tensor] = None) -> DiskImage:
    n = cfg.n_disk_sectors
    nbytes = n * SECTOR + cfg.tail_bytes
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=device)
    assert out.numel() >= nbytes
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ids = torch.arange(s, e, dtype=torch.int64, device=device)
        out[s * SECTOR:e * SECTOR] = disk_sectors(cfg, ms, ids, image_id).reshape(-1)
    if cfg.tail_bytes:
        tw = words(_key(cfg.seed, cfg.name, image_id, "tail"),
                   torch.arange((cfg.tail_bytes + 3) // 4, dtype=torch.int64, device=device))
        out[n * SECTOR:nbytes] = _words_to_bytes(tw)[:cfg.tail_bytes]
    # ground truth of the planted clusters
    pc, ps, pr = [], [], []
    counts = {KIND_RANDOM: 0, KIND_MASTER: 0, KIND_ZERO: 0, KIND_LOW: 0}
    n_cl = n // CLUSTER
    for s in range(0, n_cl, 1 << 22):
        e = min(n_cl, s + (1 << 22))
        c = torch.arange(s, e, dtype=torch.int64, device=device)
        kind, src, r, _ = _cluster_plan(cfg, ms, c, image_id)
        for kd in counts:
            counts[kd] += int((kind == kd).sum())
        sel = kind == KIND_MASTER
        pc.append(c[sel].cpu())
        ps.append(src[sel].cpu())
        pr.append(r[sel].cpu())
    cat = lambda xs: torch.cat(xs) if xs else torch.empty(0, dtype=torch.int64)  # noqa: E731
    return DiskImage(cfg, image_id, out[:nbytes], cat(pc), cat(ps), cat(pr), counts)


# --------------------------------------------------------------------------
# batched and served workloads
# --------------------------------------------------------------------------
def batch_image_specs(seed: int = 1, n_images: int = 256, min_bytes: int = 1 << 20,
                      max_bytes: int = 1 << 30, max_hit: float = 0.05):
    """Sizes log-uniform in [min_bytes, max_bytes] rounded to 4 KiB, hit rate uniform in [0, max_hit]."""
    k = _key(seed, "batch-specs")
    w = words(k, torch.arange(2 * n_images, dtype=torch.int64)).double() / _TWO32
    lo, hi = math.log(min_bytes), math.log(max_bytes)
    specs = []
    for i in range(n_images):
        size = int(math.exp(lo + (hi - lo) * float(w[2 * i])))
        size = max(4096, (size // 4096) * 4096)
        specs.append((size // SECTOR, max_hit * float(w[2 * i + 1])))
    return specs


def batch_images(cfg: CarveConfig, ms: MasterSet, device="cpu", n_images: int = 256) -> List[torch.Tensor]:
    """The batched workload's images: sizes and hit rates from
    batch_image_specs(cfg.seed, n_images), each image drawn with cfg's recipe
    (its own image_id)."""
    out = []
    for i, (n_sec, hit) in enumerate(batch_image_specs(seed=cfg.seed, n_images=n_images)):
        c = replace(cfg, n_disk_sectors=n_sec, p_master_cluster=hit)
        out.append(disk_image(c, ms, device=device, image_id=i).data)
    return out


# image ids reserved for samples that are never the measured image
TUNING_IMAGE_ID = 1 << 20


def tuning_sample(cfg: CarveConfig, ms: MasterSet, device="cpu", max_sectors: int = 1 << 22) -> torch.Tensor:
    """An image with cfg's recipe but other bytes than the benchmark's image
    (its own image_id), of at most max_sectors sectors (2 GiB): what a
    launch-shape or layout autotuner times instead of the image it will scan."""
    c = replace(cfg, n_disk_sectors=min(cfg.n_disk_sectors, max_sectors), tail_bytes=0)
    return disk_image(c, ms, device=device, image_id=TUNING_IMAGE_ID).data


def served_job_specs(seed: int = 1, rate: float = 2000.0, duration: float = 60.0,
                     min_bytes: int = 64 << 10, max_bytes: int = 256 << 20,
                     any_tau_below: int = 1 << 20):
    """Poisson arrivals: (arrival time s, size bytes (multiple of 512), tau_any flag)."""
    n_max = int(rate * duration * 1.5) + 64
    k = _key(seed, "served-specs")
    w = (words(k, torch.arange(2 * n_max, dtype=torch.int64)).double() + 0.5) / _TWO32
    gaps = -torch.log(w[0::2]) / rate
    t = torch.cumsum(gaps, 0)
    n = int((t < duration).sum())
    lo, hi = math.log(min_bytes), math.log(max_bytes)
    sizes = torch.exp(lo + (hi - lo) * w[1::2][:n])
    sizes = (sizes / SECTOR).floor().to(torch.int64).clamp(min=1) * SECTOR
    return [(float(t[i]), int(sizes[i]), int(sizes[i]) < any_tau_below) for i in range(n)]


def served_job_slices(specs, pool_sectors: int, seed: int = 1):
    """First pool sector of each served job: cluster-aligned for disk-image
    chunks (their first sector sits at cluster position 0), any sector for
    flow buffers. specs: served_job_specs() output."""
    k = _key(seed, "served-slices")
    w = words(k, torch.arange(len(specs), dtype=torch.int64))
    out = []
    for (t, size, flow), r in zip(specs, w.tolist()):
        room = max(1, pool_sectors - (size + SECTOR - 1) // SECTOR)
        first = r % room
        if not flow:
            first -= first % CLUSTER
        out.append(first)
    return out


# --------------------------------------------------------------------------
# fragments (Section 5): small files embedded in a larger image
# --------------------------------------------------------------------------
@dataclass
class FragmentConfig:
    name: str
    seed: int
    n_files: int          # master "logo" files
    min_bytes: int        # their sizes: log-uniform in [min_bytes, max_bytes]
    max_bytes: int
    image_bytes: int
    n_embedded: int       # whole copies of master files placed in the image
    p_aligned: float      # share of copies that start on a 4-byte boundary


FRAGMENT_CONFIGS = {
    # 2000 logos of 2-32 KiB (about 22 MB, 346,577 fragments), 25000 copies in a
    # 2 GiB image (a scan keeps about 15 B of workspace per 4-byte window)
    "logos": FragmentConfig("logos", 1, 2000, 2048, 32768, 2 << 30, 25000, 0.8),
}


def fragment_files(cfg: FragmentConfig, device="cpu") -> List[torch.Tensor]:
    """The master files' bytes (uint8 tensors of log-uniform sizes)."""
    k = _key(cfg.seed, cfg.name, "frag-files")
    r = words(k, torch.arange(cfg.n_files, dtype=torch.int64)).double() / float(1 << 32)
    lo, hi = float(cfg.min_bytes), float(cfg.max_bytes)
    sizes = torch.exp(torch.log(torch.tensor(lo)) + r * (torch.log(torch.tensor(hi)) - torch.log(torch.tensor(lo))))
    out = []
    for f, n in enumerate(sizes.long().tolist()):
        w = words(_key(cfg.seed, cfg.name, "frag-file", f), torch.arange((n + 3) // 4, dtype=torch.int64, device=device))
        out.append(_words_to_bytes(w)[:n].clone())
    return out


def fragment_image(cfg: FragmentConfig, files: List[torch.Tensor], device="cpu",
                   chunk_words: int = 1 << 26) -> torch.Tensor:
    """Uniform random bytes with n_embedded whole copies of master files, each
    at an offset that is a multiple of 4 with probability p_aligned (else 1-3
    past one). Later copies may overwrite earlier ones."""
    n = cfg.image_bytes
    img = torch.empty(n, dtype=torch.uint8, device=device)
    k = _key(cfg.seed, cfg.name, "frag-image")
    n_words = (n + 3) // 4
    for w0 in range(0, n_words, chunk_words):
        w1 = min(n_words, w0 + chunk_words)
        b = _words_to_bytes(words(k, torch.arange(w0, w1, dtype=torch.int64, device=device)))
        img[4 * w0: min(n, 4 * w1)] = b[: min(n, 4 * w1) - 4 * w0]
    places = fragment_placements(cfg, [f.numel() for f in files])
    # The copies are placed in order, a later one overwriting an earlier one
    # where they overlap; the bytes each copy keeps (those no later copy
    # covers) are found on the host, so that every image byte is written at
    # most once and all copies go in with one device scatter.
    starts, ends = [], []            # disjoint intervals covered by later copies, ascending
    pieces = []                      # (image offset, file, offset in the file, length)
    for o, f in reversed(places):
        a, b = o, o + files[f].numel()
        i = j = bisect.bisect_right(ends, a)
        cur = a
        while j < len(starts) and starts[j] < b:
            if starts[j] > cur:
                pieces.append((cur, f, cur - o, starts[j] - cur))
            cur = max(cur, ends[j])
            j += 1
        if cur < b:
            pieces.append((cur, f, cur - o, b - cur))
        na, nb = (min(a, starts[i]), max(b, ends[j - 1])) if j > i else (a, b)
        starts[i:j], ends[i:j] = [na], [nb]
    if not pieces:
        return img
    file_start = [0]
    for f in files:
        file_start.append(file_start[-1] + f.numel())
    src = torch.cat([f.to(device) for f in files])
    dst0 = torch.tensor([p[0] for p in pieces], dtype=torch.int64, device=device)
    src0 = torch.tensor([file_start[p[1]] + p[2] for p in pieces], dtype=torch.int64, device=device)
    lens = torch.tensor([p[3] for p in pieces], dtype=torch.int64, device=device)
    within = torch.arange(int(lens.sum()), dtype=torch.int64, device=device) - torch.repeat_interleave(
        torch.cumsum(lens, 0) - lens, lens)
    img[torch.repeat_interleave(dst0, lens) + within] = src[torch.repeat_interleave(src0, lens) + within]
    return img


def fragment_placements(cfg: FragmentConfig, file_sizes: List[int]):
    """(image offset, file) of each embedded copy, in placement order: an
    offset that is a multiple of 4 with probability p_aligned, else 1-3 past
    one; copies that would not fit are skipped."""
    n = cfg.image_bytes
    kp = _key(cfg.seed, cfg.name, "frag-plant")
    r = words(kp, torch.arange(3 * cfg.n_embedded, dtype=torch.int64)).view(-1, 3).tolist()
    thr = _threshold(cfg.p_aligned)
    out = []
    for fsel, osel, asel in r:
        f = fsel % len(file_sizes)
        room = n - file_sizes[f]
        if room <= 4:
            continue
        o = osel % (room - 4)
        o -= o % 4
        if asel >= thr:
            o += 1 + asel % 3
        out.append((o, f))
    return out
