"""Pins of the CPU oracle against facts fixed by the paper and by arithmetic.

Each check takes the oracle's ctypes library as an argument, so the mutation
test can run the same checks against deliberately broken builds of the oracle.
Every check raises AssertionError on failure.
"""
from __future__ import annotations

import os
import random

import numpy as np

import oracle
from oracle import spec

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MOD = 1 << 64
SECTOR = 512


def golden_vectors():
    out = []
    with open(os.path.join(GOLDEN, "djb2_eq1_vectors.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            hx, val = line.split()[:2]
            out.append((b"" if hx == "-" else bytes.fromhex(hx), int(val)))
    return out


# ---------------------------------------------------------------- signature
def pin_golden(lib):
    """Hand-worked values of Eq. (1)."""
    for data, want in golden_vectors():
        got = oracle.djb2(data, lib=lib)
        assert got == want, (data, got, want)


def pin_constant_sectors(lib):
    """A sector of 512 copies of byte c has the geometric-series value
    5381*33^512 + c*(33^512 - 1)/32 (mod 2^64); c = 0 is 5381*33^512."""
    p = 33 ** 512
    for c in (0, 1, 0x20, 0x7F, 0x80, 0xFF):
        want = (5381 * p + c * ((p - 1) // 32)) % MOD
        got = oracle.djb2(bytes([c]) * SECTOR, lib=lib)
        assert got == want, (c, hex(got), hex(want))


def pin_closed_form(lib, n=64, seed=7):
    """Random sectors: the oracle equals the unrolled closed form of Eq. (1)."""
    rng = random.Random(seed)
    for _ in range(n):
        s = bytes(rng.getrandbits(8) for _ in range(SECTOR))
        assert oracle.djb2(s, lib=lib) == spec.djb2_closed(s)


def pin_mod32(lib, n=64, seed=8):
    """33 = 1 (mod 32), so h mod 32 = (5381 + sum of bytes) mod 32."""
    rng = random.Random(seed)
    for _ in range(n):
        s = bytes(rng.getrandbits(8) for _ in range(SECTOR))
        assert oracle.djb2(s, lib=lib) % 32 == (5381 + sum(s)) % 32


def pin_collisions(lib, n=32, seed=9):
    """(a, b) -> (a+1, b-33) at adjacent positions keeps the signature."""
    rng = random.Random(seed)
    done = 0
    while done < n:
        s = bytes(rng.getrandbits(8) for _ in range(SECTOR))
        i = rng.randrange(SECTOR - 1)
        if s[i] > 254 or s[i + 1] < 33:
            continue
        t = spec.collide(s, i)
        assert t != s
        assert oracle.djb2(t, lib=lib) == oracle.djb2(s, lib=lib)
        done += 1


def pin_crafted(lib, seed=10):
    """Sectors crafted in base 33 reach any chosen signature."""
    rng = random.Random(seed)
    for target in (0, 1, 5381, MOD - 1, rng.getrandbits(64), rng.getrandbits(64)):
        prefix = bytes(rng.getrandbits(8) for _ in range(rng.randrange(0, 400)))
        assert oracle.djb2(spec.craft_sector(prefix, target), lib=lib) == target


def pin_batch_signatures(lib, seed=11):
    """The threaded per-sector routine agrees with the one-sector routine."""
    rng = np.random.default_rng(seed)
    secs = rng.integers(0, 256, size=(257, SECTOR), dtype=np.uint8)
    got = oracle.sector_signatures(secs, threads=3, lib=lib)
    for i in range(0, 257, 16):
        assert int(got[i]) == spec.djb2_closed(secs[i].tobytes())


SIGNATURE_PINS = [pin_golden, pin_constant_sectors, pin_closed_form, pin_mod32, pin_collisions,
                  pin_crafted, pin_batch_signatures]


# ------------------------------------------------- CRC-64 (Section 2.1 reading)
def crc_catalogue():
    out = []
    with open(os.path.join(GOLDEN, "crc64_catalogue.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            hx, name, val = line.split()[:3]
            out.append((bytes.fromhex(hx), name, int(val, 16)))
    return out


CRC_PARAMS = {"CRC-64/GO-ISO": spec.CRC64_GO_ISO, "CRC-64/XZ": spec.CRC64_XZ}


def pin_crc_catalogue(lib):
    """The oracle's CRC-64 gives the published CRC-64/GO-ISO check value."""
    for data, name, want in crc_catalogue():
        if name == "CRC-64/GO-ISO":
            got = oracle.crc64(data, lib=lib)
            assert got == want, (hex(got), hex(want))


def pin_crc_division(lib, n=24, seed=13):
    """Special and random sectors: the oracle equals the polynomial-division
    definition (itself checked against zlib and the catalogue)."""
    rng = random.Random(seed)
    secs = [bytes(SECTOR), b"\xff" * SECTOR, bytes(i & 255 for i in range(SECTOR))]
    secs += [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(n)]
    for s in secs:
        assert oracle.crc64(s, lib=lib) == spec.crc_polydiv(s)


def pin_crc_affine(lib, n=16, seed=14):
    """A CRC with fixed length is affine over GF(2): crc(a^b^c) = crc(a)^crc(b)^crc(c)."""
    rng = random.Random(seed)
    for _ in range(n):
        a, b, c = (bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(3))
        x = bytes(p ^ q ^ r for p, q, r in zip(a, b, c))
        assert oracle.crc64(x, lib=lib) == oracle.crc64(a, lib=lib) ^ oracle.crc64(b, lib=lib) ^ oracle.crc64(c, lib=lib)


def pin_crc_collisions(lib, seed=15):
    """Flipping the bits of x^k P(x) keeps the CRC."""
    rng = random.Random(seed)
    s = bytes(rng.getrandbits(8) for _ in range(SECTOR))
    for k in (0, 7, 1000, 4096 - 65):
        t = spec.crc_collide(s, k)
        assert t != s and oracle.crc64(t, lib=lib) == oracle.crc64(s, lib=lib)


def pin_crc_sector_signatures(lib, seed=16):
    """The threaded per-sector routine with the CRC kind equals the one-sector routine."""
    rng = np.random.default_rng(seed)
    secs = rng.integers(0, 256, size=(129, SECTOR), dtype=np.uint8)
    got = oracle.sector_signatures(secs, threads=3, lib=lib, sig_kind=oracle.SIG_CRC64_GO_ISO)
    for i in range(0, 129, 8):
        assert int(got[i]) == spec.crc_bytewise(secs[i].tobytes())


SIGNATURE_PINS += [pin_crc_catalogue, pin_crc_division, pin_crc_affine, pin_crc_collisions,
                   pin_crc_sector_signatures]


# ----------------------------------------------------------- sets of results
def small_case(seed=3, n_disk=700, tail=77):
    """A tiny master set with uneven file sizes and a disk image with planted
    clusters, partial overwrites, duplicates, zero sectors and crafted
    signature collisions, as raw bytes."""
    rng = random.Random(seed)
    sizes = [37, 8, 21, 64, 3, 50]                 # sectors per file, not multiples of 8
    masters = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(sum(sizes))]
    offsets = [0]
    for s in sizes:
        offsets.append(offsets[-1] + s)
    # duplicates: same bytes at the same and at another cluster position
    masters[offsets[3] + 9] = masters[offsets[0] + 1]      # tau 1 == tau 1
    masters[offsets[5] + 4] = masters[offsets[0] + 1]      # tau 4 != tau 1
    masters[offsets[2] + 5] = masters[offsets[1] + 2]      # tau 5 != tau 2
    disk = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(n_disk)]
    truth = []
    for c in range(n_disk // 8):
        u = rng.random()
        if u < 0.3:
            f = rng.randrange(len(sizes))
            ncl = sizes[f] // 8
            if ncl == 0:
                continue
            q = rng.randrange(ncl)
            r = rng.choice([0, 0, 1, 2, 3])
            for i in range(r, 8):
                disk[8 * c + i] = masters[offsets[f] + 8 * q + i]
                truth.append((8 * c + i, f, 8 * q + i))
        elif u < 0.35:
            for i in range(8):
                disk[8 * c + i] = bytes(SECTOR)
        elif u < 0.45:
            # crafted collision of a master sector at the right position, near the end of
            # the sector: flagged, not equal
            f = rng.randrange(len(sizes))
            k = rng.randrange(sizes[f])
            i = k % 8
            src = masters[offsets[f] + k]
            pos = next(p for p in range(SECTOR - 2, 0, -1) if src[p] <= 254 and src[p + 1] >= 33)
            disk[8 * c + i] = spec.collide(src, pos)
    image = b"".join(disk) + bytes(rng.getrandbits(8) for _ in range(tail))
    return image, masters, offsets, truth


def _as_tuples(arr):
    return [(int(r["disk_sector"]), int(r["file_id"]), int(r["sector_in_file"])) for r in arr]


def pin_sets_vs_definition(lib, seed=3):
    """Flags equal the definition computed with the closed form and Python sets;
    confirmed matches equal a pure-Python all-pairs byte comparison; the C
    brute force agrees; every planted sector is flagged and confirmed."""
    image, masters, offsets, truth = small_case(seed)
    mflat = b"".join(masters)
    for tau0, any_tau in ((0, False), (3, False), (7, False), (0, True)):
        ix = oracle.Index(np.frombuffer(mflat, np.uint8), offsets, threads=2, lib=lib)
        flags = [int(x) for x in ix.flag_image(np.frombuffer(image, np.uint8), tau0, any_tau, threads=2)]
        want_flags = spec.flagged_by_definition(image, masters, offsets, tau0, any_tau)
        assert flags == want_flags, (tau0, any_tau)
        conf = _as_tuples(ix.confirm_image(np.frombuffer(image, np.uint8), flags, tau0, any_tau))
        want = spec.brute_force_matches(image, masters, offsets, tau0, any_tau)
        assert conf == want, (tau0, any_tau)
        brute = _as_tuples(oracle.bruteforce(np.frombuffer(image, np.uint8), np.frombuffer(mflat, np.uint8),
                                             offsets, tau0, any_tau, threads=2, lib=lib))
        assert brute == want
        assert set(j for j, _, _ in want) <= set(flags)
        if tau0 == 0 and not any_tau:
            assert set(truth) <= set(want)
            # crafted collisions exist and are flagged without being confirmed
            assert len(set(flags) - set(j for j, _, _ in want)) > 0


def pin_edges(lib):
    """Empty image, sub-sector image, empty master set, all-zero disk against a
    zero master sector, and a master whose signature is 0."""
    rng = random.Random(12)
    masters = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(9)]
    ix = oracle.Index(np.frombuffer(b"".join(masters), np.uint8), [0, 9], lib=lib)
    assert ix.flag_image(np.zeros(0, np.uint8)).size == 0
    assert ix.flag_image(np.frombuffer(masters[0][:511], np.uint8)).size == 0
    empty = oracle.Index(np.zeros(0, np.uint8), [0], lib=lib)
    assert empty.flag_image(np.frombuffer(b"".join(masters), np.uint8)).size == 0
    # zero master sector at cluster position 2: every zero disk sector at position 2 is flagged
    zm = list(masters)
    zm[2] = bytes(SECTOR)
    zix = oracle.Index(np.frombuffer(b"".join(zm), np.uint8), [0, 9], lib=lib)
    got = [int(x) for x in zix.flag_image(np.zeros(64 * SECTOR, np.uint8))]
    assert got == [j for j in range(64) if j % 8 == 2]
    got = [int(x) for x in zix.flag_image(np.zeros(64 * SECTOR, np.uint8), any_tau=True)]
    assert got == list(range(64))
    # a master sector whose signature is 0 is matched like any other
    crafted = spec.craft_sector(b"sig-zero", 0)
    cm = list(masters)
    cm[5] = crafted
    cix = oracle.Index(np.frombuffer(b"".join(cm), np.uint8), [0, 9], lib=lib)
    disk = bytearray(rng.getrandbits(8) for _ in range(16 * SECTOR))
    disk[13 * SECTOR:14 * SECTOR] = crafted
    assert [int(x) for x in cix.flag_image(np.frombuffer(bytes(disk), np.uint8))] == [13]


def crc_small_case(seed=4, n_disk=400):
    """The small case's layout with CRC collisions crafted in place of the djb2 ones."""
    image, masters, offsets, truth = small_case(seed, n_disk=n_disk, tail=33)
    rng = random.Random(seed + 100)
    img = bytearray(image)
    replaced = set()
    for c in range(0, n_disk // 8, 5):
        f = rng.randrange(len(offsets) - 1)
        k = rng.randrange(offsets[f + 1] - offsets[f])
        j = 8 * c + k % 8                                  # the master's cluster position
        img[j * SECTOR:(j + 1) * SECTOR] = spec.crc_collide(masters[offsets[f] + k], rng.randrange(4000))
        replaced.add(j)
    return bytes(img), masters, offsets, [t for t in truth if t[0] not in replaced]


def pin_crc_sets(lib, seed=4):
    """With the CRC signature: flags equal the definition (byte-wise CRC and
    Python sets), confirmed matches equal the all-pairs byte comparison, and
    the crafted CRC collisions are flagged without being confirmed."""
    image, masters, offsets, truth = crc_small_case(seed)
    mflat = np.frombuffer(b"".join(masters), np.uint8)
    sig_cache = {}

    def sig(b):
        if b not in sig_cache:
            sig_cache[b] = spec.crc_bytewise(b)
        return sig_cache[b]

    ix = oracle.Index(mflat, offsets, threads=2, lib=lib, sig_kind=oracle.SIG_CRC64_GO_ISO)
    img = np.frombuffer(image, np.uint8)
    for tau0, any_tau in ((0, False), (5, False), (0, True)):
        flags = [int(x) for x in ix.flag_image(img, tau0, any_tau, threads=2)]
        assert flags == spec.flagged_by_definition(image, masters, offsets, tau0, any_tau, sig=sig), (tau0, any_tau)
        conf = _as_tuples(ix.confirm_image(img, flags, tau0, any_tau))
        assert conf == spec.brute_force_matches(image, masters, offsets, tau0, any_tau)
        if tau0 == 0 and not any_tau:
            assert set(truth) <= set(conf)
            assert len(set(flags) - set(j for j, _, _ in conf)) > 0


# ------------------------------------------------- fragments (Section 5)
def fragment_small_case(seed=21, n_bytes=48 * 1024):
    """Master files of uneven byte lengths (a trailing partial fragment, a
    file too short for any), a duplicated fragment and an all-zero one; an
    image with whole files planted at 4-byte aligned offsets (found) and at
    offsets that are not (not found unless by chance), crafted djb2 collisions
    of fragments at aligned offsets, a zero run, and a ragged tail."""
    rng = random.Random(seed)
    sizes = [64 * 7 + 13, 64 * 3, 64 * 20 + 63, 64, 10, 64 * 5]
    files = [bytes(rng.getrandbits(8) for _ in range(n)) for n in sizes]
    f0 = bytearray(files[0])
    f0[64 * 2: 64 * 3] = files[2][64 * 5: 64 * 6]          # duplicated fragment
    files[0] = bytes(f0)
    f5 = bytearray(files[5])
    f5[64 * 4: 64 * 5] = bytes(64)                         # all-zero fragment
    files[5] = bytes(f5)
    frag_data, offsets = oracle.pack_fragment_files(files)
    fragments = [frag_data[i].tobytes() for i in range(frag_data.shape[0])]
    img = bytearray(rng.getrandbits(8) for _ in range(n_bytes + 37))
    truth = set()
    pos = 100
    while pos < n_bytes - 2000:
        f = rng.choice([0, 1, 2, 3])
        data = files[f]
        o = pos + rng.choice([0, 0, 0, 1, 2, 3]) + 4 * rng.randrange(8)
        img[o:o + len(data)] = data
        for k in range(len(data) // 64):
            if (o + 64 * k) % 4 == 0:
                truth.add(((o + 64 * k) // 4, f, k))
        pos = o + len(data) + rng.randrange(16, 400)
    tail = n_bytes - 1900                                  # past the planted files
    for i in range(12):                                    # flagged, not confirmed
        o = tail - tail % 4 + 68 * i
        src = fragments[rng.randrange(len(fragments))]
        p_ = next(q for q in range(60, 0, -1) if src[q] <= 254 and src[q + 1] >= 33)
        img[o:o + 64] = spec.collide(src, p_)
    z = tail - tail % 4 + 68 * 12 + 16
    img[z:z + 300] = bytes(300)                            # zero run: several aligned zero windows
    return bytes(img), fragments, frag_data, offsets, truth


def pin_fragment_sets(lib, seed=21):
    """Windows at every 4-byte boundary: flags equal the closed-form
    definition, confirmed matches equal a pure-Python comparison of every
    window with every fragment and the C brute force, planted aligned
    fragments are found, collisions are flagged only; edge sizes."""
    image, fragments, frag_data, offsets, truth = fragment_small_case(seed)
    ix = oracle.FragmentIndex(frag_data, offsets, threads=2, lib=lib)
    img = np.frombuffer(image, np.uint8)
    flags = [int(x) for x in ix.flag_windows(img, threads=2)]
    assert flags == spec.fragment_flags_by_definition(image, fragments)
    conf = _as_tuples(ix.confirm_windows(img, flags))
    want = spec.fragment_matches_by_comparison(image, fragments, offsets)
    assert conf == want
    assert _as_tuples(oracle.fragment_bruteforce(img, frag_data, offsets, lib=lib)) == want
    assert truth <= set(conf)
    assert len(set(flags) - set(j for j, _, _ in conf)) >= 12
    assert sum(1 for j, f, k in conf if f == 5 and k == 4) >= 50     # the zero run
    for n, want_windows in ((0, 0), (63, 0), (64, 1), (67, 1), (68, 2), (200, 35)):
        w = ix.flag_windows(np.zeros(n, np.uint8))
        assert len(w) == (want_windows if n else 0) and list(w) == list(range(len(w)))


SET_PINS = [pin_sets_vs_definition, pin_edges, pin_crc_sets, pin_fragment_sets]
ALL_PINS = SIGNATURE_PINS + SET_PINS
