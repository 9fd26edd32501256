"""The CPU oracle against values and facts fixed by the paper and by arithmetic."""
import pytest

import oracle
import pins
from oracle import spec


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(lib, pin):
    pin(lib)


def test_spec_forms_agree_on_golden():
    # the two pure-Python forms against the hand-worked values
    for data, want in pins.golden_vectors():
        assert spec.djb2_horner(data) == want
        assert spec.djb2_closed(data) == want


def test_spec_crc_forms_against_zlib():
    # the generic CRC forms, with CRC-32 parameters, against the zlib library routine
    import random
    import zlib
    rng = random.Random(17)
    for n in (0, 1, 3, 8, 9, 100, 512, 1031):
        d = bytes(rng.getrandbits(8) for _ in range(n))
        want = zlib.crc32(d)
        assert spec.crc_register(d, spec.CRC32_ZLIB) == want
        assert spec.crc_polydiv(d, spec.CRC32_ZLIB) == want
        assert spec.crc_bytewise(d, spec.CRC32_ZLIB) == want


def test_spec_crc_forms_against_catalogue():
    for data, name, want in pins.crc_catalogue():
        params = pins.CRC_PARAMS[name]
        assert spec.crc_register(data, params) == want, name
        assert spec.crc_polydiv(data, params) == want, name
        assert spec.crc_bytewise(data, params) == want, name


def test_spec_crc_collide_is_a_collision():
    import random
    rng = random.Random(18)
    s = bytes(rng.getrandbits(8) for _ in range(512))
    for k in (0, 3, 511, 4030):
        t = spec.crc_collide(s, k)
        assert t != s and spec.crc_polydiv(t) == spec.crc_polydiv(s)
        assert sum(bin(a ^ b).count("1") for a, b in zip(s, t)) == 5   # the five terms of P(x)


def test_spec_bruteforce_tiny():
    image, masters, offsets, truth = pins.small_case(seed=5, n_disk=96, tail=0)
    got = spec.brute_force_matches(image, masters, offsets)
    assert set(truth) <= set(got)


def test_pack_files_drops_partial_sector():
    data, off = oracle.pack_files([b"\x01" * 1100, b"", b"\x02" * 512, b"\x03" * 511])
    assert off == [0, 2, 2, 3, 3]
    assert data.shape == (3, 512)
    assert (data[0] == 1).all() and (data[2] == 2).all()
