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


def test_spec_bruteforce_tiny():
    image, masters, offsets, truth = pins.small_case(seed=5, n_disk=96, tail=0)
    got = spec.brute_force_matches(image, masters, offsets)
    assert set(truth) <= set(got)


def test_pack_files_drops_partial_sector():
    data, off = oracle.pack_files([b"\x01" * 1100, b"", b"\x02" * 512, b"\x03" * 511])
    assert off == [0, 2, 2, 3, 3]
    assert data.shape == (3, 512)
    assert (data[0] == 1).all() and (data[2] == 2).all()
