"""The probe layouts (bucketed table, the paper's per-slot linear probing from
the low signature bits, sorted array with binary search) give exactly the
oracle's flags and matches, at low and high table loads."""
import random

import numpy as np
import pytest

import oracle
import pins
import synth
from gpu_util import assert_same_matches, dev_bytes, gpu_flags_and_matches, oracle_flags_and_matches
from oracle import spec
from paper_0901_1307_amd import carve

pytestmark = pytest.mark.gpu
SECTOR = 512
MOD = 1 << 64
LAYOUTS = [carve.CARVE_LAYOUT_BUCKETED, carve.CARVE_LAYOUT_LINEAR, carve.CARVE_LAYOUT_SORTED]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("bloom", [0, carve.CARVE_BLOOM_OFF])
def test_layouts_small_case(layout, bloom):
    image, masters, offsets, truth = pins.small_case()
    mflat = b"".join(masters)
    idx = carve.build_master_index(dev_bytes(mflat), offsets, bloom_bits_per_key=bloom, layout=layout)
    for tau0, any_tau in ((0, False), (6, False), (0, True)):
        f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), tau0, any_tau)
        wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets, np.frombuffer(image, np.uint8),
                                          tau0, any_tau)
        assert np.array_equal(f, wf), (tau0, any_tau)
        assert_same_matches(m, wm)


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.CONFIGS["tiny"]
    ms = synth.master_set(cfg, device="cuda")
    img = synth.disk_image(cfg, ms, device="cuda")
    host = (ms.sectors.cpu().numpy(), img.data.cpu().numpy())
    want = {}
    for any_tau in (False, True):
        want[any_tau] = oracle_flags_and_matches(host[0], ms.file_offsets, host[1], 0, any_tau)
    return ms, img, want


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("load", [0.1, 0.9])
@pytest.mark.parametrize("sig_kind", [carve.CARVE_SIG_DJB2_64, carve.CARVE_SIG_CRC64_ISO])
def test_layouts_tiny_config(tiny, layout, load, sig_kind):
    ms, img, want = tiny
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, max_load=load, layout=layout, sig_kind=sig_kind,
                                   bloom_bits_per_key=carve.CARVE_BLOOM_OFF)
    for any_tau in (False, True):
        f, m, _ = gpu_flags_and_matches(idx, img.data, 0, any_tau)
        if sig_kind == carve.CARVE_SIG_DJB2_64:
            wf, wm = want[any_tau]
            assert np.array_equal(f, wf)
        else:
            _, wm = want[any_tau]          # the confirmed set does not depend on the signature
        assert_same_matches(m, wm)


def _crafted(prefix: bytes, targets):
    """Sectors with chosen djb2 signatures: shared prefix, 13 base-33 digits at the end."""
    body = prefix + bytes(SECTOR - 13 - len(prefix))
    base = spec.djb2_closed(body + bytes(13))
    out = []
    for t in targets:
        need = (t - base) % MOD
        d = []
        for _ in range(13):
            d.append(need % 33)
            need //= 33
        out.append(body + bytes(d[12 - i] for i in range(13)))
    return out


@pytest.mark.parametrize("bloom", [0, carve.CARVE_BLOOM_OFF])
def test_linear_layout_long_chains(bloom):
    """Two thousand master signatures with the same 32 low bits share one
    home slot of the paper's table: present and absent sectors with those low
    bits walk the whole chain."""
    rng = random.Random(11)
    low = rng.getrandbits(32)
    n_same = 2000
    highs = rng.sample(range(1, 1 << 32), 2 * n_same)
    crafted = _crafted(b"linear-chain", [(h << 32) | low for h in highs])
    masters = crafted[:n_same] + [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(3000)]
    offsets = [0, 2500, len(masters)]
    mflat = b"".join(masters)
    idx = carve.build_master_index(dev_bytes(mflat), offsets, bloom_bits_per_key=bloom,
                                   layout=carve.CARVE_LAYOUT_LINEAR, max_load=0.5)
    disk = []
    for _ in range(3000):
        r = rng.random()
        if r < 0.3:
            disk.append(crafted[rng.randrange(n_same)])
        elif r < 0.6:
            disk.append(crafted[n_same + rng.randrange(n_same)])
        else:
            disk.append(bytes(rng.getrandbits(8) for _ in range(SECTOR)))
    image = b"".join(disk)
    for any_tau in (False, True):
        f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), any_tau=any_tau)
        wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets, np.frombuffer(image, np.uint8),
                                          any_tau=any_tau)
        assert len(wf) > (500 if any_tau else 50)   # per-cluster: about one crafted sector in 8 sits right
        assert np.array_equal(f, wf)
        assert_same_matches(m, wm)


def test_sorted_layout_extremes():
    """Signatures at both ends of the sorted order (1 and 2^64 - 1), the only
    key, and the signature 0 side slot."""
    rng = random.Random(12)
    ends = _crafted(b"sorted-ends", [1, MOD - 1, 0, 2])
    for masters in ([ends[0]], [ends[1]], ends[:3], ends):
        mflat = b"".join(masters)
        offsets = [0, len(masters)]
        idx = carve.build_master_index(dev_bytes(mflat), offsets, layout=carve.CARVE_LAYOUT_SORTED,
                                       bloom_bits_per_key=carve.CARVE_BLOOM_OFF)
        disk = [ends[rng.randrange(4)] for _ in range(200)] + [bytes(rng.getrandbits(8) for _ in range(SECTOR))]
        image = b"".join(disk)
        f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), any_tau=True)
        wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets, np.frombuffer(image, np.uint8),
                                          any_tau=True)
        assert np.array_equal(f, wf)
        assert_same_matches(m, wm)


def test_layout_batch_equals_alone(tiny):
    ms, img, want = tiny
    idx = carve.build_master_index(ms.sectors, ms.file_offsets, layout=carve.CARVE_LAYOUT_SORTED)
    data = img.data
    images = [(data[: 512 * 5000 + 3], 0, 0), (data[512 * 7000: 512 * 30000], 7, carve.CARVE_TAU_ANY)]
    b = carve.scan_batch(idx, images)
    counts = carve.batch_flag_counts(b)
    for i, (t, tau0, mode) in enumerate(images):
        f, _, _ = gpu_flags_and_matches(idx, t, tau0, mode == carve.CARVE_TAU_ANY)
        assert counts[i] == len(f)
        assert np.array_equal(carve.batch_flagged_sectors(b, i).numpy().astype(np.uint64), f)


def test_unknown_layout_rejected(tiny):
    ms, img, want = tiny
    with pytest.raises(carve.CarveError) as e:
        carve.build_master_index(ms.sectors, ms.file_offsets, layout=3)
    assert e.value.code == carve.CARVE_EINVAL


@pytest.mark.parametrize("layout", [carve.CARVE_LAYOUT_LINEAR, carve.CARVE_LAYOUT_SORTED])
def test_layouts_without_table_keys(layout):
    """No master sector at all, and masters whose only signature is 0 (kept
    beside the table): the layout's probe structure exists and finds nothing;
    with signature 0 among other signatures the layout holds exactly the others."""
    rng = random.Random(13)
    zero_sig = _crafted(b"zero-only", [0])[0]
    other = [bytes(rng.getrandbits(8) for _ in range(SECTOR)) for _ in range(5)]
    disk = [zero_sig, other[2], bytes(SECTOR), zero_sig] * 20
    image = b"".join(disk)
    for masters in ([], [zero_sig], [zero_sig] + other):
        mflat = b"".join(masters)
        offsets = [0, len(masters)]
        idx = carve.build_master_index(dev_bytes(mflat), offsets, layout=layout,
                                       bloom_bits_per_key=carve.CARVE_BLOOM_OFF)
        for any_tau in (False, True):
            f, m, _ = gpu_flags_and_matches(idx, dev_bytes(image), any_tau=any_tau)
            wf, wm = oracle_flags_and_matches(np.frombuffer(mflat, np.uint8), offsets,
                                              np.frombuffer(image, np.uint8), any_tau=any_tau)
            assert np.array_equal(f, wf), (len(masters), any_tau)
            assert_same_matches(m, wm)
