"""Plausible mistakes planted in a copy of the oracle (on the CPU) must each be
caught by at least one pin: the pins are strong enough to trust the oracle."""
import os
import subprocess
import tempfile

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "carve_oracle.c")

MUTANTS = {
    "init-5380": ("uint64_t h = 5381u;", "uint64_t h = 5380u;"),
    "mult-31": ("h = h * 33u + (uint64_t)s[i];", "h = h * 31u + (uint64_t)s[i];"),
    "xor-variant": ("h = h * 33u + (uint64_t)s[i];", "h = (h * 33u) ^ (uint64_t)s[i];"),
    "signed-bytes": ("h = h * 33u + (uint64_t)s[i];", "h = h * 33u + (uint64_t)(int8_t)s[i];"),
    "reversed-order": ("h = h * 33u + (uint64_t)s[i];", "h = h * 33u + (uint64_t)s[len - 1 - i];"),
    "32-bit-accumulator": ("h = h * 33u + (uint64_t)s[i];", "h = (uint32_t)(h * 33u + (uint64_t)s[i]);"),
    "drop-tau0": ("(uint32_t)((j + tau0) % CLUSTER_SECTORS)", "(uint32_t)(j % CLUSTER_SECTORS)"),
    "tau-from-global-index": ("return any_tau || (e->k % CLUSTER_SECTORS)",
                              "return any_tau || (e->master % CLUSTER_SECTORS)"),
    "ignore-any-tau": ("return any_tau || (e->k", "return (e->k"),
    "first-entry-only": ("    if (tau_ok(&ix->e[p], j, tau0, any_tau)) return 1;\n  return 0;",
                         "    return tau_ok(&ix->e[p], j, tau0, any_tau);\n  return 0;"),
    "lower-bound-off": ("if (ix->e[mid].sig < sig) lo = mid + 1;", "if (ix->e[mid].sig <= sig) lo = mid + 1;"),
    "confirm-skips-memcmp": ("if (memcmp(s, ix->masters + e->master * SECTOR_BYTES, SECTOR_BYTES) != 0) continue;",
                             ""),
    "confirm-skips-tau": ("      if (!tau_ok(e, ids[i], tau0, any_tau)) continue;\n      if (memcmp(s,",
                          "      if (memcmp(s,"),
    "short-compare": ("if (memcmp(s, ix->masters + e->master * SECTOR_BYTES, SECTOR_BYTES) != 0) continue;",
                      "if (memcmp(s, ix->masters + e->master * SECTOR_BYTES, 8) != 0) continue;"),
    "last-sector-dropped": ("for (uint64_t j = 0; j < n; j++)\n    if (flag[j])",
                            "for (uint64_t j = 0; j + 1 < n; j++)\n    if (flag[j])"),
    "crc-poly-1a": ("#define CRC64_GO_ISO_POLY 0x000000000000001Bull", "#define CRC64_GO_ISO_POLY 0x000000000000001Aull"),
    "crc-poly-unreflected": ("const uint64_t poly_reflected = reverse64(CRC64_GO_ISO_POLY);",
                             "const uint64_t poly_reflected = CRC64_GO_ISO_POLY;"),
    "crc-zero-preset": ("uint64_t crc = ~0ull;", "uint64_t crc = 0;"),
    "crc-no-final-complement": ("return ~crc;", "return crc;"),
    "crc-byte-at-top": ("crc ^= (uint64_t)s[i];", "crc ^= (uint64_t)s[i] << 56;"),
    "window-stride-8": ("#define WINDOW_STRIDE 4u", "#define WINDOW_STRIDE 8u"),
    "window-63-bytes": ("c->image + j * WINDOW_STRIDE, FRAGMENT_BYTES);", "c->image + j * WINDOW_STRIDE, FRAGMENT_BYTES - 1);"),
    "last-window-dropped": ("(n_bytes - FRAGMENT_BYTES) / WINDOW_STRIDE + 1;", "(n_bytes - FRAGMENT_BYTES) / WINDOW_STRIDE;"),
    "fragment-confirm-skips-memcmp": ("      if (memcmp(w, ix->masters + e->master * FRAGMENT_BYTES, FRAGMENT_BYTES) != 0) continue;\n", ""),
    "crc-kind-ignored": ("return kind == ORACLE_SIG_CRC64_GO_ISO ? oracle_crc64(s, SECTOR_BYTES) : oracle_djb2(s, SECTOR_BYTES);",
                         "return oracle_djb2(s, SECTOR_BYTES);"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation site for {name} not found"
    path = os.path.join(tmpdir, f"{name}.c")
    with open(path, "w") as f:
        f.write(text.replace(old, new, 1))
    out = os.path.join(tmpdir, f"lib{name}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", path, "-o", out],
                   check=True, capture_output=True)
    return oracle.load(out)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(name, d)
        caught = []
        for pin in pins.ALL_PINS:
            try:
                pin(lib)
            except AssertionError:
                caught.append(pin.__name__)
        assert caught, f"no pin catches mutant {name}"
