"""Pure-Python forms of the sector signature -- TEST INFRASTRUCTURE ONLY.

Eq. (1) (Section 2.2) defines djb2 as hash_0 = 5381 and
hash_i = hash_{i-1} * 33 + s_i; Section 4 states that the accumulator is 64
bits wide, so every step is taken modulo 2^64 and the bytes s_i are the
sector's bytes in address order, as unsigned values.

Unrolling the recurrence gives a closed form with no loop-carried state:

    hash_n = 5381 * 33^n + sum_{i=1..n} s_i * 33^(n-i)      (mod 2^64)

which these tests use as a second, differently computed definition. Python
integers are unbounded, so the only reduction is the final one.

The other signature the paper times is a 64-bit CRC (Section 2.1, Figs. 10-11)
whose parameters it does not state. The reading taken here is CRC-64/GO-ISO
(generator x^64 + x^4 + x^3 + x + 1, reflected, preset and final complement
all ones). Two forms below: a shift register fed bit by bit, and the
definition as polynomial division over GF(2) with Python integers as
polynomials. Both are generic in width and parameters, so the same code can be
checked against zlib's CRC-32.
"""
from __future__ import annotations

from typing import Iterable, List, Sequence

MOD = 1 << 64
INIT = 5381
MULT = 33
SECTOR = 512


def djb2_horner(data: bytes) -> int:
    """Eq. (1) step by step, reduced modulo 2^64 after each step."""
    h = INIT
    for s in bytes(data):
        h = (h * MULT + s) % MOD
    return h


def djb2_closed(data: bytes) -> int:
    """The unrolled closed form of Eq. (1), reduced once at the end."""
    b = bytes(data)
    n = len(b)
    total = INIT * MULT ** n
    for i, s in enumerate(b, start=1):
        total += s * MULT ** (n - i)
    return total % MOD


def craft_sector(prefix: bytes, target: int, n: int = SECTOR) -> bytes:
    """A byte string of length n that starts with `prefix` and whose signature is `target`.

    With 13 free trailing bytes, the last 13 terms of the closed form cover
    every residue: choose digits d_i in [0, 32] of target - rest in base 33
    (33^13 > 2^64), each added to a base byte of 0.
    """
    free = 13
    assert len(prefix) <= n - free
    body = bytes(prefix) + bytes(n - free - len(prefix))
    base = djb2_closed(body + bytes(free))          # all free bytes zero
    need = (target - base) % MOD
    digits: List[int] = []
    for _ in range(free):
        digits.append(need % MULT)
        need //= MULT
    assert need == 0
    # the free byte at distance e from the end weighs 33^e
    tail = bytes(digits[free - 1 - i] for i in range(free))
    return body + tail


def collide(data: bytes, i: int) -> bytes:
    """Bytes (a, b) at positions (i, i+1) replaced by (a+1, b-33): same signature.

    a*33 + b == (a+1)*33 + (b-33), so every later step of Eq. (1) is unchanged.
    Requires a <= 254 and b >= 33."""
    b = bytearray(data)
    assert b[i] <= 254 and b[i + 1] >= 33
    b[i] += 1
    b[i + 1] -= 33
    return bytes(b)


def brute_force_matches(image: bytes, masters: Sequence[bytes], file_offsets: Sequence[int],
                        tau0: int = 0, any_tau: bool = False) -> List[tuple]:
    """Every (disk sector, file, sector in file) with equal bytes and a compatible
    cluster position, by direct comparison -- for tiny inputs only."""
    n = len(image) // SECTOR
    out = []
    for j in range(n):
        d = image[j * SECTOR:(j + 1) * SECTOR]
        for f in range(len(file_offsets) - 1):
            for k in range(file_offsets[f + 1] - file_offsets[f]):
                if not any_tau and k % 8 != (j + tau0) % 8:
                    continue
                if masters[file_offsets[f] + k] == d:
                    out.append((j, f, k))
    return out


def flagged_by_definition(image: bytes, masters: Sequence[bytes], file_offsets: Sequence[int],
                          tau0: int = 0, any_tau: bool = False, sig=None) -> List[int]:
    """Sectors whose signature (closed-form djb2 unless `sig` is given) equals
    that of some master sector at a compatible cluster position (per-position
    tables S_tau of Section 3.1)."""
    sig = sig or djb2_closed
    by_tau = {t: set() for t in range(8)}
    for f in range(len(file_offsets) - 1):
        for k in range(file_offsets[f + 1] - file_offsets[f]):
            by_tau[k % 8].add(sig(masters[file_offsets[f] + k]))
    every = set().union(*by_tau.values())
    out = []
    for j in range(len(image) // SECTOR):
        h = sig(image[j * SECTOR:(j + 1) * SECTOR])
        if (h in every) if any_tau else (h in by_tau[(j + tau0) % 8]):
            out.append(j)
    return out


def sectors_of(data: bytes) -> Iterable[bytes]:
    for j in range(len(data) // SECTOR):
        yield data[j * SECTOR:(j + 1) * SECTOR]


# ------------------------------------------------------------------- CRCs
# (width, generator without its top term in normal form, preset, final xor);
# all reflected in and out
CRC64_GO_ISO = (64, 0x1B, (1 << 64) - 1, (1 << 64) - 1)
CRC64_XZ = (64, 0x42F0E1EBA9EA3693, (1 << 64) - 1, (1 << 64) - 1)
CRC32_ZLIB = (32, 0x04C11DB7, (1 << 32) - 1, (1 << 32) - 1)


def _reflect(x: int, width: int) -> int:
    return int(format(x, f"0{width}b")[::-1], 2)


def crc_register(data: bytes, params=CRC64_GO_ISO) -> int:
    """Shift register, one input bit at a time, least significant bit of each
    byte first; the generator is applied in bit-reversed form."""
    width, poly, init, xorout = params
    rpoly = _reflect(poly, width)
    crc = init
    for byte in bytes(data):
        crc ^= byte
        for _ in range(8):
            crc = (crc >> 1) ^ rpoly if crc & 1 else crc >> 1
    return crc ^ xorout


def _gf2_mod(a: int, p: int) -> int:
    dp = p.bit_length() - 1
    while a and a.bit_length() - 1 >= dp:
        a ^= p << (a.bit_length() - 1 - dp)
    return a


def crc_polydiv(data: bytes, params=CRC64_GO_ISO) -> int:
    """The definition: with the message bits in transmission order (byte 0's
    least significant bit first) as the coefficients of M(x), highest degree
    first, over L bits, the remainder R(x) = (M(x) x^W + I(x) x^L) mod P(x),
    where I(x) is the preset register; the result is R reflected, xor the
    final value."""
    width, poly, init, xorout = params
    b = bytes(data)
    m = 0
    for byte in b:
        for k in range(8):
            m = (m << 1) | ((byte >> k) & 1)
    n_bits = 8 * len(b)
    p = (1 << width) | poly
    r = _gf2_mod((m << width) ^ (_reflect(init, width) << n_bits), p)
    return _reflect(r, width) ^ xorout


def crc_bytewise(data: bytes, params=CRC64_GO_ISO) -> int:
    """A third form, one byte per step through a 256-entry table whose entries
    are the shift register run over one byte; fast enough for sets of sectors."""
    width, poly, init, xorout = params
    table = _byte_table(params)
    crc = init
    for byte in bytes(data):
        crc = table[(crc ^ byte) & 0xFF] ^ (crc >> 8)
    return crc ^ xorout


_TABLES = {}


def _byte_table(params):
    if params not in _TABLES:
        width, poly, _, _ = params
        rpoly = _reflect(poly, width)
        t = []
        for v in range(256):
            c = v
            for _ in range(8):
                c = (c >> 1) ^ rpoly if c & 1 else c >> 1
            t.append(c)
        _TABLES[params] = t
    return _TABLES[params]


def crc_collide(data: bytes, k: int = 0, params=CRC64_GO_ISO) -> bytes:
    """`data` with the bits of x^k P(x) flipped, in the message-polynomial view
    of crc_polydiv: a different string of the same length with the same CRC
    (the CRC of a message is affine in its bits, and P(x) divides x^k P(x))."""
    width, poly, _, _ = params
    n_bits = 8 * len(data)
    p = (1 << width) | poly
    assert k + width < n_bits
    b = bytearray(data)
    for deg in range(width + 1):
        if (p >> deg) & 1:
            t = n_bits - 1 - (deg + k)          # bit t of the stream: byte t // 8, bit t % 8 (LSB first)
            b[t // 8] ^= 1 << (t % 8)
    return bytes(b)


# ------------------------------------------------------ fragments (Section 5)
FRAGMENT = 64
STRIDE = 4


def fragment_windows(image: bytes):
    """(j, bytes) of every 64-byte window starting on a 4-byte boundary."""
    for j in range(0, (len(image) - FRAGMENT) // STRIDE + 1 if len(image) >= FRAGMENT else 0):
        yield j, image[STRIDE * j: STRIDE * j + FRAGMENT]


def fragment_flags_by_definition(image: bytes, fragments: Sequence[bytes]) -> List[int]:
    sigs = {djb2_closed(f) for f in fragments}
    return [j for j, w in fragment_windows(image) if djb2_closed(w) in sigs]


def fragment_matches_by_comparison(image: bytes, fragments: Sequence[bytes], file_offsets: Sequence[int]):
    """All (window, file, fragment in file) with equal bytes, in window then master order."""
    owner = []
    for f in range(len(file_offsets) - 1):
        for k in range(file_offsets[f + 1] - file_offsets[f]):
            owner.append((f, k))
    by_bytes = {}
    for m, frag in enumerate(fragments):
        by_bytes.setdefault(bytes(frag), []).append(owner[m])
    return [(j, f, k) for j, w in fragment_windows(image) for f, k in by_bytes.get(w, [])]
