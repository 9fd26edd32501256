"""Pure-Python forms of the sector signature -- TEST INFRASTRUCTURE ONLY.

Eq. (1) (Section 2.2) defines djb2 as hash_0 = 5381 and
hash_i = hash_{i-1} * 33 + s_i; Section 4 states that the accumulator is 64
bits wide, so every step is taken modulo 2^64 and the bytes s_i are the
sector's bytes in address order, as unsigned values.

Unrolling the recurrence gives a closed form with no loop-carried state:

    hash_n = 5381 * 33^n + sum_{i=1..n} s_i * 33^(n-i)      (mod 2^64)

which these tests use as a second, differently computed definition. Python
integers are unbounded, so the only reduction is the final one.
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
                          tau0: int = 0, any_tau: bool = False) -> List[int]:
    """Sectors whose closed-form signature equals that of some master sector at a
    compatible cluster position (per-position tables S_tau of Section 3.1)."""
    by_tau = {t: set() for t in range(8)}
    for f in range(len(file_offsets) - 1):
        for k in range(file_offsets[f + 1] - file_offsets[f]):
            by_tau[k % 8].add(djb2_closed(masters[file_offsets[f] + k]))
    every = set().union(*by_tau.values())
    out = []
    for j in range(len(image) // SECTOR):
        h = djb2_closed(image[j * SECTOR:(j + 1) * SECTOR])
        if (h in every) if any_tau else (h in by_tau[(j + tau0) % 8]):
            out.append(j)
    return out


def sectors_of(data: bytes) -> Iterable[bytes]:
    for j in range(len(data) // SECTOR):
        yield data[j * SECTOR:(j + 1) * SECTOR]
