"""Counter-based random bits and stochastic rounding to BF16 (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of this package: it lets the tests
predict, cell by cell, the rounding decisions of BF16 storage with
stochastic rounding.  It shares no code with the HIP path, which implements
the same generator separately.

Generator: Philox-2x32 with 10 rounds, from its published definition
(J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): per round the first counter word is
multiplied by 0xD256D193, the new first word is the high half xor the key xor
the second word, the new second word the low half, and the key is bumped by
0x9E3779B9.

Use in the step: one call gives 64 bits, which serve four stored elements.
Element e of a field (its dense index (z*ny + y)*nx + x) takes, of the output
for counter (e // 4, step index) and key (seed + species), bits 0-15 of the
first word when e % 4 = 0, bits 16-31 when 1, and the same halves of the
second word when 2 and 3.

Stochastic rounding of a finite FP32 value x to BF16: add the 16 random bits
to the bit pattern of x and keep the high 16 bits, so the magnitude rounds
up with probability (low 16 bits of x) / 2^16 -- the expected stored value
is x.
"""
import numpy as np

_M = np.uint64(0xD256D193)
_W = np.uint64(0x9E3779B9)
_MASK = np.uint64(0xFFFFFFFF)


def philox2x32_10(c0, c1, key):
    """Philox-2x32-10 of counter (c0, c1) and key (arrays of uint32 values,
    broadcast); returns the two output words as uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    for _ in range(10):
        p = _M * c0
        c0, c1 = ((p >> np.uint64(32)) & _MASK) ^ k ^ c1, p & _MASK
        k = (k + _W) & _MASK
    return c0.astype(np.uint32), c1.astype(np.uint32)


def random16(index, step, seed, species):
    """The 16 random bits of stored element `index` (dense index
    (z*ny + y)*nx + x) of `species` at step `step` under `seed`."""
    e = np.asarray(index, dtype=np.uint64)
    w0, w1 = philox2x32_10(e >> np.uint64(2), np.uint64(step),
                           (np.uint64(seed) + np.uint64(species)) & _MASK)
    q = e & np.uint64(3)
    word = np.where(q >= np.uint64(2), w1, w0).astype(np.uint32)
    return np.where((q & np.uint64(1)) == np.uint64(1), word >> np.uint32(16),
                    word & np.uint32(0xFFFF)).astype(np.uint32)


def bf16_stochastic(x, r16):
    """Stochastic rounding of finite float32 values x to BF16 with random
    bits r16; returns the BF16 values as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    out = ((b + np.asarray(r16, dtype=np.uint64)) >> np.uint64(16)) << np.uint64(16)
    return out.astype(np.uint32).view(np.float32)
