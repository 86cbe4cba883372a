"""Word-level identities the encoder kernels rely on, checked exhaustively
over byte values (CPU only):

- a 32-bit word x has a zero byte exactly when (x - 0x01010101) & ~x &
  0x80808080 is non-zero (the escape-free test of the encoder fast paths);
- with x = w ^ 0x80808080, ((x & 0x7F7F7F7F) + 0x7F7F7F7F) | x has the top
  bit of byte i set exactly when byte i of w is not 0x80 (the per-byte test
  of the sparse encoder rounds: no carry crosses a byte)."""
import itertools

import numpy as np

FILL = (0x00, 0x01, 0x7F, 0x80, 0x81, 0xFE, 0xFF)


def _words():
    # every byte value in every position, the others from FILL, plus random
    for pos, b, other in itertools.product(range(4), range(256), FILL):
        bs = [other] * 4
        bs[pos] = b
        yield bs
    rng = np.random.default_rng(3)
    for _ in range(20000):
        yield [int(rng.choice(FILL)) if rng.random() < 0.5 else int(rng.integers(256))
               for _ in range(4)]


def _word(bs):
    return sum(b << (8 * i) for i, b in enumerate(bs))


def test_zero_byte_test():
    for bs in _words():
        x = _word(bs)
        got = ((x - 0x01010101) & ~x & 0x80808080) & 0xFFFFFFFF
        assert (got != 0) == (0 in bs), bs


def test_per_byte_not_0x80_test():
    for bs in _words():
        x = _word(bs) ^ 0x80808080
        hi = (((x & 0x7F7F7F7F) + 0x7F7F7F7F) | x) & 0x80808080
        assert [(hi >> (8 * i + 7)) & 1 for i in range(4)] == [int(b != 0x80) for b in bs], bs
