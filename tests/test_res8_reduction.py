"""The matrix-core epilogue's residue reduction, emulated on the CPU.

The int8 kernels reduce an exact int32 sum x modulo m <= 255 to a centred
residue in three vector instructions (after a fold of x at 2^16 when x sums
more than 8 stages of 64 products): u = fma(float(y), fl(1/m), 1.5 2^23), then a signed 24-bit multiply-add of u's
low 24 bits with -m, plus y. The stored byte is the low byte of that word.
This checks, for every m in 2..255, that the byte is the two's complement of
a residue r of y with |r| <= 127, on every y where the quotient's rounding can
go wrong (next to each half-integer multiple of m) and at both ends of every
range of y the epilogue sees.
"""
import numpy as np
import pytest

C = 12582912.0  # 1.5 * 2^23


def reduce_byte(y, m):
    """The kernel's arithmetic on int64 array y: returns (byte, r)."""
    f = y.astype(np.float32)
    assert np.all(f.astype(np.int64) == y)  # |y| < 2^24: exact in float
    inv = np.float32(1.0) / np.float32(m)
    p = f.astype(np.float64) * np.float64(inv)  # exact: 24 x 24 bits
    # the fma rounds p + C once; |p| < 2^22 puts that sum where the float32
    # spacing is 1, so it is C + rint(p) (ties to even, C is even) and its
    # low 24 bits are 2^22 + rint(p)
    assert np.all(np.abs(p) < 2.0**22)
    q = np.rint(p).astype(np.int64)
    s24 = (1 << 22) + q
    assert np.all((s24 >= 0) & (s24 < 1 << 23))  # a positive signed 24-bit value
    word = (s24 * -m + y) & 0xFFFFFFFF
    return word & 0xFF, y - q * m


def ranges(m):
    """The ranges of y: no fold (sums of at most 8 stages of 64, K <= 512)
    and after the fold at 2^16."""
    r16 = 65536 % m
    return [(-512 * 127 * 127, 512 * 127 * 127), (-(2**15) * r16, (2**15 - 1) * r16 + 65535)]


@pytest.mark.parametrize("m", range(2, 256))
def test_reduction_byte_is_centred_residue(m):
    for lo, hi in ranges(m):
        k = np.arange(lo // m - 1, hi // m + 2, dtype=np.int64)
        near_half = (k[:, None] * m + np.array([m // 2 - 1, m // 2, (m + 1) // 2, (m + 1) // 2 + 1])).reshape(-1)
        ends = np.concatenate([np.arange(lo, min(hi, lo + 4096) + 1), np.arange(max(lo, hi - 4096), hi + 1)])
        y = np.concatenate([near_half, ends])
        y = y[(y >= lo) & (y <= hi)]
        byte, r = reduce_byte(y, m)
        assert np.all(np.abs(r) <= 127), (m, int(np.abs(r).max()))
        assert np.all((r - y) % m == 0)
        assert np.all(byte == (r & 0xFF))


def test_reduction_catches_wrong_rounding():
    # with the quotient truncated instead of rounded, residues reach m - 1
    y = np.arange(0, 100000, dtype=np.int64)
    m = 251
    q = (y.astype(np.float64) / m).astype(np.int64)
    assert np.abs(y - q * m).max() > 127
    _, r = reduce_byte(y, m)
    assert np.abs(r).max() <= 127
