"""Write pattern of the contraction epilogue's candidate threshold words (host model).

The direct-to-LDS contraction kernels write the bitmap as 32-bit half-words from each
256 x 256 upper-triangle tile (8 waves of 64 x 128, 32 x 32 blocks): a block (bi, bj)
writes row row0 + l's half-word at its column block and, off the diagonal block, the
mirrored row col0 + l's half-word at its row block; diagonal tiles skip the blocks
below the diagonal.  This replays that index arithmetic (with the kernel's guards) on
the host and checks that every half-word of every row is written exactly once and
nothing outside the p x 2*ceil(p/64) half-word array is touched."""
import pytest


def _writes(p):
    BT, nwords = 256, (p + 63) // 64
    nh = 2 * nwords
    T = (p + BT - 1) // BT
    seen = {}
    for I in range(T):
        for J in range(I, T):
            rowI0, rowJ0 = I * BT, J * BT
            for wm in range(4):
                for wn in range(2):
                    for i in range(2):
                        for j in range(4):
                            bi, bj = wm * 2 + i, wn * 4 + j
                            diag = I == J
                            if diag and bj < bi:
                                continue
                            dblk = diag and bi == bj
                            row0, col0 = rowI0 + bi * 32, rowJ0 + bj * 32
                            for l in range(32):
                                targets = []
                                if dblk:
                                    if row0 + l < p:
                                        targets.append((row0 + l, col0 >> 5))
                                else:
                                    if row0 + l < p and (col0 >> 5) < nh:
                                        targets.append((row0 + l, col0 >> 5))
                                    if col0 + l < p and (row0 >> 5) < nh:
                                        targets.append((col0 + l, row0 >> 5))
                                for t in targets:
                                    seen[t] = seen.get(t, 0) + 1
    return seen, nh


@pytest.mark.parametrize("p", [1, 31, 64, 200, 256, 333, 511, 600, 700, 1025])
def test_every_half_word_written_once_in_bounds(p):
    seen, nh = _writes(p)
    assert all(0 <= r < p and 0 <= h < nh for (r, h) in seen)
    assert all(c == 1 for c in seen.values()), [k for k, c in seen.items() if c != 1][:5]
    assert len(seen) == p * nh
