"""Host checks of the swap kernel's index arithmetic (csrc/shg_swap.hip): the
quotient floor(r / d) is taken as (int)((r + 0.5f) * (1.0f / d)) in float32;
this must be exact for every remainder and divisor the kernel forms
(value blocks: r < 81, d = 2la+1 <= 9; derivative blocks: r < 3*81, d = block
size <= 81), and the transposed walk must visit every element once."""
import numpy as np


def small_div(r, d):
    rd = np.float32(1.0) / np.float32(d)
    return ((np.asarray(r, np.float32) + np.float32(0.5)) * rd).astype(np.int32)


def test_small_div_exact_over_kernel_ranges():
    for d in range(1, 82):
        r = np.arange(0, 3 * 81, dtype=np.int64)
        assert np.array_equal(small_div(r, d), (r // d).astype(np.int32)), d


def test_transposed_walk_is_a_permutation():
    for la in range(5):
        for lb in range(5):
            na, nb = 2 * la + 1, 2 * lb + 1
            sz = na * nb
            src = []
            for r in range(sz):                       # destination element r of the (b, a) block
                mb = int(small_div(r, na))
                ma = r - mb * na
                src.append(ma * nb + mb)              # source element of the (a, b) block
            assert sorted(src) == list(range(sz))
            # transposition: destination (mb, ma) holds source (ma, mb)
            M = np.arange(sz).reshape(na, nb)
            assert np.array_equal(np.array(src).reshape(nb, na), M.T)
