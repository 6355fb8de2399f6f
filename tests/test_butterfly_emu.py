"""CPU emulation of the tile kernel's in-place butterfly (the FFA tree of
paper Sec. 2.1 on 2^d rows held in LDS), lane by lane and chunk by chunk:
the radix-2 levels and the radix-4 passes, with their halo copies and the
in-place writes, checked against the oracle's fold.  A chunk's reads all
happen before its writes, as in one wave instruction stream; a mistake in
the slot order, the shifts or the halo sizes fails here without a GPU."""
import numpy as np
import pytest

WAVE = 64


def bitrev(t: int, d: int) -> int:
    r = 0
    for _ in range(d):
        r = (r << 1) | (t & 1)
        t >>= 1
    return r


def _radix2(lds, P0, H, l, R):
    half = 1 << (l - 1)
    for p in range(R // 2):
        beta, v = p >> (l - 1), p & (half - 1)
        a = beta * 2 * half + bitrev(v, l - 1)
        b = a + half
        sh = v if v < P0 else v % P0
        hn = min(sh + 1, H)
        lds[b, P0:P0 + hn] = lds[b, 0:hn]
        for c0 in range(0, P0, WAVE):
            j = np.arange(c0, min(c0 + WAVE, P0))
            A, x, y = lds[a, j].copy(), lds[b, j + sh].copy(), lds[b, j + sh + 1].copy()
            lds[a, j] = A + x
            lds[b, j] = A + y


def _radix4(lds, P0, l, R):
    half = 1 << (l - 1)
    for u in range(R // 4):
        blk, v = u >> (l - 1), u & (half - 1)
        r0 = blk * 4 * half + bitrev(v, l - 1)
        r1, r2, r3 = r0 + half, r0 + 2 * half, r0 + 3 * half
        lds[r1, P0:P0 + v + 1] = lds[r1, 0:v + 1]
        lds[r2, P0:P0 + 2 * v + 2] = lds[r2, 0:2 * v + 2]
        lds[r3, P0:P0 + 3 * v + 3] = lds[r3, 0:3 * v + 3]
        for c0 in range(0, P0, WAVE):
            j = np.arange(c0, min(c0 + WAVE, P0))
            x0 = lds[r0, j].copy()
            x1 = [lds[r1, j + v + k].copy() for k in range(2)]
            x2 = [lds[r2, j + 2 * v + k].copy() for k in range(3)]
            x3 = [lds[r3, j + 3 * v + k].copy() for k in range(4)]
            a0, a1 = x0 + x1[0], x0 + x1[1]
            lds[r0, j] = a0 + (x2[0] + x3[0])
            lds[r2, j] = a0 + (x2[1] + x3[1])
            lds[r1, j] = a1 + (x2[1] + x3[2])
            lds[r3, j] = a1 + (x2[2] + x3[3])


def butterfly(rows: np.ndarray, P0: int, d: int, room: int, radix4: bool = True) -> np.ndarray:
    """The kernel's butterfly on rows (2^d, P0): room = spare bins per row
    (stride - P0), halo H = min(2^(d-1), P0).  Returns the rows in output
    order (partial t at row bitrev(t, d) of the LDS block)."""
    R = 1 << d
    H = min(1 << (d - 1), P0)
    assert room >= H
    lds = np.zeros((R, P0 + room), rows.dtype)
    lds[:, :P0] = rows
    lim = min(room, P0)
    l = 1
    while l <= d:
        half = 1 << (l - 1)
        if radix4 and l < d and 3 * half <= lim:
            _radix4(lds, P0, l, R)
            l += 2
        else:
            _radix2(lds, P0, H, l, R)
            l += 1
    return np.stack([lds[bitrev(t, d), :P0] for t in range(R)])


# (P0, d, extra room beyond the radix-2 halo)
CASES = [(5, 3, 0), (20, 7, 0), (37, 5, 0), (64, 6, 16), (100, 4, 0), (129, 6, 0), (300, 6, 17),
         (300, 7, 32), (511, 6, 16), (70, 7, 0)]


@pytest.mark.parametrize("P0,d,extra", CASES)
def test_butterfly_matches_fold(oracle_mod, P0, d, extra):
    g = np.random.default_rng(P0 * 31 + d)
    M = 1 << d
    m = M - (M // 4 if d > 2 else 0)  # some zero rows, as in a tile's padding
    x = g.integers(0, 256, size=m * P0).astype(np.int64)
    rows = np.zeros((M, P0), np.int64)
    rows[:m] = x.reshape(m, P0)
    H = min(1 << (d - 1), P0)
    want = oracle_mod.fold(x, P0, m, M)
    got = butterfly(rows, P0, d, H + extra)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(butterfly(rows, P0, d, H + extra, radix4=False), want)


def test_radix4_same_float_sums():
    """For float rows the radix-4 pass adds in the same order as two radix-2
    levels, so the results are identical bit for bit."""
    g = np.random.default_rng(5)
    P0, d = 97, 6
    rows = g.standard_normal((1 << d, P0)).astype(np.float32)
    a = butterfly(rows, P0, d, 48)
    b = butterfly(rows, P0, d, 48, radix4=False)
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
