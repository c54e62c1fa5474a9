"""Worst-case magnitude bounds of the device transform's lazy reduction
schedule (host-side check of the arithmetic the kernels rely on).

Residues are integer-valued binary64 numbers; every sum and fma of them is
exact while magnitudes stay below 2^53.  With u = 2^-53, a modular product
of |a| <= A by a root |w| <= (P-1)/2 (h = fl(aw), l = fma(a,w,-h),
q = rint(fl(h/P)), r = fma(-q,P,h), t = r + l) satisfies
    |l| <= u|h|,  |r| <= P/2 + 2u|h|,  so |t| <= P/2 + 3u A (P-1)/2 (1+u),
and a reduction x - rint(x/P) P returns at most P/2 + 2u|x| + 1.
A Cooley-Tukey butterfly maps bound A to A + t(A); a butterfly whose root is
1 (skipped product) doubles it."""
from fractions import Fraction as Fr

import pytest

P = 3 * 2 ** 49 + 2 ** 20 + 1
LIMIT = 2 ** 53
U = Fr(1, 2 ** 53)


def prod_bound(A):
    h = A * Fr(P - 1, 2) * (1 + U)
    return Fr(P, 2) + 3 * U * h + 1


def redc_bound(A):
    return Fr(P, 2) + 2 * U * A + 1


def fwd_schedule(logn):
    """(stages between reductions) of the blind rotation's forward transform."""
    return [5, 4, logn - 9]


def table_start(dmax):
    """Bound after the first two stages taken from the digit tables (Bg = 2^7):
    d0 +- T1[d2] +- (TA[d1] + TB[d3]), each stored entry reduced."""
    entry = Fr(P, 2) + 1
    return dmax + 3 * entry


def inv_schedule(logn):
    """inverse: stages 0..2 (stage s has 2^-s of its roots equal to 1), then
    3..6, then 7..logn-1, each segment starting from a reduced value."""
    return [(0, 2), (3, 6), (7, logn - 1)]


@pytest.mark.parametrize("logn,rows,dmax,tables", [(10, 6, 64, True), (10, 6, 64, False),
                                                (11, 4, 512, False)])
def test_forward_pointwise_inverse_stay_exact(logn, rows, dmax, tables):
    # forward transform of a digit polynomial (the first two stages by table
    # at Bg = 2^7, arithmetic otherwise)
    A = table_start(dmax) if tables else Fr(dmax)
    segs = fwd_schedule(logn)
    for k, n in enumerate(segs):
        for _ in range(n - 2 if tables and k == 0 else n):
            A = A + prod_bound(A)
            assert A < LIMIT
        if k < len(segs) - 1:
            A = redc_bound(A)
    # pointwise products with reduced key values, summed over the digit rows
    acc = rows * prod_bound(A)
    assert acc < LIMIT
    # inverse transform, input reduced first
    for lo, hi in inv_schedule(logn):
        A = redc_bound(acc) if lo == 0 else redc_bound(A)
        for s in range(lo, hi + 1):
            trivial = s <= 3  # stages 0..3 have roots equal to 1 in some butterflies
            A = max(2 * A if trivial else A, A + prod_bound(A))
            assert A < LIMIT, (lo, s)
    twisted = prod_bound(A)
    final = redc_bound(twisted)
    # the exact product sum must be the centred residue: |E| + |error| < P/2
    E = rows * (1 << logn) * dmax * (2 ** 31 if logn == 10 else 2 ** 15)
    assert final - Fr(P, 2) < Fr(P, 2) - E
    # the low-word extraction adds 1.5 * 2^52 and needs |e| < 2^51
    assert final < 2 ** 51


def test_bounds_are_tight_enough_to_matter():
    """One more forward stage in the first segment would overflow 2^53."""
    A = Fr(64)
    for _ in range(6):
        A = A + prod_bound(A)
    assert A > LIMIT


def test_table_start_leaves_room_for_exactly_three_stages():
    """After the two table stages, three arithmetic stages fit below 2^53 and
    a fourth would not (so the first reduction stays after stage five)."""
    A = table_start(64)
    for _ in range(3):
        A = A + prod_bound(A)
    assert A < LIMIT
    assert A + prod_bound(A) > LIMIT
