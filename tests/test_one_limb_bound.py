"""The one-limb N = 2048 key form (fs_evk_upload_form, FS_KEY_ONE_LIMB)
returns the exact external product only while every coefficient of the
integer product sum stays below (P-1)/2 of the transform prime.  Its case
rests on a distribution, not a worst case: for a key generated as the
library does, a step's key rows are uniform words independent of that
step's digits, so each coefficient V_j = sum over rows and i of
d_i k_{j-i} (negacyclic signs) is a sum of independent uniform terms with
variance sum(d^2) 2^62 / 3.  CPU only: the exact sums of real CMux steps of
the oracle's blind rotation, computed in int64, against that model."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

P_NTT = 3 * 2 ** 49 + 2 ** 20 + 1
HALF = (P_NTT - 1) // 2


def _centred(u):
    u = np.asarray(u, np.int64)
    return np.where(u >= 2 ** 31, u - 2 ** 32, u)


def _negacyclic_int(d, k):
    """Exact integer negacyclic product of two int64 polynomials."""
    N = len(d)
    full = np.convolve(d, k)  # |entries| <= N 512 2^31 = 2^51 at N = 2048
    out = full[:N].copy()
    out[:N - 1] -= full[N:]
    return out


@pytest.fixture(scope="module")
def steps():
    """Digits and exact product sums of the first CMux steps (i = 0..3) of one
    bootstrapping at N = 2048, l = 2, Bg = 2^10, with the oracle's key."""
    P = O.SHAPE_B
    K = O.keygen(P, synth.SEED_KEYS, with_ksk=False)
    m = synth.messages(synth.SEED_DATA, 1, P.p, stream=31)
    ct = O.encrypt(P, K.s, m, synth.SEED_ENC, 777)[0]
    v = O.test_poly(P.N, P.p, O.lut_fire(P.p, 4))
    out = []
    for i in range(4):
        # the accumulator after steps 0..i-1: a later a_i = 0 leaves it as is
        part = ct.copy()
        part[i:P.n] = 0
        acc = O.blind_rotate(K, v, part)
        abar = O.mod_switch(int(ct[i]), P.N)
        if abar == 0:
            continue
        dig = np.zeros((2, P.l, P.N), np.int64)
        for c in range(2):
            D = (O.mul_xpow(abar, acc[c]).astype(np.int64) - acc[c].astype(np.int64)) % 2 ** 32
            for j in range(P.N):
                dig[c, :, j] = O.gadget_digits(int(D[j]), P.l, P.bg_bit)
        V = np.zeros((2, P.N), np.int64)
        for o in range(2):
            for c in range(2):
                for lv in range(P.l):
                    key = _centred(K.bsk[i, c * P.l + lv, o])
                    V[o] += _negacyclic_int(dig[c, lv], key)
        out.append((dig, V))
    assert len(out) >= 3
    return out


def test_product_sums_follow_the_uniform_key_model(steps):
    """Once the accumulator is a full ciphertext (from the second step on;
    the first step's digits come from the structured test polynomial and
    its 4096 sums are strongly correlated), the spread of the 2 x 2048 sums
    of a step equals the model's standard deviation sqrt(sum d^2 2^62 / 3)
    within 5 %, with mean within 6 standard errors of zero."""
    for dig, V in steps[1:]:
        sigma = np.sqrt(float((dig.astype(np.float64) ** 2).sum()) * 2.0 ** 62 / 3)
        emp = V.astype(np.float64)
        assert abs(emp.std() / sigma - 1) < 0.05, emp.std() / sigma
        assert abs(emp.mean()) < 6 * sigma / np.sqrt(emp.size)


def test_exactness_limit_is_far_in_the_tail(steps):
    """Every observed sum lies below a quarter of (P-1)/2 and the limit is
    at least 20 of each step's standard deviations away (25 for the
    uniform digits of a typical step).  With every digit at its largest
    magnitude (512) it is 14.7 deviations away, where a sub-Gaussian sum
    (uniform terms are strictly sub-Gaussian) exceeds it with probability
    2 exp(-14.7^2 / 2) < 2^-150."""
    for dig, V in steps:
        assert np.abs(V).max() < HALF / 4
        sigma = np.sqrt(float((dig.astype(np.float64) ** 2).sum()) * 2.0 ** 62 / 3)
        assert HALF / sigma > 20
    worst = np.sqrt(4 * 2048 * 512.0 ** 2 * 2.0 ** 62 / 3)
    z = HALF / worst
    assert 14.6 < z < 14.8
    assert 1 - z * z / 2 / np.log(2) < -150
    # the worst case itself is past the limit: the two-limb form is what
    # makes the transform exact for every key
    assert 4 * 2048 * 512 * 2 ** 31 > HALF
