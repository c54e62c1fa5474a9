"""Pins of the CPU oracle to facts outside itself: published test vectors,
library routines on special cases, closed forms, the paper's theorems and
brute force on tiny inputs.  CPU only."""
import ctypes
import math
import os
from dataclasses import replace
from fractions import Fraction

import numpy as np
import pytest
from scipy import signal

import synth
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32 = 1 << 32


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


def _signed(x):
    x = np.asarray(x, np.int64) % U32
    return np.where(x >= U32 // 2, x - U32, x)


# ------------------------------------------------------------------ P1: ChaCha20 (RFC 8439)

def test_chacha20_rfc8439_vectors():
    L = O.lib()
    rows = {r.split()[0]: r for r in _golden("chacha20_rfc8439.txt")}
    q = rows["quarter"].split()
    vals = [ctypes.c_uint32(int(v, 16)) for v in q[1:5]]
    L.or_chacha_quarter(*[ctypes.byref(v) for v in vals])
    assert [v.value for v in vals] == [int(v, 16) for v in q[6:10]]
    key = np.array([int(v, 16) for v in rows["block_key"].split()[1:]], np.uint32)
    nonce = np.array([int(v, 16) for v in rows["block_nonce"].split()[1:]], np.uint32)
    ctr = int(rows["block_counter"].split()[1])
    out = np.zeros(16, np.uint32)
    L.or_chacha20_block(O._u32(key), ctr, O._u32(nonce), O._u32(out))
    assert [int(v) for v in out] == [int(v, 16) for v in rows["block_out"].split()[1:]]
    z = np.zeros(8, np.uint32)
    zn = np.zeros(3, np.uint32)
    L.or_chacha20_block(O._u32(z), 0, O._u32(zn), O._u32(out))
    assert out.view(np.uint8)[:16].tobytes().hex() == rows["zero_key_first16"].split()[1]


# ------------------------------------------------------------------ P2: Gaussian sampler

def test_gaussian_moments():
    L = O.lib()
    g = synth.rng(11)
    w = g.integers(0, U32, size=(2, 200000), dtype=np.uint64)
    sigma = 2.0 ** -15
    e = np.array([L.or_gauss_from_words(int(a), int(b), sigma) for a, b in zip(*w)], np.uint32)
    x = _signed(e).astype(np.float64) / U32  # on the unit torus
    n = x.size
    assert abs(x.mean()) < 5 * sigma / math.sqrt(n)
    var_ratio = x.var() / sigma ** 2
    assert abs(var_ratio - 1) < 5 * math.sqrt(2 / n)
    # fourth moment of a normal: 3 sigma^4
    k4 = (x ** 4).mean() / sigma ** 4
    assert abs(k4 - 3) < 0.1
    assert L.or_gauss_from_words(123, 456, 0.0) == 0


def test_decryption_failure_rate_under_inflated_noise(okeys_a):
    """Forced noise overflow: with sigma_lwe = 2^-7 against the half window
    1/64 = 2 sigma of p = 32, a decryption fails exactly when the Gaussian
    error leaves (-1/64, 1/64]: probability erfc(2 / sqrt 2) = 4.55 %; the
    measured rate over 20,000 encryptions sits inside 4 binomial standard
    errors, and every failure is off by one message in the error's
    direction."""
    P = replace(O.SHAPE_A, sigma_lwe=2.0 ** -7)
    n = 20000
    m = synth.messages(synth.SEED_DATA, n, P.p, stream=77)
    ct = O.encrypt(P, okeys_a.s, m, 31)
    got = O.decrypt(P.p, okeys_a.s, ct)
    err = _signed(O.phase(okeys_a.s, ct).astype(np.int64) - (m.astype(np.int64) % P.p) * P.delta)
    want = math.erfc(2 / math.sqrt(2))
    bad = got != m
    rate = bad.mean()
    assert abs(rate - want) < 4 * math.sqrt(want * (1 - want) / n), (rate, want)
    step = np.sign(err[bad]).astype(np.int64)
    assert np.array_equal(O.centred(P.p, got[bad].astype(np.int64) - m[bad] - step), np.zeros(bad.sum()))


# ------------------------------------------------------------------ P3: negacyclic products

def test_negacyclic_hand_example():
    # (1 + 2X + 3X^2 + 4X^3) * X = -4 + X + 2X^2 + 3X^3 in Z[X]/(X^4+1)
    a = np.array([1, 2, 3, 4], np.uint32)
    x = np.array([0, 1, 0, 0], np.uint32)
    assert list(_signed(O.negacyclic_mul(a, x))) == [-4, 1, 2, 3]
    # X^3 * X^3 = X^6 = -X^2
    x3 = np.array([0, 0, 0, 1], np.uint32)
    assert list(_signed(O.negacyclic_mul(x3, x3))) == [0, 0, -1, 0]


@pytest.mark.parametrize("N", [8, 16, 64])
def test_negacyclic_matches_polymul_fold(N):
    g = synth.rng(12, N)
    a = g.integers(0, U32, size=N, dtype=np.uint64).astype(np.uint32)
    b = g.integers(0, U32, size=N, dtype=np.uint64).astype(np.uint32)
    full = np.polymul(a.astype(object)[::-1], b.astype(object)[::-1])[::-1]  # ascending powers
    full = list(full) + [0] * (2 * N - len(full))
    want = [(int(full[k]) - int(full[k + N])) % U32 for k in range(N)]
    assert list(O.negacyclic_mul(a, b).astype(np.int64)) == want


def test_mul_xpow_is_monomial_product():
    N = 16
    g = synth.rng(13)
    a = g.integers(0, U32, size=N, dtype=np.uint64).astype(np.uint32)
    for e in [0, 1, 5, N - 1, N, N + 3, 2 * N - 1]:
        mono = np.zeros(N, np.uint32)
        mono[e % N] = 1 if e < N else U32 - 1   # X^e = -X^{e-N} for e >= N
        assert np.array_equal(O.mul_xpow(e, a), O.negacyclic_mul(mono, a)), e
    # X^a X^b = X^{a+b}
    assert np.array_equal(O.mul_xpow(7, O.mul_xpow(30, a)), O.mul_xpow(37 % (2 * N), a))


# ------------------------------------------------------------------ P5: gadget decomposition

@pytest.mark.parametrize("l,bg", [(3, 7), (2, 10)])
def test_gadget_digits_reconstruct(l, bg):
    g = synth.rng(14, bg)
    xs = list(g.integers(0, U32, size=3000, dtype=np.uint64)) + [0, 1, U32 - 1, U32 // 2,
                                                                 U32 // 2 - 1, U32 // 2 + 1]
    bound = 1 << (31 - l * bg)
    for x in xs:
        d = O.gadget_digits(int(x), l, bg)
        assert all(-(1 << (bg - 1)) <= v < (1 << (bg - 1)) for v in d)
        rec = sum(int(d[j]) << (32 - (j + 1) * bg) for j in range(l))
        err = (rec - int(x)) % U32
        err = err - U32 if err >= U32 // 2 else err
        assert -bound < err <= bound


# ------------------------------------------------------------------ P6: rounding to Z_2N

@pytest.mark.parametrize("N", [1024, 2048])
def test_mod_switch_is_round_half_up(N):
    g = synth.rng(15, N)
    step = U32 // (2 * N)
    xs = [int(v) for v in g.integers(0, U32, size=2000, dtype=np.uint64)]
    for k in [0, 1, 2, N, 2 * N - 1]:
        for dx in (-1, 0, 1):
            xs.append((k * step + step // 2 + dx) % U32)
    for x in xs:
        want = math.floor(Fraction(x * 2 * N, U32) + Fraction(1, 2)) % (2 * N)
        assert O.mod_switch(x, N) == want


# ------------------------------------------------------------------ P7: program functions

def test_lif_luts_match_hand_tables():
    for row in _golden("lif_luts.txt"):
        head, vals = row.split(":")
        name, p, V, tau = head.split()
        want = [int(v) for v in vals.split()]
        assert len(want) == int(p)
        got = O.lut_fire(int(p), int(V)) if name == "fire" else O.lut_reset(int(p), int(V), int(tau))
        assert list(got) == want, row


@pytest.mark.parametrize("p", [32, 64])
def test_luts_are_negacyclic_and_follow_the_intervals(p):
    for V in range(1, p // 2 + 1):
        f = O.lut_fire(p, V)
        for tau in (0, 2, 3, 5):
            r = O.lut_reset(p, V, tau)
            for t in range(p):
                assert (f[(t + p // 2) % p] + f[t]) % p == 0
                assert (r[(t + p // 2) % p] + r[t]) % p == 0
        # Eq. FHE-Fire on m = H - V: +1 for m in [0, p/2), -1 for [-p/2, 0)
        for h in range(-p // 2, p // 2):
            m = ((h - V + p // 2) % p) - p // 2
            assert f[h % p] == (1 if 0 <= m < p // 2 else -1)
    # the fourth branch as printed (p/2 - leak) breaks negacyclicity:
    bad = O.lut_reset(p, 4, 2).copy()
    bad[p // 2 + 1] = p // 2 - O.leak(1, 2)
    with pytest.raises(ValueError):
        O.test_poly(1024, p, bad)


def test_test_poly_windows():
    """Coefficient i carries message round(i p / 2N) (ties up), times Delta."""
    N, p = 1024, 32
    f = O.lut_fire(p, 4)
    v = O.test_poly(N, p, f)
    delta = U32 // p
    for i in range(N):
        m = math.floor(Fraction(i * p, 2 * N) + Fraction(1, 2)) % p
        assert int(v[i]) == (int(f[m]) % p) * delta


def test_test_poly_message_space_change_hand_example():
    """N = 8, p_in = 4, p_out = 32, f = (1, 2, -1, -2): coefficient i carries
    f(round(i p_in / 2N)) = f(floor((4 i + 8) / 16)) -> messages
    (0, 0, 1, 1, 1, 1, 2, 2), values (1, 1, 2, 2, 2, 2, -1, -1), times
    Delta_out = 2^27."""
    v = O.test_poly(8, 4, [1, 2, -1, -2], p_out=32)
    assert [int(x) for x in v] == [x * 2 ** 27 for x in (1, 1, 2, 2, 2, 2, 31, 31)]
    with pytest.raises(ValueError):  # f(r + 2) = -f(r) mod 32 fails for r = 0
        O.test_poly(8, 4, [1, 2, 1, -2], p_out=32)
    # the same space reduces to the plain definition
    f = O.lut_fire(32, 4)
    assert np.array_equal(O.test_poly(1024, 32, f, p_out=32), O.test_poly(1024, 32, f))


# ------------------------------------------------------------------ P8: encryption

def test_encrypt_decrypt_all_messages(okeys_a):
    P = O.SHAPE_A
    m = np.tile(np.arange(-P.p // 2 + 1, P.p // 2 + 1, dtype=np.int32), 8)
    ct = O.encrypt(P, okeys_a.s, m, 7)
    assert np.array_equal(O.decrypt(P.p, okeys_a.s, ct), m)
    err = _signed(O.phase(okeys_a.s, ct).astype(np.int64) - (m.astype(np.int64) % P.p) * P.delta)
    assert np.abs(err).max() < 6 * P.sigma_lwe * U32


# ------------------------------------------------------------------ P9-P11: BR / extract / KS

def _small_keys(n, sigma_bsk, s=None, seed=21):
    P = O.Params(n=n, sigma_bsk=sigma_bsk, sigma_ksk=0.0)
    s0, z = O.secret_keys(P, seed)
    s = s0 if s is None else np.asarray(s, np.int32)
    bsk = np.zeros((P.n, 2 * P.l, 2, P.N), np.uint32)
    O.lib().or_keygen_bsk_range(ctypes.byref(P.c()), seed, O._i32(s), O._i32(z), 0, P.n,
                                O._u32(bsk))
    return O.Keys(P, s, z, bsk, np.zeros((1,), np.uint32))


def _rlwe_phase(acc, z):
    return (acc[1] - O.negacyclic_mul(acc[0], z.astype(np.uint32))).astype(np.uint32)


def test_blind_rotation_special_cases():
    n = 12
    g = synth.rng(16)
    ct = g.integers(0, U32, size=n + 1, dtype=np.uint64).astype(np.uint32)
    v = O.test_poly(1024, 32, O.lut_fire(32, 4))
    N = 1024
    bbar = O.mod_switch(int(ct[n]), N)
    # s = 0 and noiseless keys: every CMux selects ACC, phase is exactly X^{-b~} v
    K = _small_keys(n, 0.0, s=np.zeros(n, np.int32))
    acc = O.blind_rotate(K, v, ct)
    assert np.array_equal(_rlwe_phase(acc, K.z), O.mul_xpow((2 * N - bbar) % (2 * N), v))
    # s = e_3: one rotation by a~_3, up to the gadget rounding error of one CMux
    s = np.zeros(n, np.int32)
    s[3] = 1
    K = _small_keys(n, 0.0, s=s)
    acc = O.blind_rotate(K, v, ct)
    a3 = O.mod_switch(int(ct[3]), N)
    want = O.mul_xpow((2 * N - bbar + a3) % (2 * N), v)
    err = _signed(_rlwe_phase(acc, K.z).astype(np.int64) - want.astype(np.int64))
    assert np.abs(err).max() <= (N + 1) * (1 << (31 - 3 * 7))
    # the direction matters: rotating the other way is far off
    wrong = O.mul_xpow((2 * N - bbar - a3) % (2 * N), v)
    assert np.abs(_signed(_rlwe_phase(acc, K.z).astype(np.int64) - wrong.astype(np.int64))).max() > 1 << 20


def test_sample_extract_phase():
    N = 1024
    g = synth.rng(17)
    acc = g.integers(0, U32, size=(2, N), dtype=np.uint64).astype(np.uint32)
    _, z = O.secret_keys(O.SHAPE_A, 3)
    ext = O.sample_extract(acc)
    assert O.phase(z, ext)[0] == _rlwe_phase(acc, z)[0]


def test_sample_extract_at_phase():
    """Extraction of coefficient k: the LWE phase is coefficient k of the
    RLWE phase, for every k (including 0 and N-1)."""
    N = 1024
    g = synth.rng(18)
    acc = g.integers(0, U32, size=(2, N), dtype=np.uint64).astype(np.uint32)
    _, z = O.secret_keys(O.SHAPE_A, 3)
    ph = _rlwe_phase(acc, z)
    for k in (0, 1, 2, 511, N - 1):
        assert O.phase(z, O.sample_extract_at(acc, k))[0] == ph[k], k
    assert np.array_equal(O.sample_extract_at(acc, 0), O.sample_extract(acc))


def test_mod_switch_even_is_doubled_rounding_to_z_n():
    N = 1024
    g = synth.rng(19)
    xs = list(g.integers(0, U32, size=200, dtype=np.uint64)) + [0, U32 - 1, 1 << 21, (1 << 21) - 1,
                                                              (1 << 22) + (1 << 21), 1 << 31]
    for x in xs:
        r = math.floor(Fraction(int(x) * N, U32) + Fraction(1, 2)) % N
        assert O.mod_switch_even(int(x), N) == 2 * r, x


def test_test_poly_two_hand_example():
    """N = 8, p = 4: u = 0..3 carries message floor((4u + 4) / 8) = 0, 1, 1, 2;
    f0 = (1, 2, -1, -2) on even and f1 = (0, 1, 0, -1) on odd coefficients,
    times Delta = 2^30."""
    v = O.test_poly_two(8, 4, [1, 2, -1, -2], [0, 1, 0, -1])
    assert [int(x) for x in v] == [x * 2 ** 30 for x in (1, 0, 2, 1, 2, 1, 3, 0)]
    with pytest.raises(ValueError):
        O.test_poly_two(8, 4, [1, 2, -1, -2], [0, 1, 1, -1])


def test_one_rotation_computes_both_functions(okeys_a):
    """Fire and Reset interleaved in one test polynomial and read from one
    even-exponent blind rotation decrypt to both functions of every message
    (p = 16, so that the doubled modulus-switching error keeps a 6-sigma
    margin; the keys do not depend on p)."""
    P = replace(O.SHAPE_A, p=16)
    K = O.Keys(P, okeys_a.s, okeys_a.z, okeys_a.bsk, okeys_a.ksk)
    m = np.arange(-P.p // 2 + 1, P.p // 2 + 1, dtype=np.int32)
    ct = O.encrypt(P, K.s, m, 12)
    s2, v = O.lif_step_one_rotation(K, 4, 2, ct)
    assert list(O.decrypt(P.p, K.s, s2)) == list(O.centred(P.p, O.plain_fire(P.p, 4, m)))
    assert list(O.decrypt(P.p, K.s, v)) == list(O.centred(P.p, O.plain_reset(P.p, 4, 2, m)))


def test_keyswitch_rounding_bound():
    P = O.Params(sigma_ksk=0.0)
    K = O.keygen(P, 5)
    g = synth.rng(18)
    x = g.integers(0, U32, size=(4, P.N + 1), dtype=np.uint64).astype(np.uint32)
    out = O.keyswitch(K, x)
    err = _signed(O.phase(K.s, out).astype(np.int64) - O.phase(K.z, x).astype(np.int64))
    wt = int(K.z.sum())
    assert np.abs(err).max() <= wt * (1 << 15)


# ------------------------------------------------------------------ P13: bootstrapping computes f

def test_pbs_computes_the_program_function(okeys_a):
    P = O.SHAPE_A
    m = np.arange(-P.p // 2 + 1, P.p // 2 + 1, dtype=np.int32)
    ct = O.encrypt(P, okeys_a.s, m, 8)
    vf, vr = O.lif_test_polys(P, 4, 2)
    fire = O.decrypt(P.p, okeys_a.s, O.pbs(okeys_a, vf, ct))
    reset = O.decrypt(P.p, okeys_a.s, O.pbs(okeys_a, vr, ct))
    assert list(fire) == list(O.centred(P.p, O.lut_fire(P.p, 4)[m % P.p]))
    assert list(reset) == list(O.centred(P.p, O.lut_reset(P.p, 4, 2)[m % P.p]))


def _triple_map(p_in, p_out):
    """f(k) = 3k on [0, p_in/2), extended negacyclically: f(k + p_in/2) = -f(k)."""
    h = p_in // 2
    return np.array([3 * k if k < h else -3 * (k - h) for k in range(p_in)], np.int32) % p_out


def test_pbs_changes_the_message_space(okeys_a):
    """Inputs in Z_16 (even messages of Z_32: Delta_16 = 2 Delta_32), f(k) = 3k
    (negacyclic extension), outputs decrypted in Z_32: every message maps to
    f(k) mod 32.  (Z_64 outputs would decrypt with a 2.2-sigma margin at
    these parameters: the output space must keep 1/(2 p_out) above the
    bootstrapping's output noise.)"""
    P = O.SHAPE_A
    k = np.arange(16, dtype=np.int32)
    ct = O.encrypt(P, okeys_a.s, 2 * k, 11)
    f = _triple_map(16, 32)
    out = O.pbs(okeys_a, O.test_poly(P.N, 16, f, p_out=32), ct)
    assert list(O.decrypt(32, okeys_a.s, out)) == list(O.centred(32, f[k]))


# ------------------------------------------------------------------ WeightSum

def test_lwe_linear_is_matrix_product():
    g = synth.rng(19)
    W = g.integers(-15, 16, size=(7, 13)).astype(np.int32)
    x = g.integers(0, U32, size=(13, 9), dtype=np.uint64).astype(np.uint32)
    want = (W.astype(object) @ x.astype(object)) % U32
    assert np.array_equal(O.lwe_linear(W, x), want.astype(np.uint32))


def test_lwe_conv2d_is_correlation():
    g = synth.rng(20)
    Ci, H, Wd, Co, K, st, pd = 2, 9, 7, 3, 5, 2, 2
    W = g.integers(-15, 16, size=(Co, Ci, K, K)).astype(np.int32)
    x = g.integers(0, U32, size=(Ci * H * Wd, 3), dtype=np.uint64).astype(np.uint32)
    y = O.lwe_conv2d(W, x, Ci, H, Wd, st, pd)
    xi = x.astype(np.int64).reshape(Ci, H, Wd, 3)
    for w in range(3):
        for co in range(Co):
            acc = 0
            for ci in range(Ci):
                xp = np.pad(xi[ci, :, :, w], pd)
                acc = acc + signal.correlate2d(xp, W[co, ci].astype(np.int64), mode="valid")
            want = (acc[::st, ::st] % U32).reshape(-1)
            Ho, Wo = acc[::st, ::st].shape
            got = y[co * Ho * Wo:(co + 1) * Ho * Wo, w]
            assert np.array_equal(got.astype(np.int64), want)


def test_weightsum_noise_growth(okeys_a):
    """Noise after WeightSum of fresh samples: std sigma*sqrt(sum w^2), below
    the bound sigma*sum|w| of Sec. 4.1 (Eq. noise_estimate_computing)."""
    P = O.SHAPE_A
    g = synth.rng(22)
    W = g.integers(-8, 9, size=(400, 64)).astype(np.int32)
    x = g.integers(0, 8, size=64).astype(np.int32)
    ct = O.encrypt(P, okeys_a.s, x, 9)
    y = O.lwe_linear(W, ct)
    mu = (W.astype(np.int64) @ x.astype(np.int64)) % P.p * P.delta
    err = _signed(O.phase(okeys_a.s, y).astype(np.int64) - mu) / U32
    ratio = err / (P.sigma_lwe * np.sqrt((W.astype(np.float64) ** 2).sum(1)))
    assert abs(ratio.std() - 1) < 0.15
    assert np.all(np.abs(err) <= 5 * P.sigma_lwe * np.abs(W).sum(1))


# ------------------------------------------------------------------ Theorem 3.1 / 4.1 on the plaintext SNN

def test_theorem_4_1_range_on_plaintext_snn():
    """With M = V + max|I| <= p/2, the integer recurrence keeps every H in
    [V - p/2, p/2) (Theorem 4.1), so the mod-p recurrence never wraps and
    equals the integer one."""
    p, V, tau = 32, 4, 2
    g = synth.rng(23)
    for _ in range(50):
        I = g.integers(-(p // 2 - V), p // 2 - V + 1, size=40)
        Hs, Ss, Vs = O.plain_lif_layer_run(p, I, V, tau, 6)
        Vt = np.zeros_like(I)
        for H, S, Vn in zip(Hs, Ss, Vs):
            Ht = Vt + I                      # unreduced integers
            assert np.all(Ht >= V - p // 2) and np.all(Ht < p // 2)
            assert np.array_equal(O.centred(p, H), Ht)
            spike = Ht >= V
            assert np.array_equal(S == 2, spike)
            Vt = np.where(spike | (Ht <= 0), 0, np.floor(Ht * (tau - 1) / tau + 0.5)).astype(np.int64)
            assert np.array_equal(O.centred(p, Vn), Vt)


def test_plaintext_lif_matches_float_discretisation():
    """Theorem 3.1: without wrap, 2S = 2 exactly when H >= V, and V' is 0
    after a spike or on H <= 0, else the leaked H."""
    p, V, tau = 64, 4, 2
    g = synth.rng(24)
    I = g.integers(0, 6, size=200)
    Hs, Ss, Vs = O.plain_lif_layer_run(p, I, V, tau, 5)
    for H, S, Vn in zip(Hs, Ss, Vs):
        H = O.centred(p, H)
        assert np.array_equal(S == 2, H >= V)
        leak = np.floor((H * (tau - 1) / tau) + 0.5)
        want = np.where((H >= V) | (H <= 0), 0, leak)
        assert np.array_equal(O.centred(p, Vn), want)
