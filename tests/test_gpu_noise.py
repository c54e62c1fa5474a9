"""Statistical checks of the GPU bootstrapping outputs (decryption, not bits):
every message maps to its program-function value, and the output noise has
the variance the standard TFHE error analysis predicts for these parameters.
Bit-exact agreement with the oracle is covered by test_gpu_parity.py; these
tests check that what is computed is the intended function at the intended
noise level (Theorem 2.1: the bootstrapping evaluates f while resetting the
noise)."""
import math

import numpy as np
import pytest
import torch

import synth
from paper_2309_09025_amd import fhesnn as F

pytestmark = pytest.mark.gpu


def _phase(s, ct, dim):
    """b - <a, key> mod 2^32 for rows of `ct` (uint32 [count][dim])."""
    a = ct[:, : dim - 1].astype(np.uint64)
    dot = (a * s.astype(np.uint64)[None, :]).sum(axis=1) & 0xFFFFFFFF
    return (ct[:, dim - 1].astype(np.uint64) - dot) & 0xFFFFFFFF


def _centred_error(phase, want, delta):
    """(phase - delta * want) as a signed torus value in [-1/2, 1/2)."""
    d = (phase.astype(np.int64) - (want.astype(np.int64) * delta)) & 0xFFFFFFFF
    d = np.where(d >= 2 ** 31, d - 2 ** 32, d)
    return d / 2.0 ** 32


def _model_variance(P, keyswitch=True):
    """Output variance of blind rotation (+ key switch) from the standard TFHE
    analysis: per CMux step (k+1) l N digit products with the key noise
    (digits uniform in [-Bg/2, Bg/2): E d^2 = (Bg^2 + 2)/12) plus the gadget
    rounding of l Bg-bit digits times (1 + N/2); the key switch adds one KSK
    noise per non-zero digit (3/4 of N t digits for uniform coefficients) and
    the 16-bit rounding of N/2 key-weighted coefficients."""
    Bg = 2 ** P.bg_bit
    sb2, sk2 = P.sigma_bsk ** 2, P.sigma_ksk ** 2
    var_br = P.n * (2 * P.l * P.N * (Bg * Bg + 2) / 12 * sb2
                    + (1 + P.N / 2) * 2.0 ** (-2 * P.l * P.bg_bit) / 12)
    if not keyswitch:
        return var_br
    base = 2 ** P.ks_base_bit
    prec = P.ks_t * P.ks_base_bit
    var_ks = P.N * P.ks_t * (base - 1) / base * sk2 + (P.N / 2) * 2.0 ** (-2 * prec) / 12
    return var_br + var_ks


def _run(ctx, dk, lut, ct, width):
    out = torch.zeros((ct.shape[0], width), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, lut, F.to_device(ct), out, keyswitch=(width == dk.params.n + 1))
    torch.cuda.synchronize()
    return F.to_host(out)


@pytest.mark.parametrize("which", ["fire", "reset"])
def test_every_message_decrypts_to_its_function_value(gpu_env, which):
    """All of Z_32 x 64 repetitions through Fire and Reset (N = 1024, after the
    key switch).  Predicted failure rate 8.7e-6 per decryption: a failure is
    accepted only with an error beyond 4 model standard deviations."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    fire, reset = F.lif_luts(4, 2, P.p)
    f = np.asarray(fire if which == "fire" else reset)
    m = np.tile(np.arange(P.p, dtype=np.int32) - P.p // 2 + 1, 64)
    ct = F.encrypt(sk, m, synth.SEED_ENC, 100000)
    out = _run(ctx, dk, f, ct, P.n + 1)
    want = np.mod(f[np.mod(m, P.p)], P.p)
    want_c = np.where(want > P.p // 2, want - P.p, want)
    got = F.decrypt(sk, out)
    bad = np.nonzero(got != want_c)[0]
    if bad.size:
        s = np.asarray(sk.export()[0], np.int64)
        err = _centred_error(_phase(s, out[bad], P.n + 1), want[bad], 2 ** 32 // P.p)
        sigma = math.sqrt(_model_variance(P))
        assert np.all(np.abs(err) > 4 * sigma), (bad, err / sigma)


def _ksk_noise(P, sk, evk):
    """Noise of every key-switching key row, e[i][j][v-1] = phase_s(row) -
    v z_i 2^{32 - (j+1) beta} as torus values (the key's own, fixed draws)."""
    s, z = (np.asarray(x, np.int64) for x in sk.export())
    _, ksk = evk.export(bsk=False, ksk=True)
    base = 2 ** P.ks_base_bit
    rows = ksk.reshape(-1, P.n + 1)
    ph = _phase(s, rows, P.n + 1).reshape(P.N, P.ks_t, base - 1)
    i, j, v = np.meshgrid(np.arange(P.N), np.arange(P.ks_t), np.arange(1, base), indexing="ij")
    msg = (v * z[i] * (2 ** (32 - (j + 1) * P.ks_base_bit))) & 0xFFFFFFFF
    d = (ph.astype(np.int64) - msg) & 0xFFFFFFFF
    return np.where(d >= 2 ** 31, d - 2 ** 32, d) / 2.0 ** 32


def test_output_noise_matches_the_error_model(gpu_env):
    """4096 Fire bootstrappings of uniform messages (the batched workload).
    With one key, the key switch's error is not zero-mean over samples: every
    digit position (i, j) subtracts the noise of the row its digit selects, so
    given the key the error has mean -(1/base) sum e_ijv and variance
    sum_ij [mean_v e_ijv^2 - (mean_v e_ijv)^2] over the digit values (value 0
    selects no row), with e the key's own KSK noise.  Added to the blind
    rotation's variance (standard analysis: (k+1) l N digit products per step
    with digits uniform in [-Bg/2, Bg/2), plus the gadget rounding) and the
    16-bit rounding of N/2 key-weighted coefficients, this predicts the
    measured mean within 4 standard errors (plus the blind rotation's own
    fixed-key offset, which the digits' mean -1/2 leaves at std
    0.5 sigma_bsk sqrt(n (k+1) l N)) and the sample variance inside its
    99.9 % chi-square interval widened by 10 % for the uniform-digit
    assumption."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    fire, _ = F.lif_luts(4, 2, P.p)
    f = np.asarray(fire)
    m = synth.messages(synth.SEED_DATA, 4096, P.p)
    ct = F.encrypt(sk, m, synth.SEED_ENC)
    out = _run(ctx, dk, f, ct, P.n + 1)
    s = np.asarray(sk.export()[0], np.int64)
    err = _centred_error(_phase(s, out, P.n + 1), np.mod(f[np.mod(m, P.p)], P.p), 2 ** 32 // P.p)

    base = 2 ** P.ks_base_bit
    e = _ksk_noise(P, sk, evk)                    # [N][t][base-1]
    sel = np.concatenate([np.zeros(e.shape[:2] + (1,)), e], axis=2)  # value 0: no row
    mean_ks = -sel.mean(axis=2).sum()
    var_ks = (sel ** 2).mean(axis=2).sum() - (sel.mean(axis=2) ** 2).sum()
    var_round = (P.N / 2) * 2.0 ** (-2 * P.ks_t * P.ks_base_bit) / 12
    var_pred = _model_variance(P, keyswitch=False) + var_ks + var_round
    br_offset = 0.5 * P.sigma_bsk * math.sqrt(P.n * 2 * P.l * P.N)

    n = err.size
    mean, var = err.mean(), err.var(ddof=1)
    se = math.sqrt(var / n)
    print(f"\nnoise: std 2^{math.log2(math.sqrt(var)):.3f}, predicted 2^{math.log2(math.sqrt(var_pred)):.3f}, "
          f"ratio {var / var_pred:.4f}; mean {mean:.3e}, predicted {mean_ks:.3e}, "
          f"(mean - predicted)/se {(mean - mean_ks) / se:.2f}")
    assert abs(mean - mean_ks) < 4 * se + 4 * br_offset
    half = 3.29 * math.sqrt(2.0 / (n - 1))  # 99.9 % two-sided, normal approximation
    assert 1 - half - 0.10 < var / var_pred < 1 + half + 0.10


def test_key_switch_first_outputs_carry_blind_rotation_noise_only(gpu_env):
    """Key-switch-first LIF activation on every message x 32 (1024 neurons,
    2048 blind rotations): outputs under z decrypt to Fire + 1 and Reset,
    and the spike outputs' error variance is the blind rotation's alone
    (model std 2^-8.85 against 2^-8.15 with the key switch after it).  A
    wrong decryption is accepted only for a neuron whose key-switched input
    lies within 5 mod-switch standard deviations of its window edge."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m = np.tile(np.arange(P.p, dtype=np.int32) - P.p // 2 + 1, 32)
    h = F.encrypt_z(sk, m, synth.SEED_ENC, 300000)
    s2 = torch.zeros((m.size, P.N + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    hd = F.to_device(h)
    F.pbs_lif_ks_first(ctx, dk, 4, 2, hd, s2, vv)
    hs = torch.zeros((m.size, P.n + 1), dtype=torch.int32, device="cuda")
    F.keyswitch(ctx, dk, hd, hs)  # the same key-switched input, for the error check
    torch.cuda.synchronize()
    got_s, got_v, got_h = F.to_host(s2), F.to_host(vv), F.to_host(hs)
    s, z = (np.asarray(x, np.int64) for x in sk.export())
    fire, reset = (np.asarray(x) for x in F.lif_luts(4, 2, P.p))
    r = np.mod(m, P.p)
    want_s = np.mod(fire[r] + 1, P.p)
    want_v = np.mod(reset[r], P.p)
    err_in = _centred_error(_phase(s, got_h, P.n + 1), r, 2 ** 32 // P.p)
    sigma_ms = math.sqrt((1 + P.n / 2) / (12 * (2 * P.N) ** 2))
    near_edge = np.abs(err_in) > 0.5 / P.p - 5 * sigma_ms
    for got, want in ((got_s, want_s), (got_v, want_v)):
        bad = F.decrypt(sk, got) != np.where(want > P.p // 2, want - P.p, want)
        assert np.all(near_edge[bad]), np.nonzero(bad)[0]
    ok = ~near_edge
    err = _centred_error(_phase(z, got_s[ok], P.N + 1), want_s[ok], 2 ** 32 // P.p)
    var_pred = _model_variance(P, keyswitch=False)
    ratio = err.var(ddof=1) / var_pred
    print(f"\nkey switch first, output noise: std 2^{math.log2(err.std()):.3f}, "
          f"model 2^{math.log2(math.sqrt(var_pred)):.3f} (ratio of variances {ratio:.3f}); "
          f"{int(near_edge.sum())} inputs near an edge")
    assert 0.7 < ratio < 1.3


def test_many_lut_outputs_follow_the_rounded_phase(gpu_env):
    """One rotation for Fire and Reset (fs_pbs_lif_many_lut), every message x
    64 at p = 32.  The phase is rounded to even exponents, so the message the
    rotation actually reads is that of the rounded phase, m~ = round(u p / N)
    with 2u = b~ - sum a~_i s_i mod 2N; computed here from the key, every
    output must decrypt to f(m~) (the blind rotation itself is exact up to
    its output noise, 4.45 sigma; at most 2 of the 4096 decryptions may fall
    in that tail).  m~ differs from m for the inputs whose
    doubled modulus-switching error crosses a window edge: that rate is
    reported against the model (about 0.2 % at 3.1 sigma)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m = np.tile(np.arange(P.p, dtype=np.int32) - P.p // 2 + 1, 64)
    ct = F.encrypt(sk, m, synth.SEED_ENC, 400000)
    s2 = torch.zeros((m.size, P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    F.pbs_lif_many_lut(ctx, dk, 4, 2, F.to_device(ct), s2, vv)
    torch.cuda.synchronize()
    got_s, got_v = F.decrypt(sk, F.to_host(s2)), F.decrypt(sk, F.to_host(vv))
    s = np.asarray(sk.export()[0], np.int64)
    N, nu = P.N, P.N.bit_length() - 1
    even = lambda x: 2 * (((x.astype(np.int64) + (1 << (31 - nu))) % 2 ** 32) >> (32 - nu)) % (2 * N)
    phase = (even(ct[:, -1]) - (even(ct[:, :-1]) * s[None, :]).sum(axis=1)) % (2 * N)
    m_read = ((phase // 2) * P.p + N // 2) // N % P.p
    fire, reset = (np.asarray(x, np.int64) for x in F.lif_luts(4, 2, P.p))
    cen = lambda r: np.where(r % P.p > P.p // 2, r % P.p - P.p, r % P.p)
    # the output side may fail with the bootstrapping's own rate (~1e-5 per
    # decryption, 4096 decryptions here)
    wrong = int((got_s != cen(fire[m_read] + 1)).sum() + (got_v != cen(reset[m_read])).sum())
    assert wrong <= 2, wrong
    moved = float(np.mean(m_read != np.mod(m, P.p)))
    sigma_ms = math.sqrt((1 + P.n / 2) / 12) / N
    model = 2 * 0.5 * math.erfc((0.5 / P.p) / sigma_ms / math.sqrt(2))
    print(f"\nmany-LUT: input message moved by the rounding in {moved:.4%} of {m.size} "
          f"(model {model:.4%}, margin {(0.5 / P.p) / sigma_ms:.2f} sigma)")
    assert moved < 0.02


def test_shape_b_blind_rotation_decrypts_before_key_switch(gpu_env):
    """N = 2048, p = 64: every message x 16 through Fire, checked on the
    extracted sample under z (after the key switch a 4.7 % failure rate is
    predicted by the model, so the pre-key-switch output is the one pinned)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(1)
    fire, _ = F.lif_luts(4, 2, P.p)
    f = np.asarray(fire)
    m = np.tile(np.arange(P.p, dtype=np.int32) - P.p // 2 + 1, 16)
    ct = F.encrypt(sk, m, synth.SEED_ENC, 200000)
    out = _run(ctx, dk, f, ct, P.N + 1)
    z = np.asarray(sk.export()[1], np.int64)
    err = _centred_error(_phase(z, out, P.N + 1), np.mod(f[np.mod(m, P.p)], P.p), 2 ** 32 // P.p)
    assert np.all(np.abs(err) < 0.5 / P.p)
    sigma = math.sqrt(_model_variance(P, keyswitch=False))
    print(f"\nshape B pre-KS noise: std 2^{math.log2(err.std()):.3f}, model 2^{math.log2(sigma):.3f}")


def test_shape_b_with_smaller_key_switch_noise_decrypts_after_key_switch(gpu_env):
    """N = 2048, p = 64 end to end (after the key switch) with the key-switching
    key's noise lowered to 2^-17: the key switch then adds std ~2^-10.2 and
    the output error (~2^-10.1 with the blind rotation's) sits ~8.5 sigma
    inside the half window 2^-7, and the doubled-N modulus switch keeps the
    input at 6.2 sigma; every message x 16 through Fire decrypts correctly.
    (A parameter choice only: its security level is not estimated here.)"""
    ctx, _ = gpu_env
    P = F.params_default(1)
    P.sigma_ksk = 2.0 ** -17
    sk, evk = F.keygen(P, synth.SEED_KEYS)
    dk = F.evk_upload(ctx, evk)
    fire, _ = F.lif_luts(4, 2, P.p)
    f = np.asarray(fire)
    m = np.tile(np.arange(P.p, dtype=np.int32) - P.p // 2 + 1, 16)
    ct = F.encrypt(sk, m, synth.SEED_ENC, 500000)
    out = _run(ctx, dk, f, ct, P.n + 1)
    want = np.mod(f[np.mod(m, P.p)], P.p)
    assert np.array_equal(F.decrypt(sk, out), np.where(want > P.p // 2, want - P.p, want))
    s = np.asarray(sk.export()[0], np.int64)
    err = _centred_error(_phase(s, out, P.n + 1), want, 2 ** 32 // P.p)
    print(f"\nshape B, sigma_ksk 2^-17, after key switch: std 2^{math.log2(err.std()):.3f}, "
          f"max |err| {np.abs(err).max() * P.p * 2:.3f} of the half window")
