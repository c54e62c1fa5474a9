"""Edge cases of the device path against the oracle: empty batches, crafted
ciphertexts at the rounding boundaries of the modulus switch and the key
switch, trivial ciphertexts (every CMux step skipped), extreme words and
weights in WeightSum, and empty ranges in a multi-range launch."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2309_09025_amd import fhesnn as F

pytestmark = pytest.mark.gpu

U32 = 2 ** 32


def _host(t):
    torch.cuda.synchronize()
    return F.to_host(t)


def test_empty_batches_are_no_ops(gpu_env):
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    e_s = F.empty_ct(0, P.n + 1)
    e_z = F.empty_ct(0, P.N + 1)
    fire, _ = F.lif_luts(4, 2, P.p)
    F.pbs(ctx, dk, fire, e_s, e_s, keyswitch=True)
    F.pbs(ctx, dk, fire, e_s, e_z, keyswitch=False)
    F.pbs_mspace(ctx, dk, fire, P.p, 8, e_s, e_s)
    F.pbs_lif(ctx, dk, 4, 2, e_s, e_s, F.empty_ct(0, P.n + 1))
    F.pbs_lif_ks_first(ctx, dk, 4, 2, e_z, e_z, F.empty_ct(0, P.N + 1))
    F.keyswitch(ctx, dk, e_z, e_s)
    F.pbs_lif_ranges(ctx, 4, 2, [])
    W = F.to_device(np.zeros((0, 5), np.int32))
    F.lwe_linear(ctx, W, F.empty_ct(5, P.n + 1), e_s)
    F.lwe_add(ctx, e_s, e_s, e_s)
    torch.cuda.synchronize()


def _boundary_cts(P, count, seed):
    """Ciphertexts whose words sit on the modulus-switch boundaries: with
    nu = log2 2N, x rounds to Z_2N at multiples of 2^(32-nu) and the ties
    (x = k 2^(32-nu) + 2^(31-nu)) go up; 0, 2^31 and 2^32 - 1 wrap."""
    nu = (2 * P.N).bit_length() - 1
    step, half = 1 << (32 - nu), 1 << (31 - nu)
    g = synth.rng(seed, 4)
    ct = g.integers(0, U32, size=(count, P.n + 1), dtype=np.uint64)
    special = np.array([0, U32 - 1, 1 << 31, half, half - 1, step - half, U32 - half,
                        U32 - half - 1, 3 * step + half, 7 * step + half - 1], np.uint64)
    mask = g.random(size=ct.shape) < 0.5
    ct[mask] = special[g.integers(0, special.size, size=int(mask.sum()))]
    ct[0, :] = special[np.arange(P.n + 1) % special.size]
    return ct.astype(np.uint32)


@pytest.mark.parametrize("shape,keyswitch", [(0, True), (0, False), (1, False)])
def test_pbs_of_boundary_words_bit_exact(gpu_env, okeys_a, okeys_b, shape, keyswitch):
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    ct = _boundary_cts(P, 5 if shape == 0 else 2, 900 + shape)
    f = O.lut_reset(P.p, 4, 2)
    width = P.n + 1 if keyswitch else P.N + 1
    out = torch.zeros((ct.shape[0], width), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, f, F.to_device(ct), out, keyswitch=keyswitch)
    assert np.array_equal(_host(out), O.pbs(ok, O.test_poly(P.N, P.p, f), ct, keyswitch=keyswitch))


def test_trivial_ciphertexts_skip_every_step(gpu_env, okeys_a):
    """a = 0 (and a_i rounding to 0): every CMux step is skipped and the result
    is the rotated test polynomial, extracted and key-switched."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m = np.arange(P.p, dtype=np.int64)
    ct = np.zeros((P.p, P.n + 1), np.uint32)
    ct[:, -1] = (m * (U32 // P.p)).astype(np.uint32)
    ct[1::2, :-1] = np.uint32(U32 - 1)  # rounds to 0 as well
    f = O.lut_fire(P.p, 4)
    out = torch.zeros((P.p, P.n + 1), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, f, F.to_device(ct), out)
    got = _host(out)
    assert np.array_equal(got, O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct))
    # noiseless input: the output decrypts to f(m) for every m (key-switch noise only)
    assert np.array_equal(F.decrypt(sk, got), O.centred(P.p, f[m % P.p]))


@pytest.mark.parametrize("shape", [0, 1])
def test_keyswitch_of_extreme_words_bit_exact(gpu_env, okeys_a, okeys_b, shape):
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    nu = 16  # the key switch rounds to t * beta = 16 bits
    half = 1 << (31 - nu)
    rows = [np.zeros(P.N + 1), np.full(P.N + 1, U32 - 1), np.full(P.N + 1, 1 << 31),
            np.full(P.N + 1, half), np.full(P.N + 1, half - 1),
            np.arange(P.N + 1) * 0x9E3779B9 % U32]
    x = np.array(rows, np.uint64).astype(np.uint32)
    out = torch.zeros((x.shape[0], P.n + 1), dtype=torch.int32, device="cuda")
    F.keyswitch(ctx, dk, F.to_device(x), out)
    assert np.array_equal(_host(out), O.keyswitch(ok, x))


def test_weightsum_of_extreme_words_and_weights_bit_exact(gpu_env):
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    g = synth.rng(synth.SEED_DATA, 950)
    O_, I = 9, 70
    W = g.integers(-2 ** 31, 2 ** 31, size=(O_, I), dtype=np.int64).astype(np.int32)
    W[0, :] = -2 ** 31
    W[1, :] = 2 ** 31 - 1
    x = g.integers(0, U32, size=(I, P.n + 1), dtype=np.uint64).astype(np.uint32)
    x[:10] = np.uint32(U32 - 1)
    add = g.integers(0, U32, size=(O_, P.n + 1), dtype=np.uint64).astype(np.uint32)
    y = torch.zeros((O_, P.n + 1), dtype=torch.int32, device="cuda")
    F.lwe_linear(ctx, F.to_device(W), F.to_device(x), y, add=F.to_device(add))
    assert np.array_equal(_host(y), O.lwe_linear(W, x, add))


def test_empty_ranges_between_ranges(gpu_env, okeys_a):
    """fs_pbs_lif_ranges with empty ranges among non-empty ones equals one
    fs_pbs_lif call per non-empty range."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m = synth.messages(synth.SEED_DATA, 7, P.p, stream=960)
    h = F.to_device(F.encrypt(sk, m, synth.SEED_ENC, 96000))
    parts = [(0, 0), (0, 3), (3, 3), (3, 7), (7, 7)]
    outs = [(torch.zeros((b - a, P.n + 1), dtype=torch.int32, device="cuda"),
             torch.zeros((b - a, P.n + 1), dtype=torch.int32, device="cuda")) for a, b in parts]
    F.pbs_lif_ranges(ctx, 4, 2, [(dk, h[a:b], s, v) for (a, b), (s, v) in zip(parts, outs)])
    s_all = torch.zeros((7, P.n + 1), dtype=torch.int32, device="cuda")
    v_all = torch.zeros_like(s_all)
    F.pbs_lif(ctx, dk, 4, 2, h, s_all, v_all)
    torch.cuda.synchronize()
    got_s = np.concatenate([F.to_host(s) for s, _ in outs])
    got_v = np.concatenate([F.to_host(v) for _, v in outs])
    assert np.array_equal(got_s, F.to_host(s_all)) and np.array_equal(got_v, F.to_host(v_all))


def test_oversized_batches_are_rejected_before_any_work(gpu_env):
    """Batch sizes past what a launch grid can address are refused with
    FS_EINVAL by the C entry points themselves (the pointers are never
    touched: they are placeholders here)."""
    import ctypes
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    L = F.lib()
    fake = ctypes.c_void_p(0x1000)
    lut = np.zeros(P.p, np.int32)
    lif = F.CLif(4, 2)
    huge = 1 << 40
    cases = {
        "fs_pbs": lambda: L.fs_pbs(ctx.h, dk.h, lut.ctypes.data_as(F._i32p), fake, huge, fake, 1,
                                   None),
        "fs_pbs_lif": lambda: L.fs_pbs_lif(ctx.h, dk.h, ctypes.byref(lif), fake, huge, fake,
                                           ctypes.c_void_p(0x2000), None),
        "fs_pbs_lif_ks_first": lambda: L.fs_pbs_lif_ks_first(ctx.h, dk.h, ctypes.byref(lif), fake,
                                                             huge, fake, ctypes.c_void_p(0x2000),
                                                             None),
        "fs_pbs_lif_many_lut": lambda: L.fs_pbs_lif_many_lut(ctx.h, dk.h, ctypes.byref(lif), fake,
                                                             huge, fake, ctypes.c_void_p(0x2000),
                                                             None),
        "fs_keyswitch": lambda: L.fs_keyswitch(ctx.h, dk.h, fake, huge, fake, None),
    }
    for name, call in cases.items():
        assert call() == F.FS_EINVAL, name
        assert "too large" in L.fs_last_error().decode(), name
