"""Parity of the HIP path with the CPU oracle: every ciphertext word must be
identical (integer work: bit-exact).  Inputs come from the shared seeded
generators; each side encrypts and generates keys with its own code."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2309_09025_amd import fhesnn as F

pytestmark = pytest.mark.gpu


def _dev(a):
    return F.to_device(a)


def _host(t):
    torch.cuda.synchronize()
    return F.to_host(t)


@pytest.mark.parametrize("N,R,dmax", [(1024, 6, 64), (2048, 4, 512)])
def test_ntt_polymul_matches_schoolbook(gpu_env, N, R, dmax):
    ctx, _ = gpu_env
    g = synth.rng(synth.SEED_DATA, 500 + N)
    for case in ("random", "extreme"):
        if case == "random":
            d = g.integers(-dmax, dmax, size=(R, N)).astype(np.int32)
            b = g.integers(0, 2 ** 32, size=(R, N), dtype=np.uint64).astype(np.uint32)
        else:  # all products aligned at the largest magnitude
            d = np.full((R, N), -dmax, np.int32)
            b = np.full((R, N), 0x80000000, np.uint32)
        out = torch.zeros(N, dtype=torch.int32, device="cuda")
        F.ntt_polymul(ctx, N, dmax, _dev(d), _dev(b), out)
        want = np.zeros(N, np.uint32)
        for r in range(R):
            want += O.negacyclic_mul(d[r].view(np.uint32), b[r])
        assert np.array_equal(_host(out), want), case


def _pbs_inputs(P, sk_lib, okeys, count, first=0):
    m = synth.messages(synth.SEED_DATA, first + count, P.p)[first:]
    ct_lib = F.encrypt(sk_lib, m, synth.SEED_ENC, first)
    ct_or = O.encrypt(okeys.params, okeys.s, m, synth.SEED_ENC, first)
    assert np.array_equal(ct_lib, ct_or)
    return m, ct_or


@pytest.mark.parametrize("keyswitch", [False, True])
def test_pbs_fire_bit_exact(gpu_env, okeys_a, keyswitch):
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m, ct = _pbs_inputs(P, sk, okeys_a, 24)
    f = O.lut_fire(P.p, 4)
    width = P.n + 1 if keyswitch else P.N + 1
    out = torch.zeros((len(m), width), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=keyswitch)
    got = _host(out)
    want = O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct, keyswitch=keyswitch)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", [0, 1])
def test_full_batch_in_the_benchmarked_configuration_sampled(gpu_env, okeys_a, okeys_b, shape):
    """The benchmarked workload at its full size: 4096 fresh encryptions of
    uniform messages through the LIF threshold function in one launch, with
    the kernel variant the tuner picked for this batch and the matrix-core
    key switch; the oracle recomputes sampled rows (first, last, the two
    halves' boundary and random ones: 64 at N = 1024, 24 at N = 2048), and at
    N = 1024 every one of the 4096 outputs decrypts to its function value (at
    N = 2048 the key switch's noise makes about 4 % of decryptions fail, a
    property of that shape's parameters)."""
    from paper_2309_09025_amd import tune
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    B = 4096
    m = synth.messages(synth.SEED_DATA, B, P.p)
    ct = F.encrypt(sk, m, synth.SEED_ENC)
    fire, _ = F.lif_luts(4, 2, P.p)
    variant, _ = tune.tune_blind_rotation(ctx, dk, B, use_cache=True)
    out = torch.zeros((B, P.n + 1), dtype=torch.int32, device="cuda")
    try:
        F.pbs(ctx, dk, fire, _dev(ct), out, keyswitch=True)
        got = _host(out)
    finally:
        ctx.set_br_variant(P.N, 0)
    g = synth.rng(synth.SEED_DATA, 880 + shape)
    idx = sorted({0, 1, B // 2 - 1, B // 2, B - 1, *g.integers(0, B, size=59 if shape == 0 else 19)})
    want = O.pbs(ok, O.test_poly(P.N, P.p, fire), ct[idx], keyswitch=True)
    assert np.array_equal(got[idx], want), variant
    if shape == 0:
        dec = F.decrypt(sk, got)
        expect = O.centred(P.p, np.asarray(fire, np.int64)[np.mod(m, P.p)])
        assert np.array_equal(dec, expect)


@pytest.mark.parametrize("variant", range(11))
def test_every_blind_rotation_variant_bit_exact(gpu_env, okeys_a, variant):
    """Every N = 1024 variant (prefetch points, register budgets, the
    lockstep form with 4 or 8 jobs per workgroup, held forward roots, held
    forward and inverse roots) on a
    batch of 8 (a lockstep workgroup of 8 fully used, or partly empty with 4)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    assert F.br_variants(P.N) == 11
    m, ct = _pbs_inputs(P, sk, okeys_a, 8, first=200 + 8 * variant)
    f = O.lut_reset(P.p, 4, 2)
    out = torch.zeros((len(m), P.N + 1), dtype=torch.int32, device="cuda")
    ctx.set_br_variant(P.N, variant)
    try:
        with ctx.groups("one"):  # the one-group kernel of this variant
            F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=False)
            got = _host(out)
    finally:
        ctx.set_br_variant(P.N, 0)
    assert np.array_equal(got, O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct, keyswitch=False))


@pytest.mark.parametrize("variant", range(9))
def test_every_blind_rotation_variant_shape_b_bit_exact(gpu_env, okeys_b, variant):
    """Every N = 2048 variant of the exact two-limb key (lockstep pairs
    included) on 5 ciphertexts: an odd count, so the last lockstep pair
    repeats a job without writing."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(1)
    assert F.br_variants(P.N) == 9
    m, ct = _pbs_inputs(P, sk, okeys_b, 5, first=600 + 5 * variant)
    f = O.lut_fire(P.p, 4)
    out = torch.zeros((len(m), P.N + 1), dtype=torch.int32, device="cuda")
    ctx.set_br_variant(P.N, variant)
    try:
        with ctx.groups("one"):  # the one-group kernel of this variant
            F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=False)
            got = _host(out)
    finally:
        ctx.set_br_variant(P.N, 0)
    assert np.array_equal(got, O.pbs(okeys_b, O.test_poly(P.N, P.p, f), ct, keyswitch=False))


@pytest.mark.parametrize("shape,count,keyswitch", [(0, 5, True), (0, 70, True), (0, 9, False),
                                                     (0, 1, True), (1, 3, True), (1, 66, True)])
def test_split_blind_rotation_bit_exact(gpu_env, okeys_a, okeys_b, shape, count, keyswitch):
    """One thread group per digit row, two per job (alone or two jobs per
    workgroup, odd counts included) and one per job give the oracle's bits,
    with and without the key switch."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    m, ct = _pbs_inputs(P, sk, ok, count, first=900 + 97 * shape + count)
    f = O.lut_reset(P.p, 4, 2)
    width = P.n + 1 if keyswitch else P.N + 1
    want = O.pbs(ok, O.test_poly(P.N, P.p, f), ct, keyswitch=keyswitch)
    for mode in ("rows", "paired", "two", "one"):
        with ctx.groups(mode):
            out = torch.zeros((count, width), dtype=torch.int32, device="cuda")
            F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=keyswitch)
            assert np.array_equal(_host(out), want), mode


@pytest.mark.parametrize("p_in,p_out,keyswitch", [(16, 32, True), (32, 8, True), (32, 8, False),
                                                   (64, 2 ** 20, False)])
def test_pbs_message_space_change_bit_exact(gpu_env, okeys_a, p_in, p_out, keyswitch):
    """f: Z_p_in -> Z_p_out (k -> 3k + 1 on the lower half, extended
    negacyclically): bits equal to the oracle's; where the output space keeps
    a wide decryption margin (p_out = 8) every output decrypts to f."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    h = p_in // 2
    f = np.array([3 * k + 1 if k < h else -(3 * (k - h) + 1) for k in range(p_in)], np.int32)
    k = synth.rng(synth.SEED_DATA, 850 + p_in).integers(0, p_in, size=40).astype(np.int32)
    if p_in <= P.p:  # message k of Z_p_in is message k p / p_in of the key's Z_p
        ct = F.encrypt(sk, k * (P.p // p_in), synth.SEED_ENC, 62000 + p_in)
    else:  # a finer space than the key's: an encryption of 0 plus k 2^32 / p_in
        ct = F.encrypt(sk, np.zeros_like(k), synth.SEED_ENC, 62000 + p_in)
        ct[:, -1] += (k.astype(np.int64) * (2 ** 32 // p_in)).astype(np.uint32)
    width = P.n + 1 if keyswitch else P.N + 1
    out = torch.zeros((k.size, width), dtype=torch.int32, device="cuda")
    F.pbs_mspace(ctx, dk, f, p_in, p_out, _dev(ct), out, keyswitch=keyswitch)
    got = _host(out)
    want = O.pbs(okeys_a, O.test_poly(P.N, p_in, f, p_out), ct, keyswitch=keyswitch)
    assert np.array_equal(got, want)
    if p_out == 8:
        key = okeys_a.s if keyswitch else okeys_a.z
        assert np.array_equal(O.decrypt(p_out, key, got), O.centred(p_out, f[k] % p_out))
    with pytest.raises(ValueError):
        F.pbs_mspace(ctx, dk, f[:-1], p_in, p_out, _dev(ct), out, keyswitch=keyswitch)


def test_pbs_lif_bit_exact(gpu_env, okeys_a):
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m, ct = _pbs_inputs(P, sk, okeys_a, 16, first=100)
    s2 = torch.zeros((len(m), P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    F.pbs_lif(ctx, dk, 4, 2, _dev(ct), s2, vv)
    spikes, vnew = O.lif_step(okeys_a, 4, 2, ct)
    assert np.array_equal(_host(s2), spikes)
    assert np.array_equal(_host(vv), vnew)


def test_pbs_lif_batched_key_switch_bit_exact(gpu_env, okeys_a):
    """37 neurons = 74 bootstrappings: the key switch's 64-sample groups
    end in a ragged last group."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m, ct = _pbs_inputs(P, sk, okeys_a, 37, first=300)
    s2 = torch.zeros((len(m), P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    F.pbs_lif(ctx, dk, 4, 2, _dev(ct), s2, vv)
    spikes, vnew = O.lif_step(okeys_a, 4, 2, ct)
    assert np.array_equal(_host(s2), spikes)
    assert np.array_equal(_host(vv), vnew)


@pytest.mark.parametrize("shape,count,mode", [(0, 1, "two"), (0, 37, "two"), (0, 37, "one"),
                                              (0, 21, "rows"), (0, 600, "one"), (0, 19, "paired"),
                                              (1, 3, "two"), (1, 5, "one"), (1, 4, "rows")])
def test_pbs_lif_key_switch_first_bit_exact(gpu_env, okeys_a, okeys_b, shape, count, mode):
    """Key switch of LWE_z(H), then Fire and Reset rotations extracted
    straight into the two outputs under z (one- and two-group kernels,
    ragged batch sizes): the oracle recomputes sampled neurons; at N = 1024
    every neuron also decrypts to the LIF functions of its message."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    m = synth.messages(synth.SEED_DATA, count, P.p, stream=800 + count)
    h = F.encrypt_z(sk, m, synth.SEED_ENC, 60000 + 1000 * shape + count)
    s2 = torch.zeros((count, P.N + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    with ctx.groups(mode):
        F.pbs_lif_ks_first(ctx, dk, 4, 2, _dev(h), s2, vv)
    got_s, got_v = _host(s2), _host(vv)
    idx = sorted({0, count // 2, count - 1})
    spikes, vnew = O.lif_step_ks_first(ok, 4, 2, h[idx])
    assert np.array_equal(got_s[idx], spikes)
    assert np.array_equal(got_v[idx], vnew)
    if shape == 0:
        # the input error after the key switch is ~4.5 sigma from a window
        # edge: a rare flip (7e-6 per neuron) is the scheme's, not the kernel's
        wrong = (F.decrypt(sk, got_s) != O.centred(P.p, O.plain_fire(P.p, 4, m))).sum()
        wrong += (F.decrypt(sk, got_v) != O.centred(P.p, O.plain_reset(P.p, 4, 2, m))).sum()
        assert wrong <= 1, wrong


@pytest.mark.parametrize("shape,count,mode", [(0, 1, "two"), (0, 37, "two"), (0, 37, "one"),
                                              (0, 13, "rows"), (0, 1100, "one"), (0, 23, "paired"),
                                              (1, 3, "two"), (1, 5, "one"), (1, 4, "rows")])
def test_pbs_lif_many_lut_bit_exact(gpu_env, okeys_a, okeys_b, shape, count, mode):
    """Fire and Reset from one even-exponent rotation per neuron (one- and
    two-group kernels, ragged batches, both shapes): sampled neurons equal
    the oracle's."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(shape)
    ok = okeys_a if shape == 0 else okeys_b
    m = synth.messages(synth.SEED_DATA, count, P.p, stream=870 + count)
    h = F.encrypt(sk, m, synth.SEED_ENC, 64000 + 1000 * shape + count)
    s2 = torch.zeros((count, P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    with ctx.groups(mode):
        F.pbs_lif_many_lut(ctx, dk, 4, 2, _dev(h), s2, vv)
    idx = sorted({0, count // 2, count - 1})
    spikes, vnew = O.lif_step_one_rotation(ok, 4, 2, h[idx])
    assert np.array_equal(_host(s2)[idx], spikes)
    assert np.array_equal(_host(vv)[idx], vnew)


def test_pbs_lif_key_switch_first_output_may_alias_input(gpu_env, okeys_a):
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m = synth.messages(synth.SEED_DATA, 9, P.p, stream=899)
    h = F.encrypt_z(sk, m, synth.SEED_ENC, 61000)
    hv = _dev(h)
    s2 = torch.zeros((9, P.N + 1), dtype=torch.int32, device="cuda")
    F.pbs_lif_ks_first(ctx, dk, 4, 2, hv, s2, hv)  # V' overwrites H
    spikes, vnew = O.lif_step_ks_first(okeys_a, 4, 2, h[[0, 8]])
    assert np.array_equal(_host(s2)[[0, 8]], spikes)
    assert np.array_equal(_host(hv)[[0, 8]], vnew)
    with pytest.raises(ValueError):
        F.pbs_lif_ks_first(ctx, dk, 4, 2, hv, s2[:, : P.n + 1].contiguous(), hv)


@pytest.mark.parametrize("count", [1, 21, 64, 65, 200])
def test_keyswitch_bit_exact(gpu_env, okeys_a, count):
    """Ragged batch sizes around the 64-sample groups of the matrix-core
    key switch (padding samples must not leak into real ones)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    x = synth.rng(synth.SEED_DATA, 600 + count).integers(0, 2 ** 32, size=(count, P.N + 1),
                                                          dtype=np.uint64).astype(np.uint32)
    out = torch.zeros((count, P.n + 1), dtype=torch.int32, device="cuda")
    F.keyswitch(ctx, dk, _dev(x), out)
    assert np.array_equal(_host(out), O.keyswitch(okeys_a, x))


@pytest.mark.parametrize("count", [3, 70])
def test_keyswitch_shape_b_bit_exact(gpu_env, okeys_b, count):
    ctx, get = gpu_env
    P, sk, evk, dk = get(1)
    x = synth.rng(synth.SEED_DATA, 700 + count).integers(0, 2 ** 32, size=(count, P.N + 1),
                                                          dtype=np.uint64).astype(np.uint32)
    out = torch.zeros((count, P.n + 1), dtype=torch.int32, device="cuda")
    F.keyswitch(ctx, dk, _dev(x), out)
    assert np.array_equal(_host(out), O.keyswitch(okeys_b, x))


@pytest.mark.parametrize("O_,I", [(1, 1), (32, 64), (37, 129), (256, 300)])
def test_lwe_linear_bit_exact(gpu_env, O_, I):
    ctx, _ = gpu_env
    g = synth.rng(synth.SEED_DATA, 700 + I)
    W = g.integers(-15, 16, size=(O_, I)).astype(np.int32)
    x = g.integers(0, 2 ** 32, size=(I, 631), dtype=np.uint64).astype(np.uint32)
    add = g.integers(0, 2 ** 32, size=(O_, 631), dtype=np.uint64).astype(np.uint32)
    y = torch.zeros((O_, 631), dtype=torch.int32, device="cuda")
    F.lwe_linear(ctx, _dev(W), _dev(x), y, add=_dev(add))
    assert np.array_equal(_host(y), O.lwe_linear(W, x, add))
    y2 = torch.zeros((O_, 631), dtype=torch.int32, device="cuda")
    F.lwe_linear(ctx, _dev(W), _dev(x), y2)
    assert np.array_equal(_host(y2), O.lwe_linear(W, x))


@pytest.mark.parametrize("geom", [(1, 28, 28, 8, 5, 2, 2), (2, 7, 9, 3, 3, 1, 1), (3, 5, 5, 2, 5, 2, 0)])
def test_lwe_conv2d_bit_exact(gpu_env, geom):
    ctx, _ = gpu_env
    Ci, H, Wd, Co, K, st, pd = geom
    g = synth.rng(synth.SEED_DATA, 800 + H)
    W = g.integers(-15, 16, size=(Co, Ci, K, K)).astype(np.int32)
    x = g.integers(0, 2 ** 32, size=(Ci * H * Wd, 631), dtype=np.uint64).astype(np.uint32)
    Ho = (H + 2 * pd - K) // st + 1
    Wo = (Wd + 2 * pd - K) // st + 1
    y = torch.zeros((Co * Ho * Wo, 631), dtype=torch.int32, device="cuda")
    F.lwe_conv2d(ctx, _dev(W), _dev(x), y, Ci, H, Wd, st, pd)
    assert np.array_equal(_host(y), O.lwe_conv2d(W, x, Ci, H, Wd, st, pd))


@pytest.mark.parametrize("keyswitch", [False, True])
def test_pbs_shape_b_bit_exact(gpu_env, okeys_b, keyswitch):
    """Second shape: N = 2048, l = 2, Bg = 2^10, p = 64 (the key is split in
    two 16-bit halves inside the transform)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(1)
    m, ct = _pbs_inputs(P, sk, okeys_b, 6, first=400)
    f = O.lut_fire(P.p, 4)
    width = P.n + 1 if keyswitch else P.N + 1
    out = torch.zeros((len(m), width), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=keyswitch)
    want = O.pbs(okeys_b, O.test_poly(P.N, P.p, f), ct, keyswitch=keyswitch)
    assert np.array_equal(_host(out), want)


def test_shape_b_lif_batched_key_switch_bit_exact(gpu_env, okeys_b):
    ctx, get = gpu_env
    P, sk, evk, dk = get(1)
    m, ct = _pbs_inputs(P, sk, okeys_b, 35, first=500)
    s2 = torch.zeros((len(m), P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    F.pbs_lif(ctx, dk, 4, 2, _dev(ct), s2, vv)
    # the oracle on a sample of the 70 bootstrappings (each takes seconds)
    idx = [0, 17, 34]
    spikes, vnew = O.lif_step(okeys_b, 4, 2, ct[idx])
    assert np.array_equal(_host(s2)[idx], spikes)
    assert np.array_equal(_host(vv)[idx], vnew)


def test_group_form_tuner_sets_ordered_thresholds(gpu_env, okeys_a):
    """The autotuner times the thread-group forms at 1 and 2 x CUs jobs on a
    context of its own and sets ordered thresholds; a batch in each tuned
    interval still gives the oracle's bits."""
    from paper_2309_09025_amd import tune
    _, get = gpu_env
    P, sk, evk, _ = get(0)
    ctx = F.Context(0)
    dk = F.evk_upload(ctx, evk)
    (rows, paired, split), times = tune.tune_groups(ctx, dk, intervals=2, reps=1,
                                                    use_cache=False, store=False)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert sorted(times) == [cus, 2 * cus]
    assert all(ms > 0 for t in times.values() for ms in t.values())
    assert 0 <= rows <= paired <= split <= 2 * cus
    f = O.lut_reset(P.p, 4, 2)
    for count in (3, cus + 1):
        m, ct = _pbs_inputs(P, sk, okeys_a, count, first=7000 + count)
        out = torch.zeros((count, P.n + 1), dtype=torch.int32, device="cuda")
        F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=True)
        idx = sorted({0, count // 2, count - 1})
        want = O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct[idx], keyswitch=True)
        assert np.array_equal(_host(out)[idx], want), count


@pytest.mark.parametrize("mode", ["paired", "two"])
def test_two_group_forms_beyond_one_workgroup_per_cu(gpu_env, okeys_a, mode):
    """601 jobs (an odd count) forced onto the two-group forms: more
    workgroups than CUs, so several share a CU; sampled rows (first, middle,
    the repeated last job of the paired form) equal the oracle's."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    count = 601
    m, ct = _pbs_inputs(P, sk, okeys_a, count, first=9100)
    f = O.lut_fire(P.p, 4)
    out = torch.zeros((count, P.n + 1), dtype=torch.int32, device="cuda")
    with ctx.groups(mode):
        F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=True)
    idx = [0, 300, count - 2, count - 1]
    want = O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct[idx], keyswitch=True)
    assert np.array_equal(_host(out)[idx], want)



@pytest.mark.parametrize("count,first", [(1, 9400), (1, 9401), (300, 9500)])
def test_half_row_latency_kernel_bit_exact(gpu_env, okeys_a, count, first):
    """The N = 1024 latency form (one wave per digit-row half, 12 per job)
    alone for one bootstrapping, and forced onto more jobs than the device
    has CUs (several workgroups per CU in turn): outputs before the key
    switch equal the oracle's (every row of one job, sampled rows of 300)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    m, ct = _pbs_inputs(P, sk, okeys_a, count, first=first)
    f = O.lut_reset(P.p, 4, 2)
    out = torch.zeros((count, P.N + 1), dtype=torch.int32, device="cuda")
    with ctx.groups("rows"):
        F.pbs(ctx, dk, f, _dev(ct), out, keyswitch=False)
        got = _host(out)
    idx = list(range(count)) if count < 4 else [0, 150, count - 1]
    want = O.pbs(okeys_a, O.test_poly(P.N, P.p, f), ct[idx], keyswitch=False)
    assert np.array_equal(got[idx], want)
