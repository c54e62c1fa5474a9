"""The one-limb N = 2048 key form (FS_KEY_ONE_LIMB: whole 32-bit key
coefficients in the transform, half the products and inverse transforms of
the exact form) against the oracle, bit for bit: every kernel variant, both
thread-group forms, the LIF activation, a full 4096 batch against the
two-limb form; keys of different forms are refused in one multi-key
launch."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2309_09025_amd import fhesnn as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def one_limb():
    """Shape B keys (seed 1) uploaded in the one-limb form on a context of
    their own."""
    P = F.params_default(1)
    sk, evk = F.keygen(P, synth.SEED_KEYS)
    ctx = F.Context(0)
    dk = F.evk_upload(ctx, evk, F.FS_KEY_ONE_LIMB)
    return P, sk, evk, ctx, dk


def _inputs(P, sk, okeys, count, first):
    m = synth.messages(synth.SEED_DATA, first + count, P.p)[first:]
    ct = F.encrypt(sk, m, synth.SEED_ENC, first)
    assert np.array_equal(ct, O.encrypt(okeys.params, okeys.s, m, synth.SEED_ENC, first))
    return m, ct


def _host(t):
    torch.cuda.synchronize()
    return F.to_host(t)


def test_form_and_resident_bytes(one_limb, gpu_env):
    P, sk, evk, ctx, dk = one_limb
    assert dk.form == F.FS_KEY_ONE_LIMB
    _, get = gpu_env
    dk2 = get(1)[3]
    assert dk2.form == F.FS_KEY_EXACT
    bsk_one = P.n * 2 * P.l * 2 * P.N * 8  # doubles, one limb
    assert dk2.nbytes - dk.nbytes == bsk_one
    # at N = 1024 the two forms are the same key
    Pa = F.params_default(0)
    ska, evka = F.keygen(Pa, synth.SEED_KEYS)
    assert F.evk_upload(ctx, evka, F.FS_KEY_ONE_LIMB).form == F.FS_KEY_EXACT


@pytest.mark.parametrize("keyswitch", [False, True])
def test_one_limb_pbs_bit_exact(one_limb, okeys_b, keyswitch):
    """A small batch (the two-group form) against the oracle."""
    P, sk, evk, ctx, dk = one_limb
    m, ct = _inputs(P, sk, okeys_b, 6, 1400)
    f = O.lut_fire(P.p, 4)
    width = P.n + 1 if keyswitch else P.N + 1
    out = torch.zeros((len(m), width), dtype=torch.int32, device="cuda")
    F.pbs(ctx, dk, f, F.to_device(ct), out, keyswitch=keyswitch)
    assert np.array_equal(_host(out), O.pbs(okeys_b, O.test_poly(P.N, P.p, f), ct,
                                            keyswitch=keyswitch))


@pytest.mark.parametrize("variant", range(9))
def test_one_limb_every_variant_bit_exact(one_limb, okeys_b, variant):
    P, sk, evk, ctx, dk = one_limb
    m, ct = _inputs(P, sk, okeys_b, 5, 1500 + 5 * variant)
    f = O.lut_reset(P.p, 4, 2)
    out = torch.zeros((len(m), P.N + 1), dtype=torch.int32, device="cuda")
    ctx.set_br_variant(P.N, variant)
    try:
        with ctx.groups("one", P.N):
            F.pbs(ctx, dk, f, F.to_device(ct), out, keyswitch=False)
            got = _host(out)
    finally:
        ctx.set_br_variant(P.N, 0)
    assert np.array_equal(got, O.pbs(okeys_b, O.test_poly(P.N, P.p, f), ct, keyswitch=False))


def test_one_limb_lif_bit_exact_and_forms_not_mixed(one_limb, okeys_b, gpu_env):
    P, sk, evk, ctx, dk = one_limb
    m, ct = _inputs(P, sk, okeys_b, 35, 1600)
    s2 = torch.zeros((len(m), P.n + 1), dtype=torch.int32, device="cuda")
    vv = torch.zeros_like(s2)
    F.pbs_lif(ctx, dk, 4, 2, F.to_device(ct), s2, vv)
    idx = [0, 34]
    spikes, vnew = O.lif_step(okeys_b, 4, 2, ct[idx])
    assert np.array_equal(_host(s2)[idx], spikes)
    assert np.array_equal(_host(vv)[idx], vnew)
    # a multi-key launch of one-limb keys equals the single-key call
    s3, v3 = torch.zeros_like(s2), torch.zeros_like(s2)
    h = F.to_device(ct)
    F.pbs_lif_ranges(ctx, 4, 2, [(dk, h[:20], s3[:20], v3[:20]), (dk, h[20:], s3[20:], v3[20:])])
    assert torch.equal(s3, s2) and torch.equal(v3, vv)
    # keys of both forms in one launch are refused
    _, get = gpu_env
    dk2 = get(1)[3]
    ctx2 = F.Context(0)
    with pytest.raises(F.FsError) as ei:
        F.pbs_lif_ranges(ctx2, 4, 2, [(dk, h[:20], s3[:20], v3[:20]),
                                       (dk2, h[20:], s3[20:], v3[20:])])
    assert ei.value.code == F.FS_EPARAM


def test_one_limb_full_batch_equals_two_limb_form(one_limb, okeys_b, gpu_env):
    """4096 fresh ciphertexts through the one-group kernel in both key forms:
    the same bits (the two-limb form is exact for every key), and sampled
    rows against the oracle."""
    P, sk, evk, ctx, dk = one_limb
    ctx0, get = gpu_env
    dk2 = get(1)[3]
    B = 4096
    m = synth.messages(synth.SEED_DATA, B, P.p)
    ct = F.encrypt(sk, m, synth.SEED_ENC)
    fire, _ = F.lif_luts(4, 2, P.p)
    h = F.to_device(ct)
    out1 = torch.zeros((B, P.N + 1), dtype=torch.int32, device="cuda")
    out2 = torch.zeros_like(out1)
    F.pbs(ctx, dk, fire, h, out1, keyswitch=False)
    F.pbs(ctx0, dk2, fire, h, out2, keyswitch=False)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    idx = [0, 2047, 4095]
    want = O.pbs(okeys_b, O.test_poly(P.N, P.p, fire), ct[idx], keyswitch=False)
    assert np.array_equal(_host(out1)[idx], want)
