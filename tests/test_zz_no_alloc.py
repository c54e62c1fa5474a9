"""The LIF activation entry point that allocates nothing (fs_pbs_lif_noalloc,
static device scratch) against fs_pbs_lif on the same inputs: bit-exact on
two calls in a row, the second smaller and with another LIF function, at
the largest batch the static scratch holds, on both shapes; oversized
batches are refused before any work; the context's own scratch stays
unallocated."""
import numpy as np
import pytest
import torch

import synth
from paper_2309_09025_amd import fhesnn as F

pytestmark = pytest.mark.gpu


def _both(ctx, dk, sk, B, v_th, tau, stream_id):
    P = dk.params
    m = synth.messages(synth.SEED_DATA, B, P.p, stream=stream_id)
    h = F.to_device(F.encrypt(sk, m, synth.SEED_ENC, 90000 + 1000 * stream_id))
    ref_s, ref_v = F.empty_ct(B, P.n + 1), F.empty_ct(B, P.n + 1)
    F.pbs_lif(ctx, dk, v_th, tau, h, ref_s, ref_v)
    got_s = torch.full((B, P.n + 1), -1, dtype=torch.int32, device="cuda")
    got_v = torch.full_like(got_s, -1)
    F.pbs_lif_noalloc(ctx, dk, v_th, tau, h, got_s, got_v)
    torch.cuda.synchronize()
    return F.to_host(ref_s), F.to_host(ref_v), F.to_host(got_s), F.to_host(got_v)


@pytest.mark.parametrize("shape,sizes", [(0, (300, 37)), (1, (64, 5))])
def test_noalloc_equals_pbs_lif_on_two_calls(shape, sizes):
    P = F.params_default(shape)
    sk, evk = F.keygen(P, synth.SEED_KEYS)
    ctx = F.Context(0)
    dk = F.evk_upload(ctx, evk)
    # second call: smaller batch and another program-function pair, so the
    # test polynomials in the static scratch must be rewritten
    for k, (B, v_th, tau) in enumerate(((sizes[0], 4, 2), (sizes[1], 3, 0))):
        print(f"noalloc: shape {shape} call {k} B={B} v_th={v_th} tau={tau}", flush=True)
        rs, rv, gs, gv = _both(ctx, dk, sk, B, v_th, tau, 50 + 10 * shape + k)
        assert np.array_equal(gs, rs), f"spike ciphertexts differ (call {k})"
        assert np.array_equal(gv, rv), f"reset ciphertexts differ (call {k})"


def test_noalloc_largest_batch_and_refusal():
    P = F.params_default(0)
    sk, evk = F.keygen(P, synth.SEED_KEYS)
    ctx = F.Context(0)
    dk = F.evk_upload(ctx, evk)
    # only the static scratch: this fresh context's own scratch stays empty
    B = 4096
    m = synth.messages(synth.SEED_DATA, B, P.p, stream=77)
    h = F.to_device(F.encrypt(sk, m, synth.SEED_ENC, 123000))
    s1 = torch.full((B, P.n + 1), -1, dtype=torch.int32, device="cuda")
    v1 = torch.full_like(s1, -1)
    print(f"noalloc: largest batch B={B}", flush=True)
    F.pbs_lif_noalloc(ctx, dk, 4, 2, h, s1, v1)
    torch.cuda.synchronize()
    assert ctx.scratch_bytes() == (0, 0)
    # one batch too many: refused on the host, outputs untouched
    hb = torch.zeros((B + 1, P.n + 1), dtype=torch.int32, device="cuda")
    sb = torch.full((B + 1, P.n + 1), 7, dtype=torch.int32, device="cuda")
    vb = torch.full_like(sb, 7)
    with pytest.raises(F.FsError) as ei:
        F.pbs_lif_noalloc(ctx, dk, 4, 2, hb, sb, vb)
    assert ei.value.code == F.FS_EINVAL and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((sb == 7).all()) and bool((vb == 7).all())
    # the largest batch against the allocating entry point
    s2, v2 = F.empty_ct(B, P.n + 1), F.empty_ct(B, P.n + 1)
    F.pbs_lif(ctx, dk, 4, 2, h, s2, v2)
    torch.cuda.synchronize()
    assert np.array_equal(F.to_host(s1), F.to_host(s2))
    assert np.array_equal(F.to_host(v1), F.to_host(v2))
