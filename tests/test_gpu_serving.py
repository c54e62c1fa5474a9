"""Multi-key batching and the serving loop: every result is byte-identical
whether its work ran alone or batched with other requests and clients."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2309_09025_amd import fhesnn as F
from paper_2309_09025_amd import network as NW
from paper_2309_09025_amd import serve as SV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clients(gpu_env):
    ctx, get = gpu_env
    P = F.params_default(0)
    out = {}
    for cid, seed in enumerate((synth.SEED_KEYS, 11, 12)):
        sk, evk = F.keygen(P, seed)
        out[cid] = (sk, evk, F.evk_upload(ctx, evk))
    return out


@pytest.mark.parametrize("variant,mode", [(0, "rows"), (0, "two"), (0, "paired"), (1, "one"),
                                          (2, "one")])
def test_pbs_lif_ranges_equals_one_call_per_range(gpu_env, clients, okeys_a, variant, mode):
    """Multi-key launch == one launch per range == oracle, on the row and
    two-group kernels (small batches) and on two one-group variants."""
    ctx, _ = gpu_env
    P = F.params_default(0)
    ctx.set_br_variant(P.N, variant)
    try:
        with ctx.groups(mode):
            _ranges_case(ctx, clients, okeys_a, P)
    finally:
        ctx.set_br_variant(P.N, 0)


def _ranges_case(ctx, clients, okeys_a, P):
    sizes = [(0, 10), (1, 7), (0, 5), (2, 40)]  # (client, neurons); 124 bootstrappings
    hs, outs, ranges = [], [], []
    for k, (cid, cnt) in enumerate(sizes):
        sk, evk, dk = clients[cid]
        m = synth.messages(synth.SEED_DATA, cnt, P.p, stream=50 + k)
        h = F.to_device(F.encrypt(sk, m, synth.SEED_ENC, 7000 + 100 * k))
        s2 = torch.zeros((cnt, P.n + 1), dtype=torch.int32, device="cuda")
        v = torch.zeros_like(s2)
        hs.append((cid, h, m))
        outs.append((s2, v))
        ranges.append((dk, h, s2, v))
    F.pbs_lif_ranges(ctx, 4, 2, ranges)
    torch.cuda.synchronize()
    for (cid, h, m), (s2, v) in zip(hs, outs):
        dk = clients[cid][2]
        a2 = torch.zeros_like(s2)
        av = torch.zeros_like(v)
        F.pbs_lif(ctx, dk, 4, 2, h, a2, av)
        torch.cuda.synchronize()
        assert np.array_equal(F.to_host(s2), F.to_host(a2))
        assert np.array_equal(F.to_host(v), F.to_host(av))
    # the first range (client 0 = keys of seed 1) against the oracle
    cid, h, m = hs[0]
    spikes, vnew = O.lif_step(okeys_a, 4, 2, F.to_host(h))
    assert np.array_equal(F.to_host(outs[0][0]), spikes)
    assert np.array_equal(F.to_host(outs[0][1]), vnew)


def _server(ctx, base, widths, budget):
    nets = {}
    for h in widths:
        cfg = synth.ConvSNN(**{**base.__dict__, "hidden": h})
        _, Wc, W1, W2 = cfg.data()
        nets[h] = (W1, W2)
    geom = (base.Ci, base.H, base.Wd, base.stride, base.pad)
    return SV.Server(ctx, Wc, nets, geom, NW.LifSpec(base.vth, base.tau), budget_bytes=budget)


def test_serving_results_equal_alone_and_in_the_mix(gpu_env, clients):
    ctx, _ = gpu_env
    base = synth.CONV_SNN_MINI
    widths = (8, 12)
    spec = [(0, 2, 8, 0.0), (1, 3, 12, 0.0), (2, 1, 12, 0.0), (0, 3, 8, 0.05),
            (2, 2, 8, 0.05), (1, 1, 12, 0.1)]  # (client, T, hidden, arrival)
    reqs = []
    for rid, (cid, T, H, at) in enumerate(spec):
        sk = clients[cid][0]
        px = synth.ConvSNN(**{**base.__dict__}).data(image_stream=rid)[0]
        reqs.append(SV.Request(rid, cid, F.encrypt(sk, px, synth.SEED_ENC, 100000 * rid), T, H, at))
    srv = _server(ctx, base, widths, budget=0)
    for cid, (sk, evk, dk) in clients.items():
        srv.keys[cid] = dk
        srv.width = dk.params.n + 1
    srv.budget = 3 * max(srv.request_bytes(h) for h in widths)  # at most 3 in flight
    done = srv.run(reqs)
    assert srv.pbs_count == sum(2 * r.T * (base.l1 + r.hidden) for r in reqs)
    assert all(r.latency > 0 for r in done)
    for r in reqs:
        alone = _server(ctx, base, widths, budget=1 << 30)
        alone.keys = {r.client: clients[r.client][2]}
        alone.width = srv.width
        solo = SV.Request(r.rid, r.client, r.px_ct, r.T, r.hidden, 0.0)
        alone.run([solo])
        assert np.array_equal(solo.score, r.score), r.rid
        # and the same as the single-image network
        W1, W2 = alone.nets[r.hidden]
        net = NW.ConvSNN(ctx, clients[r.client][2], synth.CONV_SNN_MINI.data()[1],
                         F.to_host(W1).view(np.int32), F.to_host(W2).view(np.int32),
                         (base.Ci, base.H, base.Wd, base.stride, base.pad),
                         NW.LifSpec(base.vth, base.tau))
        score, _ = net.run(F.to_device(r.px_ct), r.T)
        assert np.array_equal(score, r.score), r.rid
    stats = SV.latency_stats(done)
    assert stats["p99_s"] >= stats["p50_s"] > 0


def test_checkpoint_and_resume_on_another_server_is_byte_identical(gpu_env, clients):
    """A request checkpointed after two of its four timesteps, its device
    memory freed, and resumed on a second server with its own context (a
    restart) finishes with the same score bits as an uninterrupted run; a
    cancelled request releases its memory; an oversized resume is refused."""
    ctx, _ = gpu_env
    base = synth.CONV_SNN_MINI
    widths = (8, 12)
    cid, T, H = 1, 4, 12
    sk, evk, dk = clients[cid]
    px = synth.ConvSNN(**{**base.__dict__}).data(image_stream=7)[0]
    ct = F.encrypt(sk, px, synth.SEED_ENC, 700000)

    ref = _server(ctx, base, widths, budget=1 << 30)
    ref.keys = {cid: dk}
    ref.width = dk.params.n + 1
    whole = SV.Request(0, cid, ct, T, H)
    ref.run([whole])

    first = _server(ctx, base, widths, budget=1 << 30)
    first.keys = {cid: dk}
    first.width = ref.width
    r = SV.Request(1, cid, ct, T, H)
    first.admit(r)
    assert first.step([r]) == [] and first.step([r]) == []
    state = first.checkpoint(r)
    assert first.mem_used == 0 and state["t"] == 2

    ctx2 = F.Context(0)  # a fresh context and key upload, as after a restart
    second = _server(ctx2, base, widths, budget=1 << 30)
    second.register(cid, evk)
    r2 = SV.Request(2, cid, ct, T, H)
    second.resume(r2, state)
    done = []
    while not done:
        done = second.step([r2])
    assert np.array_equal(r2.score, whole.score)

    tiny = _server(F.Context(0), base, widths, budget=1)  # one server per context
    tiny.keys, tiny.width = second.keys, second.width
    with pytest.raises(MemoryError):
        tiny.resume(SV.Request(3, cid, ct, T, H), state)
    second.admit(r3 := SV.Request(4, cid, ct, T, H))
    second.cancel(r3)
    assert second.mem_used == 0


def test_admission_by_device_memory_returns_fs_ebudget(gpu_env):
    """fs_ctx_admit / fs_ctx_release through the C ABI: requests are admitted
    while their bytes fit the budget, FS_EBUDGET (nothing admitted) past it
    or past the device's free memory, released bytes admit the next one."""
    ctx = F.Context(0)
    L = F.lib()
    assert ctx.admission() == (0, 0)
    ctx.set_budget(1000)
    assert L.fs_ctx_admit(ctx.h, 600) == F.FS_OK
    assert L.fs_ctx_admit(ctx.h, 600) == F.FS_EBUDGET
    assert "budget" in L.fs_last_error().decode()
    assert ctx.admission() == (1000, 600)
    assert ctx.admit(400) and not ctx.admit(1)
    ctx.release(600)
    assert ctx.admit(500) and ctx.admission() == (1000, 900)
    with pytest.raises(F.FsError) as ei:
        ctx.release(901)
    assert ei.value.code == F.FS_EINVAL
    ctx.release(900)
    # no budget: the device's free memory still bounds a request
    ctx.set_budget(0)
    total = torch.cuda.get_device_properties(0).total_memory
    assert L.fs_ctx_admit(ctx.h, 2 * total) == F.FS_EBUDGET
    assert ctx.admit(1 << 20) and ctx.admission() == (0, 1 << 20)
    ctx.release(1 << 20)
