"""Context state on the GPU: scratch growth after a graph capture, the
thread-group thresholds per ring degree, and the multi-range launch refusing
capture."""
import numpy as np
import pytest
import torch

import synth
from paper_2309_09025_amd import fhesnn as F
from paper_2309_09025_amd import network as NW
from paper_2309_09025_amd import tune

pytestmark = pytest.mark.gpu


def test_scratch_growth_after_capture_keeps_the_graph_valid(gpu_env):
    """A network captures its timestep with the scratch sized for its own
    layer; a larger call then grows the context's scratch.  The old buffer
    is retired, not freed, so replays of the captured step still run on
    valid memory, and every replay gives the same bits as before the
    growth."""
    _, get = gpu_env
    P, sk, evk, dk = get(0)
    ctx = F.Context(0)  # fresh scratch
    cfg = synth.TinyLIF()
    x, W = cfg.data()
    xd = F.to_device(F.encrypt(sk, x, synth.SEED_ENC))
    net = NW.LifLayerNet(ctx, dk, W, NW.LifSpec(cfg.vth, cfg.tau), capture=True)
    before = net.run(xd, 3)  # step 1 eager, step 2 captured and replayed, step 3 replayed
    live0, retired0 = ctx.scratch_bytes()
    assert retired0 == 0 and live0 > 0
    # a larger batch on the same context grows its scratch
    B = 700
    h = F.to_device(F.encrypt(sk, synth.messages(synth.SEED_DATA, B, P.p), synth.SEED_ENC, 7000))
    s2, v = F.empty_ct(B, P.n + 1), F.empty_ct(B, P.n + 1)
    F.pbs_lif(ctx, dk, cfg.vth, cfg.tau, h, s2, v)
    torch.cuda.synchronize()
    live1, retired1 = ctx.scratch_bytes()
    assert live1 >= 2 * B * (P.N + 1) * 4 and retired1 == live0
    after = net.run(xd, 3)  # replays the graph captured before the growth
    for t in range(3):
        for a, b in zip(before[t], after[t]):
            assert np.array_equal(a, b), t
    # and the grown scratch serves the large batch like a fresh context
    ref = F.Context(0)
    s2r, vr = F.empty_ct(B, P.n + 1), F.empty_ct(B, P.n + 1)
    F.pbs_lif(ref, dk, cfg.vth, cfg.tau, h, s2r, vr)
    torch.cuda.synchronize()
    assert np.array_equal(F.to_host(s2), F.to_host(s2r))
    assert np.array_equal(F.to_host(v), F.to_host(vr))


def test_thresholds_are_kept_per_ring_degree(gpu_env):
    """Setting (or tuning) the thread-group thresholds of one ring degree
    leaves the other's unchanged."""
    _, get = gpu_env
    ctx = F.Context(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert ctx.set_rows(2048, 512) == cus        # default: one job per CU
    assert ctx.set_rows(1024, cus) == cus        # untouched by the N = 2048 change
    assert ctx.set_paired(1024, 2 * cus) == 2 * cus
    assert ctx.set_split(1024, 3 * cus) == 3 * cus
    assert ctx.set_split(2048, 0) == 0
    P, sk, evk, dk = get(1)
    limits, _ = tune.tune_groups(ctx, dk, store=False)
    assert ctx.set_rows(2048, limits[0]) == limits[0]
    assert (ctx.set_rows(1024, cus), ctx.set_paired(1024, 2 * cus),
            ctx.set_split(1024, 3 * cus)) == (cus, 2 * cus, 3 * cus)


def test_multi_range_launch_refuses_capture(gpu_env):
    """fs_pbs_lif_ranges copies its range table from host memory at the
    call, so it returns FS_ENOTSUP on a capturing stream (before enqueueing
    anything)."""
    ctx, get = gpu_env
    P, sk, evk, dk = get(0)
    h = F.to_device(F.encrypt(sk, synth.messages(synth.SEED_DATA, 4, P.p), synth.SEED_ENC))
    s2, v = F.empty_ct(4, P.n + 1), F.empty_ct(4, P.n + 1)
    F.pbs_lif_ranges(ctx, 4, 2, [(dk, h, s2, v)])  # fills the caches eagerly
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g):
        s2.add_(0)
        try:
            F.pbs_lif_ranges(ctx, 4, 2, [(dk, h, s2, v)])
        except F.FsError as e:
            err = e
    assert err is not None and err.code == F.FS_ENOTSUP
    assert "captured" in str(err)
