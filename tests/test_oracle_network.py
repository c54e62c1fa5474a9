"""The encrypted LIF network of the oracle against the plaintext integer SNN,
spike for spike (Theorem 3.1 recurrence; Sec. 4.2 FHE-Fire / FHE-Reset;
Sec. 4.1 WeightSum), on the tiny LIF layer workload: 64 encrypted 3-bit
inputs, weights in [-8, 8], 32 LIF neurons (V = 4, tau = 2), T = 2."""
import numpy as np

import synth
from oracle import oracle as O


def test_tiny_lif_layer_encrypted_equals_plaintext(okeys_a):
    P = O.SHAPE_A
    cfg = synth.TinyLIF()
    x, W = cfg.data()
    x_ct = O.encrypt(P, okeys_a.s, x, synth.SEED_ENC)
    I_ct = O.lwe_linear(W, x_ct)
    Hs, Ss, Vs = O.lif_layer_run(okeys_a, I_ct, cfg.vth, cfg.tau, cfg.T)
    I = (W.astype(np.int64) @ x.astype(np.int64))
    pH, pS, pV = O.plain_lif_layer_run(P.p, I, cfg.vth, cfg.tau, cfg.T)
    for t in range(cfg.T):
        assert np.array_equal(O.decrypt(P.p, okeys_a.s, Hs[t]), O.centred(P.p, pH[t])), t
        assert np.array_equal(O.decrypt(P.p, okeys_a.s, Ss[t]), O.centred(P.p, pS[t])), t
        assert np.array_equal(O.decrypt(P.p, okeys_a.s, Vs[t]), O.centred(P.p, pV[t])), t


def test_tiny_lif_layer_key_switch_first_equals_plaintext(okeys_a):
    """The same layer with the key switch in front of each blind rotation:
    inputs and states under z, decrypted with z, spike for spike with the
    plaintext SNN; the spike outputs' error is that of blind rotation alone."""
    P = O.SHAPE_A
    cfg = synth.TinyLIF()
    x, W = cfg.data()
    x_ct = O.encrypt_z(P, okeys_a.z, x, synth.SEED_ENC)
    assert x_ct.shape == (x.size, P.N + 1)
    I_ct = O.lwe_linear(W, x_ct)
    Hs, Ss, Vs = O.lif_layer_run(okeys_a, I_ct, cfg.vth, cfg.tau, cfg.T, ks_first=True)
    I = (W.astype(np.int64) @ x.astype(np.int64))
    pH, pS, pV = O.plain_lif_layer_run(P.p, I, cfg.vth, cfg.tau, cfg.T)
    for t in range(cfg.T):
        assert Ss[t].shape == (cfg.neurons, P.N + 1)
        assert np.array_equal(O.decrypt(P.p, okeys_a.z, Hs[t]), O.centred(P.p, pH[t])), t
        assert np.array_equal(O.decrypt(P.p, okeys_a.z, Ss[t]), O.centred(P.p, pS[t])), t
        assert np.array_equal(O.decrypt(P.p, okeys_a.z, Vs[t]), O.centred(P.p, pV[t])), t
    # spike outputs: blind-rotation noise only (std 2^-8.85 by the standard
    # analysis), far inside the half window 1/64; with the key switch after
    # the rotation it would be 2^-8.15
    err = (O.phase(okeys_a.z, Ss[-1]).astype(np.int64) - (pS[-1] % P.p) * P.delta) & 0xFFFFFFFF
    err = np.where(err >= 2 ** 31, err - 2 ** 32, err) / 2.0 ** 32
    assert np.abs(err).max() < 4.5 * 2.0 ** -8.85


def test_sum_pool_decrypts_to_window_sums(okeys_a):
    """Average-pool numerator on ciphertexts (Sec. 3.3): the window sums of
    the decrypted grid, computed here by reshaping into k x k blocks."""
    P = O.SHAPE_A
    C, H, W, k = 2, 6, 6, 2
    m = synth.uniform_int(synth.SEED_DATA, C * H * W, 0, 2, stream=61)
    ct = O.encrypt(P, okeys_a.s, m, synth.SEED_ENC, 3000)
    got = O.decrypt(P.p, okeys_a.s, O.lwe_sum_pool(ct, C, H, W, k))
    want = m.reshape(C, H // k, k, W // k, k).sum(axis=(2, 4)).reshape(-1)
    assert np.array_equal(got, O.centred(P.p, want))


def test_paper_csnn_counts_match_table_1():
    """Table 1: (1440 x 2 + 2 x 160 + 2 x 10) T bootstrappings per image."""
    c = synth.PAPER_CSNN
    assert (c.l1, c.pooled) == (1440, 360)
    assert c.pbs_count() == (1440 * 2 + 2 * 160 + 2 * 10) * c.T


def test_paper_csnn_oracle_first_layer_equals_plaintext(okeys_a):
    """A small instance of the paper's topology on the oracle: the first LIF
    layer (noise 2^-15 x conv weights, far inside the window) decrypts spike
    for spike to the plaintext network, and every stored step is the
    recurrence of Theorem 3.1 layer by layer (the pooled FC input is the
    window sum of the layer-1 spikes).  Deeper layers sum many bootstrapping
    outputs (noise 2^-8.3 each) with weights up to 8: their decryptions are
    not pinned (the same holds for the paper's network without its trained,
    discretised weights)."""
    P = O.SHAPE_A
    cfg = synth.PaperCSNN(H=6, Wd=6, Co=2, K=4, stride=2, pad=1, hidden=4, classes=2, T=2)
    px, Wc, W1, W2 = cfg.data()
    geom = (cfg.Ci, cfg.H, cfg.Wd, cfg.stride, cfg.pad)
    ct = O.encrypt(P, okeys_a.s, px, synth.SEED_ENC)
    I1, steps = O.paper_csnn_run(okeys_a, ct, Wc, W1, W2, geom, cfg.pool, cfg.vth, cfg.tau, cfg.T)
    _, psteps = O.plain_paper_csnn_run(P.p, px, Wc, W1, W2, geom, cfg.pool, cfg.vth, cfg.tau, cfg.T)
    for t in range(cfg.T):
        for k in ("H1", "S1", "V1"):
            assert np.array_equal(O.decrypt(P.p, okeys_a.s, steps[t][k]),
                                  O.centred(P.p, psteps[t][k])), (t, k)
        pooled = O.lwe_sum_pool(steps[t]["S1"], cfg.Co, cfg.Ho, cfg.Wo, cfg.pool)
        V2prev = steps[t - 1]["V2"] if t else O.zero_ct(cfg.hidden, P.n + 1)
        assert np.array_equal(steps[t]["H2"], O.lwe_linear(W1, pooled, add=V2prev))
        V3prev = steps[t - 1]["V3"] if t else O.zero_ct(cfg.classes, P.n + 1)
        assert np.array_equal(steps[t]["H3"], O.lwe_linear(W2, steps[t]["S2"], add=V3prev))


def test_poisson_counts_match_table_1():
    """Table 1: (784 + 2 x 160 + 2 x 10) T1 bootstrappings per image."""
    c = synth.POISSON_SNN
    assert c.pbs_count() == (784 + 2 * 160 + 2 * 10) * c.T


def test_add_plain_rows_adds_each_rows_plaintext(okeys_a):
    """A per-row plaintext added to ciphertexts decrypts to the sums mod p."""
    P = O.SHAPE_A
    m = synth.uniform_int(synth.SEED_DATA, 40, -15, 16, stream=71)
    c = synth.uniform_int(synth.SEED_DATA, 40, -40, 40, stream=72)
    ct = O.encrypt(P, okeys_a.s, m, synth.SEED_ENC, 9000)
    got = O.decrypt(P.p, okeys_a.s, O.add_plain_rows(P.p, ct, c))
    assert np.array_equal(got, O.centred(P.p, m.astype(np.int64) + c))


def test_poisson_snn_oracle_spikes_equal_plaintext(okeys_a):
    """Poisson coding on ciphertexts (Sec. 2.3: X = 1 iff pixel > threshold,
    as one Sign bootstrapping) decrypts to 2X of the plaintext coding at every
    step, and each layer's input is the WeightSum of the previous layer's
    spikes plus V (Theorem 3.1).  The LIF layers' decryptions are not pinned:
    their inputs sum 16 bootstrapped spikes with weights up to 8."""
    P = O.SHAPE_A
    cfg = synth.PoissonSNN(H=4, Wd=4, hidden=4, classes=2, T=3)
    px, W1, W2 = cfg.data()
    thr = cfg.thresholds()
    ct = O.encrypt(P, okeys_a.s, px, synth.SEED_ENC)
    steps = O.poisson_snn_run(okeys_a, ct, thr, W1, W2, cfg.vth, cfg.tau, cfg.T)
    psteps = O.plain_poisson_snn_run(P.p, px, thr, W1, W2, cfg.vth, cfg.tau, cfg.T)
    for t in range(cfg.T):
        assert np.array_equal(O.decrypt(P.p, okeys_a.s, steps[t]["S0"]),
                              O.centred(P.p, psteps[t]["S0"])), t
        V1prev = steps[t - 1]["V1"] if t else O.zero_ct(cfg.hidden, P.n + 1)
        assert np.array_equal(steps[t]["H1"], O.lwe_linear(W1, steps[t]["S0"], add=V1prev))
        V2prev = steps[t - 1]["V2"] if t else O.zero_ct(cfg.classes, P.n + 1)
        assert np.array_equal(steps[t]["H2"], O.lwe_linear(W2, steps[t]["S1"], add=V2prev))
    assert any(psteps[t]["S0"].any() for t in range(cfg.T))  # some pixel spiked



# ---------------------------------------------------------------------------
# Whole networks against the plaintext integer SNN.  With real noise the
# layers after the first sum dozens of bootstrapped outputs (std 2^-8.15
# each) and no longer decrypt reliably, so the compositions are pinned with
# noiseless keys (okeys_a_quiet): every ciphertext of every step, the score
# accumulators included, must decrypt to the mod-p recurrence of Theorem 3.1
# (Eq. DiscretEquation) with WeightSum layers (Sec. 4.1) and scores summed
# over the T steps.  A wrong operand anywhere (a missing V, a layer fed the
# wrong spikes, a score not accumulated) changes some decryption; the
# checks below also make sure each instance exercises those terms.

def _decrypts_to(keys, ct, plain, p):
    return np.array_equal(O.decrypt(p, keys.s, ct), O.centred(p, plain))


def _exercises(psteps, V, S, score):
    """The instance makes the recurrence matter: some potential V survives
    a step, some neuron of the layer spikes and some does not, and the
    score changes after the first step."""
    assert any(np.any(st[V] % 32 != 0) for st in psteps[:-1]), V
    spikes = np.concatenate([st[S] for st in psteps])
    assert np.any(spikes == 2) and np.any(spikes == 0), S
    assert any(not np.array_equal(psteps[t][score], psteps[0][score])
               for t in range(1, len(psteps))), score


def test_conv_snn_oracle_equals_plaintext_at_every_step(okeys_a_quiet):
    """conv_snn_run (conv (LIF) -> FC (LIF) -> FC score accumulators) against
    plain_conv_snn_run, every state and the scores, T = 3."""
    K = okeys_a_quiet
    P = K.params
    cfg = synth.ConvSNN(H=6, Wd=6, Co=2, K=3, stride=2, pad=1, hidden=4, classes=3,
                        w_lo=-2, w_hi=2, T=3)
    px, Wc, W1, W2 = cfg.data()
    geom = (cfg.Ci, cfg.H, cfg.Wd, cfg.stride, cfg.pad)
    ct = O.encrypt(P, K.s, px, synth.SEED_ENC)
    I1, steps = O.conv_snn_run(K, ct, Wc, W1, W2, geom, cfg.vth, cfg.tau, cfg.T)
    pI1, psteps = O.plain_conv_snn_run(P.p, px, Wc, W1, W2, geom, cfg.vth, cfg.tau, cfg.T)
    assert _decrypts_to(K, I1, pI1, P.p)
    for t in range(cfg.T):
        for k in ("H1", "S1", "V1", "H2", "S2", "V2", "score"):
            assert _decrypts_to(K, steps[t][k], psteps[t][k], P.p), (t, k)
    _exercises(psteps, "V1", "S1", "score")
    _exercises(psteps, "V2", "S2", "score")
    # the score is the sum over steps of W2 2S[t], not the last step's alone
    tot = sum(np.asarray(W2, np.int64) @ psteps[t]["S2"] for t in range(cfg.T)) % P.p
    assert np.array_equal(psteps[-1]["score"], tot)


def test_paper_csnn_oracle_equals_plaintext_at_every_step(okeys_a_quiet):
    """paper_csnn_run (conv (LIF) -> sum pool -> FC (LIF) -> FC (LIF), spike
    counts as scores) against plain_paper_csnn_run, every state and the
    scores."""
    K = okeys_a_quiet
    P = K.params
    cfg = synth.PaperCSNN(H=8, Wd=8, Co=2, K=4, stride=2, pad=1, hidden=4, classes=3,
                          w_lo=-3, w_hi=3, T=3)
    px, Wc, W1, W2 = cfg.data()
    geom = (cfg.Ci, cfg.H, cfg.Wd, cfg.stride, cfg.pad)
    ct = O.encrypt(P, K.s, px, synth.SEED_ENC)
    _, steps = O.paper_csnn_run(K, ct, Wc, W1, W2, geom, cfg.pool, cfg.vth, cfg.tau, cfg.T)
    _, psteps = O.plain_paper_csnn_run(P.p, px, Wc, W1, W2, geom, cfg.pool, cfg.vth, cfg.tau,
                                       cfg.T)
    for t in range(cfg.T):
        for k in ("H1", "S1", "V1", "H2", "S2", "V2", "H3", "S3", "V3", "score"):
            assert _decrypts_to(K, steps[t][k], psteps[t][k], P.p), (t, k)
    _exercises(psteps, "V2", "S2", "score")
    tot = sum(psteps[t]["S3"] for t in range(cfg.T)) % P.p
    assert np.array_equal(psteps[-1]["score"], tot)


def test_poisson_snn_oracle_equals_plaintext_at_every_step(okeys_a_quiet):
    """poisson_snn_run (Sign coding -> FC (LIF) -> FC (LIF), spike counts as
    scores) against plain_poisson_snn_run, every state and the scores."""
    K = okeys_a_quiet
    P = K.params
    cfg = synth.PoissonSNN(H=4, Wd=4, hidden=4, classes=3, w_lo=-3, w_hi=3, T=3)
    px, W1, W2 = cfg.data()
    thr = cfg.thresholds()
    ct = O.encrypt(P, K.s, px, synth.SEED_ENC)
    steps = O.poisson_snn_run(K, ct, thr, W1, W2, cfg.vth, cfg.tau, cfg.T)
    psteps = O.plain_poisson_snn_run(P.p, px, thr, W1, W2, cfg.vth, cfg.tau, cfg.T)
    for t in range(cfg.T):
        for k in ("S0", "H1", "S1", "V1", "H2", "S2", "V2", "score"):
            assert _decrypts_to(K, steps[t][k], psteps[t][k], P.p), (t, k)
    _exercises(psteps, "V1", "S1", "score")
    tot = sum(psteps[t]["S2"] for t in range(cfg.T)) % P.p
    assert np.array_equal(psteps[-1]["score"], tot)
