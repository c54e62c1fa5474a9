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
