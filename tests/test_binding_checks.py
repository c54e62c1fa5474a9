"""The binding checks every buffer's shape and placement before a call: the
C side receives raw device pointers and cannot see sizes, so a wrong-sized
output would become out-of-bounds device writes.  These run without a GPU:
the checks raise ValueError before anything reaches the library (CPU
tensors of the right shape are then rejected as not on a device)."""
import types

import pytest
import torch

from paper_2309_09025_amd import fhesnn as F

P = F.params_default(0)
W1 = P.n + 1
WZ = P.N + 1
CTX = types.SimpleNamespace(h=None)  # never reaches the library
DK = types.SimpleNamespace(h=None, params=P)


def ct(rows, width=W1, dtype=torch.int32):
    return torch.zeros((rows, width), dtype=dtype)


def test_dptr_rejects_host_tensors_wrong_dtype_and_non_contiguous():
    with pytest.raises(ValueError, match="device"):
        F._dptr(ct(2))
    with pytest.raises(TypeError):
        F._dptr(ct(4).numpy())


@pytest.mark.parametrize("bad", ["spike2_out", "v_out", "h"])
def test_pbs_lif_shapes(bad):
    bufs = {"h": ct(8), "spike2_out": ct(8), "v_out": ct(8)}
    bufs[bad] = ct(7) if bad != "h" else ct(8, W1 + 1)
    with pytest.raises(ValueError, match="pbs_lif"):
        F.pbs_lif(CTX, DK, 4, 2, bufs["h"], bufs["spike2_out"], bufs["v_out"])


def test_pbs_lif_right_shapes_reach_the_placement_check():
    with pytest.raises(ValueError, match="device"):
        F.pbs_lif(CTX, DK, 4, 2, ct(8), ct(8), ct(8))


def test_keyswitch_shapes():
    with pytest.raises(ValueError, match="keyswitch"):
        F.keyswitch(CTX, DK, ct(4, W1), ct(4, W1))      # input must be under z: N+1 wide
    with pytest.raises(ValueError, match="keyswitch"):
        F.keyswitch(CTX, DK, ct(4, WZ), ct(3, W1))      # one output row per input
    with pytest.raises(ValueError, match="keyswitch"):
        F.keyswitch(CTX, DK, ct(4, WZ), ct(4, WZ))      # outputs are n+1 wide


def test_lwe_linear_shapes():
    W = torch.zeros((5, 3), dtype=torch.int32)
    with pytest.raises(ValueError, match="x must be"):
        F.lwe_linear(CTX, W, ct(4), ct(5))
    with pytest.raises(ValueError, match="y must be"):
        F.lwe_linear(CTX, W, ct(3), ct(4))
    with pytest.raises(ValueError, match="add must be"):
        F.lwe_linear(CTX, W, ct(3), ct(5), add=ct(5, W1 + 1))
    with pytest.raises(ValueError, match="device"):
        F.lwe_linear(CTX, W, ct(3), ct(5), add=ct(5))


def test_lwe_conv2d_shapes():
    W = torch.zeros((2, 1, 3, 3), dtype=torch.int32)   # Co 2, Ci 1, K 3
    # 6 x 6 input, stride 2, pad 1 -> 3 x 3 outputs per channel
    with pytest.raises(ValueError, match="x must be"):
        F.lwe_conv2d(CTX, W, ct(35), ct(18), 1, 6, 6, 2, 1)
    with pytest.raises(ValueError, match="y must be"):
        F.lwe_conv2d(CTX, W, ct(36), ct(17), 1, 6, 6, 2, 1)
    with pytest.raises(ValueError, match="add must be"):
        F.lwe_conv2d(CTX, W, ct(36), ct(18), 1, 6, 6, 2, 1, add=ct(16))
    with pytest.raises(ValueError, match=r"W must be"):
        F.lwe_conv2d(CTX, W, ct(72), ct(18), 2, 6, 6, 2, 1)  # W has one input channel


def test_lwe_add_and_add_plain_shapes():
    with pytest.raises(ValueError, match="lwe_add"):
        F.lwe_add(CTX, ct(4), ct(3), ct(4))
    with pytest.raises(ValueError, match="lwe_add"):
        F.lwe_add(CTX, ct(4), ct(4), ct(5))
    c = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(ValueError, match="c must be"):
        F.lwe_add_plain(CTX, 32, ct(5), c, ct(5))
    with pytest.raises(ValueError, match="y must be"):
        F.lwe_add_plain(CTX, 32, ct(4), c, ct(3))


def test_other_bootstrapping_entry_points_check_shapes():
    with pytest.raises(ValueError):
        F.pbs(CTX, DK, [1] * 16 + [-1] * 16, ct(4), ct(4, WZ), keyswitch=True)
    with pytest.raises(ValueError):
        F.pbs_lif_many_lut(CTX, DK, 4, 2, ct(4), ct(4), ct(3))
    with pytest.raises(ValueError):
        F.pbs_lif_ks_first(CTX, DK, 4, 2, ct(4, WZ), ct(4, W1), ct(4, WZ))
    with pytest.raises(ValueError):
        F.pbs_lif_ranges(CTX, 4, 2, [(DK, ct(4), ct(4), ct(5))])


def test_ntt_polymul_shapes():
    d = torch.zeros((2, 1024), dtype=torch.int32)
    with pytest.raises(ValueError, match="b must be"):
        F.ntt_polymul(CTX, 1024, 64, d, torch.zeros((1, 1024), dtype=torch.int32),
                      torch.zeros(1024, dtype=torch.int32))
    with pytest.raises(ValueError, match="out must be"):
        F.ntt_polymul(CTX, 1024, 64, d, d, torch.zeros(512, dtype=torch.int32))
