"""Shared fixtures.  `-m "not gpu"` tests run anywhere; `-m gpu` tests need a
HIP device and the built libfhesnn.so."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X) and libfhesnn.so")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")


@pytest.fixture(scope="session")
def okeys_a():
    """Oracle keys, shape A (N = 1024), seed 1."""
    return O.keygen(O.SHAPE_A, synth.SEED_KEYS)


@pytest.fixture(scope="session")
def okeys_a_quiet():
    """Oracle keys, shape A, seed 1, with every noise deviation set to 0.
    The only errors left are the roundings of the modulus switch (std
    2^-8.6 at the blind rotation's input, 6.2 sigma inside a message
    window), the gadget decomposition and the key switch (about 2^-12.9 at
    a bootstrapping's output), so a layer input summing dozens of
    bootstrapped spikes still decrypts to its plaintext value."""
    from dataclasses import replace
    P = replace(O.SHAPE_A, sigma_lwe=0.0, sigma_bsk=0.0, sigma_ksk=0.0)
    return O.keygen(P, synth.SEED_KEYS)


@pytest.fixture(scope="session")
def okeys_b():
    """Oracle keys, shape B (N = 2048), seed 1."""
    return O.keygen(O.SHAPE_B, synth.SEED_KEYS)


@pytest.fixture(scope="session")
def gpu_env():
    """Library keys uploaded to device 0, both shapes (lazily per shape)."""
    import torch
    from paper_2309_09025_amd import fhesnn as F
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    F.lib()
    ctx = F.Context(0)
    cache = {}

    def get(shape):
        if shape not in cache:
            P = F.params_default(shape)
            sk, evk = F.keygen(P, synth.SEED_KEYS)
            dk = F.evk_upload(ctx, evk)
            cache[shape] = (P, sk, evk, dk)
        return cache[shape]
    return ctx, get
