"""Seeded synthetic inputs shared by the tests, the bench and the oracle's network runs.

This module holds none of the method's arithmetic: it only draws plaintext
messages, integer weights, spike patterns and images with numpy's PCG64, so
that the HIP path and the oracle can be fed the same plaintext data.  Keys,
encryption randomness and noise are drawn by each side from its own
counter-based generator, not here.

Seeds used throughout: keys 1, encryptions 2, data and weights 3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_KEYS = 1
SEED_ENC = 2
SEED_DATA = 3


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def messages(seed: int, count: int, p: int, stream: int = 0) -> np.ndarray:
    """Messages uniform in Z_p = {-p/2+1, ..., p/2}."""
    return rng(seed, stream).integers(-p // 2 + 1, p // 2 + 1, size=count, dtype=np.int64).astype(np.int32)


def uniform_int(seed: int, shape, lo: int, hi: int, stream: int = 0) -> np.ndarray:
    """Integers uniform in [lo, hi] (both ends included)."""
    return rng(seed, stream).integers(lo, hi + 1, size=shape, dtype=np.int64).astype(np.int32)


def image_like_digit(seed: int, stream: int = 0, size: int = 28) -> np.ndarray:
    """A 28x28 uint8 image with the shape and value statistics of a
    handwritten-digit scan: black background, 1-3 anti-aliased strokes
    2-3 px wide at intensity 128-255, about a fifth of the pixels non-zero."""
    g = rng(seed, 1000 + stream)
    img = np.zeros((size, size), np.float64)
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    for _ in range(int(g.integers(1, 4))):
        # a quadratic Bezier stroke inside the central 20x20 box
        pts = g.uniform(4, size - 4, size=(3, 2))
        width = g.uniform(1.0, 1.5)
        level = g.uniform(128, 255)
        for tt in np.linspace(0, 1, 40):
            c = (1 - tt) ** 2 * pts[0] + 2 * (1 - tt) * tt * pts[1] + tt ** 2 * pts[2]
            d = np.hypot(yy - c[0], xx - c[1])
            img = np.maximum(img, level * np.clip(width + 0.5 - d, 0, 1))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def quantise_pixels(img: np.ndarray) -> np.ndarray:
    """Pixels to 4-bit messages: q = pixel >> 4 in [0, 15]."""
    return (img.astype(np.int32) >> 4).reshape(-1)


# ------------------------------------------------------------------ workloads

@dataclass(frozen=True)
class TinyLIF:
    """Tiny encrypted LIF layer: 64 inputs with 3-bit values, weights in
    [-8, 8], 32 LIF neurons (threshold 4, leak tau 2, reset 0), T = 2."""
    inputs: int = 64
    neurons: int = 32
    w_lo: int = -8
    w_hi: int = 8
    x_max: int = 7
    vth: int = 4
    tau: int = 2
    T: int = 2

    def data(self, seed: int = SEED_DATA):
        x = uniform_int(seed, self.inputs, 0, self.x_max, stream=1)
        W = uniform_int(seed, (self.neurons, self.inputs), self.w_lo, self.w_hi, stream=2)
        return x, W


@dataclass(frozen=True)
class ConvSNN:
    """Conv SNN on one image: conv Ci->Co KxK stride s pad pd (LIF) ->
    FC (LIF) -> FC accumulators, weights in [-15, 15], T steps."""
    H: int = 28
    Wd: int = 28
    Ci: int = 1
    Co: int = 8
    K: int = 5
    stride: int = 2
    pad: int = 2
    hidden: int = 256
    classes: int = 10
    w_lo: int = -15
    w_hi: int = 15
    vth: int = 4
    tau: int = 2
    T: int = 4

    @property
    def Ho(self):
        return (self.H + 2 * self.pad - self.K) // self.stride + 1

    @property
    def Wo(self):
        return (self.Wd + 2 * self.pad - self.K) // self.stride + 1

    @property
    def l1(self):
        return self.Co * self.Ho * self.Wo

    def pbs_count(self) -> int:
        """Two bootstrappings per LIF neuron per step."""
        return 2 * (self.l1 + self.hidden) * self.T

    def data(self, seed: int = SEED_DATA, image_stream: int = 0):
        if self.H == 28 and self.Wd == 28:
            px = quantise_pixels(image_like_digit(seed, image_stream))
        else:
            px = uniform_int(seed, self.Ci * self.H * self.Wd, 0, 15, stream=10 + image_stream)
        Wc = uniform_int(seed, (self.Co, self.Ci, self.K, self.K), self.w_lo, self.w_hi, stream=3)
        W1 = uniform_int(seed, (self.hidden, self.l1), self.w_lo, self.w_hi, stream=4)
        W2 = uniform_int(seed, (self.classes, self.hidden), self.w_lo, self.w_hi, stream=5)
        return px, Wc, W1, W2


CONV_SNN = ConvSNN()
# a small instance of the same topology the oracle can run end to end
CONV_SNN_MINI = ConvSNN(H=8, Wd=8, Co=2, K=3, stride=2, pad=1, hidden=8, classes=4, T=2)


@dataclass(frozen=True)
class PaperCSNN:
    """The CSNN of the paper (Sec. 3.1): conv Ci->Co KxK stride s pad pd
    (LIF) -> average pool PxP -> FC (LIF) -> FC (LIF), the output layer's
    spikes counted as scores; synthetic integer weights in [w_lo, w_hi]."""
    H: int = 28
    Wd: int = 28
    Ci: int = 1
    Co: int = 10
    K: int = 8
    stride: int = 2
    pad: int = 1
    pool: int = 2
    hidden: int = 160
    classes: int = 10
    w_lo: int = -8
    w_hi: int = 8
    vth: int = 4
    tau: int = 2
    T: int = 4

    @property
    def Ho(self):
        return (self.H + 2 * self.pad - self.K) // self.stride + 1

    @property
    def Wo(self):
        return (self.Wd + 2 * self.pad - self.K) // self.stride + 1

    @property
    def l1(self):
        return self.Co * self.Ho * self.Wo

    @property
    def pooled(self):
        return self.Co * (self.Ho // self.pool) * (self.Wo // self.pool)

    def pbs_count(self) -> int:
        """Two bootstrappings per LIF neuron per step (all three layers)."""
        return 2 * (self.l1 + self.hidden + self.classes) * self.T

    def data(self, seed: int = SEED_DATA, image_stream: int = 0):
        if self.H == 28 and self.Wd == 28:
            px = quantise_pixels(image_like_digit(seed, image_stream))
        else:
            px = uniform_int(seed, self.Ci * self.H * self.Wd, 0, 15, stream=20 + image_stream)
        Wc = uniform_int(seed, (self.Co, self.Ci, self.K, self.K), self.w_lo, self.w_hi, stream=13)
        W1 = uniform_int(seed, (self.hidden, self.pooled), self.w_lo, self.w_hi, stream=14)
        W2 = uniform_int(seed, (self.classes, self.hidden), self.w_lo, self.w_hi, stream=15)
        return px, Wc, W1, W2


PAPER_CSNN = PaperCSNN()
# the same topology at a size the oracle runs end to end
PAPER_CSNN_MINI = PaperCSNN(H=8, Wd=8, Co=2, K=4, stride=2, pad=1, hidden=6, classes=3, T=2)


@dataclass(frozen=True)
class PoissonSNN:
    """The paper's Poisson-encoded SNN (Sec. 2.3 Poisson coding; Sec. 5.1,
    Table 1): every step each pixel spikes when it exceeds a fresh uniform
    threshold, then FC (LIF) -> FC (LIF) with the output spikes counted.
    Pixels are 4-bit (q = pixel >> 4) and the thresholds m_t uniform in
    [0, 15] on the same scale; weights in [w_lo, w_hi]."""
    H: int = 28
    Wd: int = 28
    hidden: int = 160
    classes: int = 10
    w_lo: int = -8
    w_hi: int = 8
    vth: int = 4
    tau: int = 2
    T: int = 20

    @property
    def pixels(self):
        return self.H * self.Wd

    def pbs_count(self) -> int:
        """One Sign bootstrapping per pixel and two per LIF neuron, per step."""
        return (self.pixels + 2 * self.hidden + 2 * self.classes) * self.T

    def data(self, seed: int = SEED_DATA, image_stream: int = 0):
        if self.H == 28 and self.Wd == 28:
            px = quantise_pixels(image_like_digit(seed, image_stream))
        else:
            px = uniform_int(seed, self.pixels, 0, 15, stream=30 + image_stream)
        W1 = uniform_int(seed, (self.hidden, self.pixels), self.w_lo, self.w_hi, stream=16)
        W2 = uniform_int(seed, (self.classes, self.hidden), self.w_lo, self.w_hi, stream=17)
        return px, W1, W2

    def thresholds(self, seed: int = SEED_DATA, image_stream: int = 0):
        """The uniform matrices M_t of Poisson coding, [T][pixels] in [0, 15]."""
        return uniform_int(seed, (self.T, self.pixels), 0, 15, stream=40 + image_stream)


POISSON_SNN = PoissonSNN()
# a small instance the oracle runs end to end
POISSON_SNN_MINI = PoissonSNN(H=4, Wd=4, hidden=5, classes=3, T=3)


def uneven_batch(seed: int = SEED_DATA, images: int = 64):
    """Per-image timestep counts in {2..8} and hidden widths in {256, 800}."""
    g = rng(seed, 77)
    T = g.integers(2, 9, size=images)
    H = np.where(g.integers(0, 2, size=images) == 0, 256, 800)
    return T.astype(np.int32), H.astype(np.int32)
