"""Encrypted LIF networks driven through the C ABI.

The recurrence is that of Theorem 3.1 (Eq. DiscretEquation) on ciphertexts:
    H[t] = V[t-1] + I[t]                    (fs_lwe_add / fs_lwe_linear epilogue)
    2S[t] = FHE-Fire(H[t]) + 1              (fs_pbs_lif, Eq. FHE-Fire)
    V[t]  = FHE-Reset(H[t])                 (fs_pbs_lif, Eq. FHE-Reset)
with WeightSum layers between LIF layers (Sec. 4.1) and score accumulators at
the output (the encrypted scores summed over the T steps, Sec. 5.3
procedure).  V[0] is the all-zero ciphertext and a static encrypted image
gives the first layer's current once.

All state lives in preallocated device buffers, so one timestep can be
captured in a HIP graph (torch.cuda.CUDAGraph) and replayed T times; every
kernel in the step is one of the library's.
"""
from __future__ import annotations

import contextlib
import gc
from dataclasses import dataclass

import numpy as np
import torch

from . import fhesnn as F


def _zeros(rows, width):
    return torch.zeros((rows, width), dtype=torch.int32, device="cuda")


@dataclass
class LifSpec:
    v_th: int = 4
    tau: int = 2


class StepGraph:
    """Runs `fn` eagerly once (so test polynomials and scratch are in place),
    then captures it into a HIP graph; `replay()` replays it.

    The cyclic garbage collector is held off while a capture is open: a
    network holding its own StepGraph (through the bound step method) is a
    reference cycle, and destroying its graph from inside another capture is
    an operation the runtime forbids during capture."""

    def __init__(self, fn, capture: bool):
        self.fn = fn
        self.graph = None
        self.capture = capture

    def run(self):
        if not self.capture:
            self.fn()
            return
        if self.graph is None:
            # the first step runs eagerly: it fills the caches the capture needs
            self.fn()
            torch.cuda.synchronize()
            self.graph = torch.cuda.CUDAGraph()
            self._pending = True
            return
        if self._pending:
            was_enabled = gc.isenabled()
            gc.disable()
            try:
                with torch.cuda.graph(self.graph):
                    self.fn()
            finally:
                if was_enabled:
                    gc.enable()
            self._pending = False
        self.graph.replay()


class LifLayerNet:
    """One LIF layer fed by a static current I = W x (the tiny LIF workload).

    ks_first: the key-switch-first order (fs_pbs_lif_ks_first); inputs and
    states are then ciphertexts under z, [.][N+1].  many_lut: Fire and Reset
    from one blind rotation (fs_pbs_lif_many_lut)."""

    def __init__(self, ctx, dk, W: np.ndarray, lif: LifSpec = LifSpec(), capture: bool = False,
                 ks_first: bool = False, many_lut: bool = False):
        self.ctx, self.dk, self.lif = ctx, dk, lif
        P = dk.params
        if ks_first and many_lut:
            raise ValueError("choose one of ks_first and many_lut")
        self.ks_first, self.many_lut = ks_first, many_lut
        self.width = (P.N if ks_first else P.n) + 1
        self.W = F.to_device(np.ascontiguousarray(W, np.int32))
        self.O = W.shape[0]
        self.I = _zeros(self.O, self.width)
        self.H = _zeros(self.O, self.width)
        self.V = _zeros(self.O, self.width)
        self.S = _zeros(self.O, self.width)
        self.capture = capture
        self.graph = None
        self.pbs_count = 0
        ctx.reserve(P.N, 2 * self.O)

    def _step(self):
        F.lwe_add(self.ctx, self.V, self.I, self.H)
        act = (F.pbs_lif_ks_first if self.ks_first else
               F.pbs_lif_many_lut if self.many_lut else F.pbs_lif)
        act(self.ctx, self.dk, self.lif.v_th, self.lif.tau, self.H, self.S, self.V)

    def run(self, x_ct: torch.Tensor, T: int, record: bool = True):
        """x_ct: device [inputs][width].  Returns per-step host copies (H, 2S, V)."""
        if x_ct.shape[1] != self.width:
            raise ValueError(f"inputs must be [inputs][{self.width}] ciphertexts")
        F.lwe_linear(self.ctx, self.W, x_ct, self.I)
        self.V.zero_()
        if self.graph is None:  # the step reads and writes the same buffers for every input
            self.graph = StepGraph(self._step, self.capture)
        out = []
        for _ in range(T):
            self.graph.run()
            self.pbs_count += 2 * self.O
            if record:
                torch.cuda.synchronize()
                out.append((F.to_host(self.H), F.to_host(self.S), F.to_host(self.V)))
        return out


class ConvSNN:
    """conv (LIF) -> FC (LIF) -> FC score accumulators on one encrypted image.
    many_lut: Fire and Reset from one blind rotation per neuron
    (fs_pbs_lif_many_lut)."""

    def __init__(self, ctx, dk, Wc, W1, W2, geom, lif: LifSpec = LifSpec(), capture: bool = False,
                 many_lut: bool = False):
        self.ctx, self.dk, self.lif = ctx, dk, lif
        self.act = F.pbs_lif_many_lut if many_lut else F.pbs_lif
        self.many_lut = many_lut
        P = dk.params
        self.width = P.n + 1
        self.Ci, self.H, self.Wd, self.stride, self.pad = geom
        Co, _, K, _ = Wc.shape
        self.Ho = (self.H + 2 * self.pad - K) // self.stride + 1
        self.Wo = (self.Wd + 2 * self.pad - K) // self.stride + 1
        self.l1 = Co * self.Ho * self.Wo
        self.hidden = W1.shape[0]
        self.classes = W2.shape[0]
        self.Wc = F.to_device(np.ascontiguousarray(Wc, np.int32))
        self.W1 = F.to_device(np.ascontiguousarray(W1, np.int32))
        self.W2 = F.to_device(np.ascontiguousarray(W2, np.int32))
        w = self.width
        self.I1, self.H1, self.V1, self.S1 = (_zeros(self.l1, w) for _ in range(4))
        self.H2, self.V2, self.S2 = (_zeros(self.hidden, w) for _ in range(3))
        self.score = _zeros(self.classes, w)
        self.capture = capture
        self.graph = None
        self.pbs_count = 0
        ctx.reserve(P.N, 2 * max(self.l1, self.hidden))

    def _step(self):
        c, dk, L = self.ctx, self.dk, self.lif
        F.lwe_add(c, self.V1, self.I1, self.H1)
        self.act(c, dk, L.v_th, L.tau, self.H1, self.S1, self.V1)
        F.lwe_linear(c, self.W1, self.S1, self.H2, add=self.V2)
        self.act(c, dk, L.v_th, L.tau, self.H2, self.S2, self.V2)
        F.lwe_linear(c, self.W2, self.S2, self.score, add=self.score)

    def run(self, px_ct: torch.Tensor, T: int, record: bool = False):
        """px_ct: device [Ci*H*Wd][n+1].  Returns the score ciphertexts (host)
        and, if record, per-step host copies of every state buffer."""
        F.lwe_conv2d(self.ctx, self.Wc, px_ct, self.I1, self.Ci, self.H, self.Wd,
                     self.stride, self.pad)
        for b in (self.V1, self.V2, self.score):
            b.zero_()
        if self.graph is None:  # the step reads and writes the same buffers for every image
            self.graph = StepGraph(self._step, self.capture)
        steps = []
        for _ in range(T):
            self.graph.run()
            self.pbs_count += 2 * (self.l1 + self.hidden)
            if record:
                torch.cuda.synchronize()
                steps.append({k: F.to_host(getattr(self, k)) for k in
                              ("H1", "S1", "V1", "H2", "S2", "V2", "score")})
        torch.cuda.synchronize()
        return F.to_host(self.score), steps

    def run_pipelined(self, px_ct: torch.Tensor, T: int, record: bool = False):
        """run() with the two LIF layers software-pipelined over time: layer 1
        at step t+1 depends only on its own state and the static current, so
        it is bootstrapped in the same launch (fs_pbs_lif_ranges) as layer 2
        at step t.  T + 1 launches instead of 2T, fewer partly filled rounds
        for one image; the results are bit-identical to run()."""
        c, dk, L = self.ctx, self.dk, self.lif
        F.lwe_conv2d(c, self.Wc, px_ct, self.I1, self.Ci, self.H, self.Wd, self.stride,
                     self.pad)
        for b in (self.V1, self.V2, self.score):
            b.zero_()
        steps = [{} for _ in range(T)] if record else []
        for k in range(T + 1):
            jobs = []
            if k >= 1:  # layer 2 at step k-1 reads S1 before this launch overwrites it
                F.lwe_linear(c, self.W1, self.S1, self.H2, add=self.V2)
                jobs.append((dk, self.H2, self.S2, self.V2))
            if k < T:
                F.lwe_add(c, self.V1, self.I1, self.H1)
                jobs.append((dk, self.H1, self.S1, self.V1))
            F.pbs_lif_ranges(c, L.v_th, L.tau, jobs, many_lut=self.many_lut)
            self.pbs_count += sum(2 * j[1].shape[0] for j in jobs)
            if k >= 1:
                F.lwe_linear(c, self.W2, self.S2, self.score, add=self.score)
            if record:
                torch.cuda.synchronize()
                if k < T:
                    steps[k].update({n: F.to_host(getattr(self, n)) for n in ("H1", "S1", "V1")})
                if k >= 1:
                    steps[k - 1].update({n: F.to_host(getattr(self, n))
                                         for n in ("H2", "S2", "V2", "score")})
        torch.cuda.synchronize()
        return F.to_host(self.score), steps


def fold_avg_pool(W1: np.ndarray, C: int, H: int, W: int, k: int) -> np.ndarray:
    """Weights of an FC layer over a k x k sum pool, moved onto the unpooled
    grid (Sec. 3.3: the pool's division goes into the next layer's weight
    scale, so the layer multiplies window sums of spikes): returns
    [O][C*H*W] with W1f[o][c, y, x] = W1[o][c, y // k, x // k] (zero for rows
    and columns the pool does not cover).  A product with W1f is then exactly
    the product of W1 with the window sums."""
    O_, _ = W1.shape
    Hp, Wp = H // k, W // k
    W1 = np.asarray(W1, np.int32).reshape(O_, C, Hp, Wp)
    Wf = np.zeros((O_, C, H, W), np.int32)
    Wf[:, :, : k * Hp, : k * Wp] = np.repeat(np.repeat(W1, k, axis=2), k, axis=3)
    return Wf.reshape(O_, C * H * W)


class PaperCSNN:
    """The paper's CSNN on one encrypted image (Sec. 3.1): conv (LIF) ->
    average pool -> FC (LIF) -> FC (LIF) with the output layer's spikes
    counted as scores.  The pool is folded into FC1's weights
    (fold_avg_pool), so a timestep is the same five library calls as
    ConvSNN's plus the output layer; each timestep is one HIP graph."""

    def __init__(self, ctx, dk, Wc, W1, W2, geom, pool: int = 2, lif: LifSpec = LifSpec(),
                 capture: bool = True, many_lut: bool = False):
        self.ctx, self.dk, self.lif = ctx, dk, lif
        self.many_lut = many_lut  # Fire and Reset from one blind rotation per neuron
        self.act = F.pbs_lif_many_lut if many_lut else F.pbs_lif
        P = dk.params
        self.width = w = P.n + 1
        self.Ci, self.H, self.Wd, self.stride, self.pad = geom
        Co, _, K, _ = Wc.shape
        Ho = (self.H + 2 * self.pad - K) // self.stride + 1
        Wo = (self.Wd + 2 * self.pad - K) // self.stride + 1
        self.l1 = Co * Ho * Wo
        self.hidden, self.classes = W1.shape[0], W2.shape[0]
        self.Wc = F.to_device(np.ascontiguousarray(Wc, np.int32))
        self.W1 = F.to_device(fold_avg_pool(W1, Co, Ho, Wo, pool))
        self.W2 = F.to_device(np.ascontiguousarray(W2, np.int32))
        self.I1, self.H1, self.V1, self.S1 = (_zeros(self.l1, w) for _ in range(4))
        self.H2, self.V2, self.S2 = (_zeros(self.hidden, w) for _ in range(3))
        self.H3, self.V3, self.S3 = (_zeros(self.classes, w) for _ in range(3))
        self.score = _zeros(self.classes, w)
        self.capture = capture
        self.graph = None
        self.pbs_count = 0
        ctx.reserve(P.N, 2 * max(self.l1, self.hidden))

    def _step(self):
        c, dk, L = self.ctx, self.dk, self.lif
        F.lwe_add(c, self.V1, self.I1, self.H1)
        self.act(c, dk, L.v_th, L.tau, self.H1, self.S1, self.V1)
        F.lwe_linear(c, self.W1, self.S1, self.H2, add=self.V2)
        self.act(c, dk, L.v_th, L.tau, self.H2, self.S2, self.V2)
        F.lwe_linear(c, self.W2, self.S2, self.H3, add=self.V3)
        self.act(c, dk, L.v_th, L.tau, self.H3, self.S3, self.V3)
        F.lwe_add(c, self.score, self.S3, self.score)

    def run(self, px_ct, T: int, record: bool = False):
        """Returns the encrypted spike counts (host) and, if record,
        per-step host copies of every state buffer."""
        F.lwe_conv2d(self.ctx, self.Wc, px_ct, self.I1, self.Ci, self.H, self.Wd,
                     self.stride, self.pad)
        for b in (self.V1, self.V2, self.V3, self.score):
            b.zero_()
        if self.graph is None:
            self.graph = StepGraph(self._step, self.capture)
        steps = []
        for _ in range(T):
            self.graph.run()
            self.pbs_count += 2 * (self.l1 + self.hidden + self.classes)
            if record:
                torch.cuda.synchronize()
                steps.append({k: F.to_host(getattr(self, k)) for k in
                              ("H1", "S1", "V1", "H2", "S2", "V2", "H3", "S3", "V3", "score")})
        torch.cuda.synchronize()
        return F.to_host(self.score), steps

    def run_pipelined(self, px_ct, T: int, record: bool = False):
        """run() with the three LIF layers software-pipelined over time: wave
        k bootstraps layer 1 at step k, layer 2 at step k-1 and layer 3 at
        step k-2 in one launch (each layer's next step depends on its own
        state and the previous layer's spikes of the same step).  T + 2
        launches instead of 3T; bit-identical to run()."""
        c, dk, L = self.ctx, self.dk, self.lif
        F.lwe_conv2d(c, self.Wc, px_ct, self.I1, self.Ci, self.H, self.Wd, self.stride,
                     self.pad)
        for b in (self.V1, self.V2, self.V3, self.score):
            b.zero_()
        steps = [{} for _ in range(T)] if record else []
        for k in range(T + 2):
            jobs = []
            # inputs first, deepest layer first: each reads the previous
            # layer's spikes before this wave's launch overwrites them
            if 2 <= k:
                F.lwe_linear(c, self.W2, self.S2, self.H3, add=self.V3)
                jobs.append((dk, self.H3, self.S3, self.V3))
            if 1 <= k <= T:
                F.lwe_linear(c, self.W1, self.S1, self.H2, add=self.V2)
                jobs.append((dk, self.H2, self.S2, self.V2))
            if k < T:
                F.lwe_add(c, self.V1, self.I1, self.H1)
                jobs.append((dk, self.H1, self.S1, self.V1))
            F.pbs_lif_ranges(c, L.v_th, L.tau, jobs, many_lut=self.many_lut)
            self.pbs_count += sum(2 * j[1].shape[0] for j in jobs)
            if 2 <= k:
                F.lwe_add(c, self.score, self.S3, self.score)
            if record:
                torch.cuda.synchronize()
                for layer, t in ((1, k), (2, k - 1), (3, k - 2)):
                    if 0 <= t < T:
                        steps[t].update({f"{n}{layer}": F.to_host(getattr(self, f"{n}{layer}"))
                                         for n in ("H", "S", "V")})
                if 2 <= k:
                    steps[k - 2]["score"] = F.to_host(self.score)
        torch.cuda.synchronize()
        return F.to_host(self.score), steps


class PoissonSNN:
    """The paper's Poisson-encoded SNN on one encrypted 4-bit image (Sec. 2.3,
    Sec. 5.1): every step each pixel ciphertext LWE(q) gets the plaintext
    -m_t of that step's threshold matrix added and goes through the Fire
    function with threshold 1 (one Sign bootstrapping), +1 afterwards, which
    gives LWE(2 [q > m_t]); then FC (LIF) -> FC (LIF), output spikes counted.
    The thresholds are inputs (the server's public randomness).  Each
    timestep is one HIP graph; the step's threshold row is copied into a
    fixed buffer before the replay."""

    def __init__(self, ctx, dk, W1, W2, lif: LifSpec = LifSpec(), capture: bool = True,
                 many_lut: bool = False):
        self.ctx, self.dk, self.lif = ctx, dk, lif
        self.many_lut = many_lut  # the LIF layers read Fire and Reset from one rotation
        self.act = F.pbs_lif_many_lut if many_lut else F.pbs_lif
        P = dk.params
        self.p = P.p
        self.width = w = P.n + 1
        self.pixels = W1.shape[1]
        self.hidden, self.classes = W1.shape[0], W2.shape[0]
        self.W1 = F.to_device(np.ascontiguousarray(W1, np.int32))
        self.W2 = F.to_device(np.ascontiguousarray(W2, np.int32))
        self.fire1, _ = F.lif_luts(1, 0, P.p)  # +1 iff q - m_t >= 1
        self.px = _zeros(self.pixels, w)
        self.neg_thr = torch.zeros(self.pixels, dtype=torch.int32, device="cuda")
        self.ones = torch.ones(self.pixels, dtype=torch.int32, device="cuda")
        self.H0, self.S0 = _zeros(self.pixels, w), _zeros(self.pixels, w)
        self.H1, self.V1, self.S1 = (_zeros(self.hidden, w) for _ in range(3))
        self.H2, self.V2, self.S2 = (_zeros(self.classes, w) for _ in range(3))
        self.score = _zeros(self.classes, w)
        self.capture = capture
        self.graph = None
        self.pbs_count = 0
        ctx.reserve(P.N, max(self.pixels, 2 * self.hidden))

    def _step(self):
        c, dk, L = self.ctx, self.dk, self.lif
        F.lwe_add_plain(c, self.p, self.px, self.neg_thr, self.H0)
        F.pbs(c, dk, self.fire1, self.H0, self.S0, keyswitch=True)
        F.lwe_add_plain(c, self.p, self.S0, self.ones, self.S0)
        F.lwe_linear(c, self.W1, self.S0, self.H1, add=self.V1)
        self.act(c, dk, L.v_th, L.tau, self.H1, self.S1, self.V1)
        F.lwe_linear(c, self.W2, self.S1, self.H2, add=self.V2)
        self.act(c, dk, L.v_th, L.tau, self.H2, self.S2, self.V2)
        F.lwe_add(c, self.score, self.S2, self.score)

    def run(self, px_ct, thresholds, record: bool = False):
        """px_ct: device [pixels][n+1]; thresholds: host [T][pixels] in [0, p).
        Returns the encrypted spike counts (host) and, if record, per-step host
        copies of every state buffer."""
        T = len(thresholds)
        self.px.copy_(px_ct)
        neg = torch.from_numpy(-np.ascontiguousarray(thresholds, np.int32)).to("cuda")
        for b in (self.V1, self.V2, self.score):
            b.zero_()
        if self.graph is None:
            self.graph = StepGraph(self._step, self.capture)
        steps = []
        for t in range(T):
            self.neg_thr.copy_(neg[t])
            self.graph.run()
            self.pbs_count += self.pixels + 2 * (self.hidden + self.classes)
            if record:
                torch.cuda.synchronize()
                steps.append({k: F.to_host(getattr(self, k)) for k in
                              ("S0", "H1", "S1", "V1", "H2", "S2", "V2", "score")})
        torch.cuda.synchronize()
        return F.to_host(self.score), steps

    def run_pipelined(self, px_ct, thresholds, record: bool = False, side_ctx=None):
        """run() software-pipelined over time: wave k codes step k's pixel
        spikes (one Sign launch) and bootstraps layer 1 at step k-1 and layer
        2 at step k-2 together (one fs_pbs_lif_ranges launch).  2 launches
        per step instead of 3; bit-identical to run().  side_ctx: a second
        Context (its own scratch); the pixel coding then runs on a second
        stream, concurrently with the same wave's LIF launch, ordered by
        events against the reads and writes of S0."""
        c, dk, L = self.ctx, self.dk, self.lif
        T = len(thresholds)
        self.px.copy_(px_ct)
        neg = torch.from_numpy(-np.ascontiguousarray(thresholds, np.int32)).to("cuda")
        for b in (self.V1, self.V2, self.score):
            b.zero_()
        main = torch.cuda.current_stream()
        side = torch.cuda.Stream() if side_ctx is not None else main
        cs = side_ctx if side_ctx is not None else c
        sign_mode = None
        if side_ctx is not None:
            # beside the LIF launch (one wave per digit row, 76 KiB of LDS per
            # job) the coding runs best on two groups per job: measured 452 ms
            # per image against 560 ms with the one-group kernel it would
            # otherwise get at 784 jobs
            cus = torch.cuda.get_device_properties(px_ct.device).multi_processor_count
            if self.pixels <= 4 * cus:
                sign_mode = "two"
        steps = [{} for _ in range(T)] if record else []
        for k in range(T + 2):
            jobs = []
            if 2 <= k:  # layer 2 at step k-2 (reads S1 before it is overwritten)
                F.lwe_linear(c, self.W2, self.S1, self.H2, add=self.V2)
                jobs.append((dk, self.H2, self.S2, self.V2))
            if 1 <= k <= T:  # layer 1 at step k-1 (reads S0 before the coding below)
                F.lwe_linear(c, self.W1, self.S0, self.H1, add=self.V1)
                jobs.append((dk, self.H1, self.S1, self.V1))
            coded = None
            if k < T:
                if side is not main:
                    read = torch.cuda.Event()
                    read.record(main)  # S0 of step k-1 consumed; thresholds uploaded
                    side.wait_event(read)
                F.lwe_add_plain(cs, self.p, self.px, neg[k], self.H0, stream=side)
                with side_ctx.groups(sign_mode) if sign_mode else contextlib.nullcontext():
                    F.pbs(cs, dk, self.fire1, self.H0, self.S0, keyswitch=True, stream=side)
                F.lwe_add_plain(cs, self.p, self.S0, self.ones, self.S0, stream=side)
                self.pbs_count += self.pixels
                if side is not main:
                    coded = torch.cuda.Event()
                    coded.record(side)
            if jobs:
                F.pbs_lif_ranges(c, L.v_th, L.tau, jobs, stream=main, many_lut=self.many_lut)
                self.pbs_count += sum(2 * j[1].shape[0] for j in jobs)
            if 2 <= k:
                F.lwe_add(c, self.score, self.S2, self.score)
            if coded is not None:
                main.wait_event(coded)  # the next wave reads S0 of step k
            if record:
                torch.cuda.synchronize()
                if k < T:
                    steps[k]["S0"] = F.to_host(self.S0)
                for layer, t in ((1, k - 1), (2, k - 2)):
                    if 0 <= t < T:
                        steps[t].update({f"{n}{layer}": F.to_host(getattr(self, f"{n}{layer}"))
                                         for n in ("H", "S", "V")})
                if 2 <= k:
                    steps[k - 2]["score"] = F.to_host(self.score)
        torch.cuda.synchronize()
        return F.to_host(self.score), steps

    def run_coded_ahead(self, px_ct, thresholds, record: bool = False, chain_mode=None):
        """run() with the pixel coding of all T steps first: the thresholds
        are known before the image is processed and the coding reads only the
        image, so the T x pixels Sign bootstrappings form one batched launch.
        Then the LIF layers run software-pipelined (wave k bootstraps layer 1
        at step k and layer 2 at step k-1 in one fs_pbs_lif_ranges launch):
        T + 1 small launches on the critical path instead of 2 T.  Holds the
        coded spikes of every step (T x pixels ciphertexts); bit-identical to
        run().  chain_mode: thread-group form of the LIF launches (see
        Context.groups; None = chosen by batch size)."""
        c, dk, L = self.ctx, self.dk, self.lif
        T = len(thresholds)
        px = self.pixels
        neg = torch.from_numpy(-np.ascontiguousarray(thresholds, np.int32).reshape(-1)).to("cuda")
        for b in (self.V1, self.V2, self.score):
            b.zero_()
        H0 = px_ct.repeat(T, 1)  # row t * pixels + i: pixel i at step t
        S0 = torch.empty_like(H0)
        if T:
            F.lwe_add_plain(c, self.p, H0, neg, H0)
            F.pbs(c, dk, self.fire1, H0, S0, keyswitch=True)
            F.lwe_add_plain(c, self.p, S0, self.ones.repeat(T), S0)
            self.pbs_count += T * px
        steps = [{} for _ in range(T)] if record else []
        for k in range(T + 1 if T else 0):
            jobs = []
            if k >= 1:  # layer 2 at step k-1 reads S1 before layer 1 overwrites it
                F.lwe_linear(c, self.W2, self.S1, self.H2, add=self.V2)
                jobs.append((dk, self.H2, self.S2, self.V2))
            if k < T:
                F.lwe_linear(c, self.W1, S0[k * px:(k + 1) * px], self.H1, add=self.V1)
                jobs.append((dk, self.H1, self.S1, self.V1))
            with c.groups(chain_mode) if chain_mode else contextlib.nullcontext():
                F.pbs_lif_ranges(c, L.v_th, L.tau, jobs, many_lut=self.many_lut)
            self.pbs_count += sum(2 * j[1].shape[0] for j in jobs)
            if k >= 1:
                F.lwe_add(c, self.score, self.S2, self.score)
            if record:
                torch.cuda.synchronize()
                if k < T:
                    steps[k]["S0"] = F.to_host(S0[k * px:(k + 1) * px])
                    steps[k].update({f"{n}1": F.to_host(getattr(self, f"{n}1"))
                                     for n in ("H", "S", "V")})
                if k >= 1:
                    steps[k - 1].update({f"{n}2": F.to_host(getattr(self, f"{n}2"))
                                         for n in ("H", "S", "V")})
                    steps[k - 1]["score"] = F.to_host(self.score)
        torch.cuda.synchronize()
        return F.to_host(self.score), steps


def pbs_count_paper_csnn(T: int) -> int:
    """Bootstrappings per image of the paper's CSNN (Table 1): 2 per LIF
    neuron per step over the 10x12x12, 160 and 10 LIF neurons."""
    return (1440 * 2 + 2 * 160 + 2 * 10) * T


class UnevenBatch:
    """Many images, each with its own number of steps T_i and hidden width
    H_i (one network per width), evaluated together: per timestep one
    fs_pbs_lif launch bootstraps the first-layer neurons of every still
    active image and one more the hidden neurons of all of them.  Images are
    kept in descending T order so the active ones form a prefix of every
    buffer.  Each distinct active set is captured once as a HIP graph and
    replayed for as many steps as it lasts."""

    def __init__(self, ctx, dk, Wc, nets: dict, geom, lif: LifSpec = LifSpec(),
                 capture: bool = True, many_lut: bool = False):
        """nets: hidden width -> (W1 [H][l1], W2 [classes][H]); many_lut: Fire
        and Reset from one blind rotation per neuron."""
        self.ctx, self.dk, self.lif = ctx, dk, lif
        self.act = F.pbs_lif_many_lut if many_lut else F.pbs_lif
        P = dk.params
        self.width = P.n + 1
        self.Ci, self.Hh, self.Wd, self.stride, self.pad = geom
        Co, _, K, _ = Wc.shape
        Ho = (self.Hh + 2 * self.pad - K) // self.stride + 1
        Wo = (self.Wd + 2 * self.pad - K) // self.stride + 1
        self.l1 = Co * Ho * Wo
        self.Wc = F.to_device(np.ascontiguousarray(Wc, np.int32))
        self.nets = {h: (F.to_device(np.ascontiguousarray(a, np.int32)),
                         F.to_device(np.ascontiguousarray(b, np.int32))) for h, (a, b) in nets.items()}
        self.classes = next(iter(nets.values()))[1].shape[0]
        self.capture = capture
        self.pbs_count = 0

    def run(self, px_cts, Ts, Hs, record: bool = False):
        """px_cts: list of device [Ci*H*Wd][n+1]; returns host score
        ciphertexts per image (input order).  record: also return, per
        timestep, each active image's host copies of H1, S1, V1, H2, S2, V2
        and its score ({image index: {...}}), one step at a time."""
        ctx, w = self.ctx, self.width
        order = sorted(range(len(px_cts)), key=lambda i: (-Ts[i], i))
        B = len(order)
        Ts_s = [int(Ts[i]) for i in order]
        Hs_s = [int(Hs[i]) for i in order]
        off2 = np.concatenate([[0], np.cumsum(Hs_s)]).astype(int)
        l1 = self.l1
        I1, H1, V1, S1 = (_zeros(B * l1, w) for _ in range(4))
        H2, V2, S2 = (_zeros(int(off2[-1]), w) for _ in range(3))
        score = _zeros(B * self.classes, w)
        self.ctx.reserve(self.dk.params.N, 2 * max(B * l1, int(off2[-1])))
        for k, i in enumerate(order):
            F.lwe_conv2d(ctx, self.Wc, px_cts[i], I1[k * l1:(k + 1) * l1], self.Ci, self.Hh, self.Wd,
                         self.stride, self.pad)
        L = self.lif

        def make_step(active):
            n1 = active * l1
            n2 = int(off2[active])

            def step():
                F.lwe_add(ctx, V1[:n1], I1[:n1], H1[:n1])
                self.act(ctx, self.dk, L.v_th, L.tau, H1[:n1], S1[:n1], V1[:n1])
                for k in range(active):
                    W1, W2 = self.nets[Hs_s[k]]
                    a, b = int(off2[k]), int(off2[k + 1])
                    F.lwe_linear(ctx, W1, S1[k * l1:(k + 1) * l1], H2[a:b], add=V2[a:b])
                self.act(ctx, self.dk, L.v_th, L.tau, H2[:n2], S2[:n2], V2[:n2])
                for k in range(active):
                    W1, W2 = self.nets[Hs_s[k]]
                    a, b = int(off2[k]), int(off2[k + 1])
                    sc = score[k * self.classes:(k + 1) * self.classes]
                    F.lwe_linear(ctx, W2, S2[a:b], sc, add=sc)
            return step, 2 * (n1 + n2)

        def snapshot(active):
            rec = {}
            for k in range(active):
                a, b = int(off2[k]), int(off2[k + 1])
                r1 = slice(k * l1, (k + 1) * l1)
                rec[order[k]] = {"H1": F.to_host(H1[r1]), "S1": F.to_host(S1[r1]),
                                 "V1": F.to_host(V1[r1]), "H2": F.to_host(H2[a:b]),
                                 "S2": F.to_host(S2[a:b]), "V2": F.to_host(V2[a:b]),
                                 "score": F.to_host(score[k * self.classes:(k + 1) * self.classes])}
            return rec

        steps = []
        t = 0
        Tmax = Ts_s[0] if B else 0
        while t < Tmax:
            active = sum(1 for x in Ts_s if x > t)
            span = min(x for x in Ts_s if x > t) - t  # steps this active set lasts
            fn, count = make_step(active)
            g = StepGraph(fn, self.capture)
            for _ in range(span):
                g.run()
                self.pbs_count += count
                if record:
                    steps.append(snapshot(active))
            t += span
        torch.cuda.synchronize()
        host = F.to_host(score).reshape(B, self.classes, w)
        out = [None] * B
        for k, i in enumerate(order):
            out[i] = host[k]
        return (out, steps) if record else out
