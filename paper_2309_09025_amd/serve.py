"""Serving loop: continuous batching of encrypted-image requests from several
clients (the deployment of Sec. 5.3: the client uploads its encrypted image
and evaluation key, the server evaluates the network and returns encrypted
scores).

* Every registered client's evaluation key stays resident in HBM.
* A request is admitted when it has arrived and its state buffers fit the
  device-memory budget, which the library keeps on the context
  (fs_ctx_admit: FS_EBUDGET when the admitted bytes would pass the budget or
  the device's free memory); it leaves when its last timestep is done,
  releasing its bytes for the next arrivals.  One server per context.
* One tick advances every in-flight request by one timestep.  Within a tick
  the LIF neurons of a layer of all in-flight requests, whatever their
  client, are bootstrapped by one fs_pbs_lif_ranges launch (each neuron with
  its own client's key), so requests that arrived at different times share
  the device; WeightSum layers run per request (own widths and weights).
* Latency = completion - arrival, on the host clock.
* A request's state between timesteps is its step counter, its LIF
  potentials and its score ciphertexts: `checkpoint` copies them to the host
  and frees the device memory, `resume` (on this or another server, after a
  restart) re-admits the request from them, and the rest of its run is
  byte-identical to an uninterrupted one.  `cancel` drops a request.

Every request's result is a deterministic function of its own inputs and
key: it is byte-identical alone and in any mix.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fhesnn as F
from .network import LifSpec, _zeros


@dataclass
class Request:
    rid: int
    client: int
    px_ct: np.ndarray      # host [Ci*H*Wd][n+1] encrypted pixels
    T: int
    hidden: int
    arrival: float = 0.0   # seconds after the start of the run
    done: float = 0.0
    score: np.ndarray = None
    # device state while in flight
    t: int = 0
    bufs: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.arrival


class Server:
    def __init__(self, ctx: F.Context, Wc, nets: dict, geom, lif: LifSpec = LifSpec(),
                 budget_bytes: int = 1 << 30):
        """nets: hidden width -> (W1 [H][l1], W2 [classes][H])."""
        self.ctx, self.lif = ctx, lif
        self.budget = budget_bytes
        self.Ci, self.H, self.Wd, self.stride, self.pad = geom
        Co, _, K, _ = Wc.shape
        Ho = (self.H + 2 * self.pad - K) // self.stride + 1
        Wo = (self.Wd + 2 * self.pad - K) // self.stride + 1
        self.l1 = Co * Ho * Wo
        self.Wc = F.to_device(np.ascontiguousarray(Wc, np.int32))
        self.nets = {h: (F.to_device(np.ascontiguousarray(a, np.int32)),
                         F.to_device(np.ascontiguousarray(b, np.int32))) for h, (a, b) in nets.items()}
        self.classes = next(iter(nets.values()))[1].shape[0]
        self.keys = {}
        self.width = None
        self.pbs_count = 0
        self.ticks = 0

    @property
    def budget(self) -> int:
        """Device bytes admissible for in-flight requests (0: no budget)."""
        return self._budget

    @budget.setter
    def budget(self, nbytes: int):
        self._budget = int(nbytes)
        self.ctx.set_budget(self._budget)

    @property
    def mem_used(self) -> int:
        """Bytes of the requests admitted now."""
        return self.ctx.admission()[1]

    # ---------------------------------------------------------------- clients
    def register(self, client: int, evk: F.EvalKey) -> F.DevKey:
        dk = F.evk_upload(self.ctx, evk)
        self.keys[client] = dk
        self.width = dk.params.n + 1
        return dk

    def key_bytes(self) -> int:
        return sum(dk.nbytes for dk in self.keys.values())

    # ---------------------------------------------------------------- requests
    def request_bytes(self, hidden: int) -> int:
        rows = 4 * self.l1 + 3 * hidden + self.classes + self.Ci * self.H * self.Wd
        return rows * self.width * 4

    def _admit(self, r: Request):
        w = self.width
        b = {
            "px": F.to_device(r.px_ct),
            "I1": _zeros(self.l1, w), "H1": _zeros(self.l1, w), "V1": _zeros(self.l1, w),
            "S1": _zeros(self.l1, w), "H2": _zeros(r.hidden, w), "V2": _zeros(r.hidden, w),
            "S2": _zeros(r.hidden, w), "score": _zeros(self.classes, w),
        }
        F.lwe_conv2d(self.ctx, self.Wc, b["px"], b["I1"], self.Ci, self.H, self.Wd,
                     self.stride, self.pad)
        r.bufs = b
        r.t = 0

    # ---------------------------------------------------------------- state
    STATE_KEYS = ("V1", "V2", "score")

    def checkpoint(self, r: Request) -> dict:
        """Host copy of an in-flight request's state at a timestep boundary
        (the static conv current is recomputed from the pixels on resume);
        the request leaves the device."""
        torch.cuda.synchronize()
        state = {"t": r.t, "hidden": r.hidden, "client": r.client}
        state.update({k: F.to_host(r.bufs[k]) for k in self.STATE_KEYS})
        self.cancel(r)
        return state

    def resume(self, r: Request, state: dict):
        """Re-admit a request from a checkpoint taken on any server with the
        same networks and the client's key registered."""
        if (state["hidden"], state["client"]) != (r.hidden, r.client):
            raise ValueError("checkpoint of a different request")
        if not self.ctx.admit(self.request_bytes(r.hidden)):
            raise MemoryError("request does not fit the memory budget")
        self._admit(r)
        for k in self.STATE_KEYS:
            r.bufs[k].copy_(F.to_device(state[k]))
        r.t = int(state["t"])

    def cancel(self, r: Request):
        """Drop an in-flight request and free its device memory."""
        if r.bufs:
            r.bufs = {}
            self.ctx.release(self.request_bytes(r.hidden))

    def step(self, inflight):
        """One tick over the given in-flight requests (each advances one
        timestep); returns those that are now complete (their scores filled
        in and their memory freed)."""
        self._tick(inflight)
        torch.cuda.synchronize()
        done = []
        for r in inflight:
            r.t += 1
            if r.t >= r.T:
                self._retire(r, time.perf_counter())
                done.append(r)
        return done

    def admit(self, r: Request):
        """Admit a request now (budget permitting)."""
        if not self.ctx.admit(self.request_bytes(r.hidden)):
            raise MemoryError("request does not fit the memory budget")
        self._admit(r)

    def _retire(self, r: Request, now: float):
        r.score = F.to_host(r.bufs["score"])
        r.done = now
        r.bufs = {}
        self.ctx.release(self.request_bytes(r.hidden))

    def _tick(self, inflight):
        c, L = self.ctx, self.lif
        for r in inflight:
            b = r.bufs
            F.lwe_add(c, b["V1"], b["I1"], b["H1"])
        F.pbs_lif_ranges(c, L.v_th, L.tau,
                         [(self.keys[r.client], r.bufs["H1"], r.bufs["S1"], r.bufs["V1"])
                          for r in inflight])
        for r in inflight:
            b = r.bufs
            W1, _ = self.nets[r.hidden]
            F.lwe_linear(c, W1, b["S1"], b["H2"], add=b["V2"])
        F.pbs_lif_ranges(c, L.v_th, L.tau,
                         [(self.keys[r.client], r.bufs["H2"], r.bufs["S2"], r.bufs["V2"])
                          for r in inflight])
        for r in inflight:
            b = r.bufs
            _, W2 = self.nets[r.hidden]
            F.lwe_linear(c, W2, b["S2"], b["score"], add=b["score"])
            self.pbs_count += 2 * (self.l1 + r.hidden)
        self.ticks += 1

    def run(self, requests, log=None):
        """Serve requests (each with its arrival time, seconds after start).
        Returns them with done/score filled in."""
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        inflight = []
        t0 = time.perf_counter()
        max_req = max(self.request_bytes(h) for h in self.nets)
        if self.budget and max_req > self.budget:
            raise ValueError("budget smaller than one request")
        while pending or inflight:
            now = time.perf_counter() - t0
            # admission: arrived requests, in order, while the library admits
            # them (budget and free device memory)
            while pending and pending[0].arrival <= now and \
                    self.ctx.admit(self.request_bytes(pending[0].hidden)):
                r = pending.popleft()
                self._admit(r)
                inflight.append(r)
            if not inflight:
                wait = pending[0].arrival - now
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            self._tick(inflight)
            torch.cuda.synchronize()
            now = time.perf_counter() - t0
            still = []
            for r in inflight:
                r.t += 1
                if r.t >= r.T:
                    self._retire(r, now)
                else:
                    still.append(r)
            inflight = still
            if log is not None and self.ticks % 10 == 0:
                log(f"tick {self.ticks}: {len(inflight)} in flight, {len(pending)} waiting, "
                    f"{self.pbs_count} bootstrappings, t={now:.1f}s")
        return requests


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64([seed, 99]))
    return np.cumsum(g.exponential(1.0 / rate, size=n))


def latency_stats(reqs):
    lat = np.array([r.latency for r in reqs])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
