"""Autotuner for the blind-rotation kernel.

Every kernel variant computes the same bits; the tuner times each one on a
batch of the caller's shape (bootstrapping runtime does not depend on the
ciphertext contents, apart from the rare skipped step a~_i = 0, so uniform
random samples are representative) and keeps the fastest.  Results are
cached in tune_cache.json next to this file, keyed by
(GPU architecture, N, l, Bg, key form, batch bucket).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import fhesnn as F

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _bucket(jobs: int) -> int:
    """Batch sizes are tuned per power-of-two bucket."""
    b = 1
    while b < jobs:
        b *= 2
    return b


def _form(dk) -> str:
    """Cache-key suffix of the device key's form (the one-limb N = 2048 key
    runs other kernel instances)."""
    return "|one_limb" if getattr(dk, "form", 0) == F.FS_KEY_ONE_LIMB else ""


def _key(arch: str, P, jobs: int, form: str = "") -> str:
    return f"{arch}|N={P.N}|l={P.l}|bg={P.bg_bit}{form}|jobs={_bucket(jobs)}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _check_device(ctx: F.Context):
    """The timing buffers and stream are torch's current device's."""
    import torch
    if torch.cuda.current_device() != ctx.device:
        raise ValueError(f"tuning a context of device {ctx.device} needs it to be torch's "
                         f"current device (now {torch.cuda.current_device()})")


def arch_name(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tune_blind_rotation(ctx: F.Context, dk: F.DevKey, jobs: int, reps: int = 2,
                        use_cache: bool = True, store: bool = True):
    """Pick the fastest blind-rotation variant for `jobs` bootstrappings per
    launch; sets it on ctx and returns (variant, {variant: ms})."""
    import torch
    P = dk.params
    _check_device(ctx)
    key = _key(arch_name(ctx.device), P, jobs, _form(dk))
    cache = _load() if use_cache else {}
    if key in cache:
        best = int(cache[key]["variant"])
        ctx.set_br_variant(P.N, best)
        return best, {int(k): v for k, v in cache[key]["ms"].items()}
    g = np.random.Generator(np.random.PCG64(1234))
    x = F.to_device(g.integers(0, 2 ** 32, size=(jobs, P.n + 1), dtype=np.uint64).astype(np.uint32))
    ext = F.empty_ct(jobs, P.N + 1)
    lut = np.where(np.arange(P.p) < P.p // 2, 1, -1).astype(np.int32)
    stream = torch.cuda.current_stream()
    times = {}
    for v in range(F.br_variants(P.N)):
        ctx.set_br_variant(P.N, v)
        F.pbs(ctx, dk, lut, x, ext, keyswitch=False, stream=stream)  # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            F.pbs(ctx, dk, lut, x, ext, keyswitch=False, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times[v] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    ctx.set_br_variant(P.N, best)
    if store:
        cache = _load()
        cache[key] = {"variant": best, "ms": {str(k): round(t, 4) for k, t in times.items()}}
        _store(cache)
    return best, times


# Thread-group forms in the order the library checks their thresholds.
FORMS = ("rows", "paired", "two", "one")


def thresholds_from_best(best, cus: int):
    """Batch-size thresholds (rows_max, paired_max, split_max) from the best
    form of each interval ((k-1) CUs, k CUs], k = 1, 2, ...: the library
    tries the forms in FORMS order, so each threshold ends the leading run
    of intervals whose best form is that one or an earlier one."""
    limits = {}
    k = 0
    for form in FORMS[:-1]:
        while k < len(best) and FORMS.index(best[k]) <= FORMS.index(form):
            k += 1
        limits[form] = k * cus
    return limits["rows"], limits["paired"], limits["two"]


def tune_groups(ctx: F.Context, dk: F.DevKey, intervals: int = 4, reps: int = 2,
                use_cache: bool = True, store: bool = True):
    """Time every thread-group form at k x CUs jobs (the largest batch of
    each interval; the forms' times are steps at multiples of the CU count)
    for k = 1..intervals, set the resulting thresholds on ctx and return
    (thresholds, {jobs: {form: ms}}).  The paired form exists at N = 1024
    only (elsewhere it falls back to two groups and is skipped), the row form
    not for the one-limb N = 2048 key.  The thresholds are the context's for
    ring degree N, whatever the key form."""
    import torch
    P = dk.params
    _check_device(ctx)
    cus = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    key = f"{arch_name(ctx.device)}|N={P.N}|l={P.l}|bg={P.bg_bit}{_form(dk)}|groups|cus={cus}"
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]["best"]
        times = {int(j): v for j, v in cache[key]["ms"].items()}
    else:
        forms = FORMS if P.N == 1024 else tuple(f for f in FORMS if f != "paired")
        if _form(dk):  # the one-limb key has no row form (it runs two groups there)
            forms = tuple(f for f in forms if f != "rows")
        g = np.random.Generator(np.random.PCG64(4321))
        lut = np.where(np.arange(P.p) < P.p // 2, 1, -1).astype(np.int32)
        stream = torch.cuda.current_stream()
        times, best = {}, []
        for k in range(1, intervals + 1):
            jobs = k * cus
            x = F.to_device(g.integers(0, 2 ** 32, size=(jobs, P.n + 1),
                                       dtype=np.uint64).astype(np.uint32))
            ext = F.empty_ct(jobs, P.N + 1)
            times[jobs] = {}
            for form in forms:
                with ctx.groups(form, P.N):
                    F.pbs(ctx, dk, lut, x, ext, keyswitch=False, stream=stream)  # warm
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        F.pbs(ctx, dk, lut, x, ext, keyswitch=False, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                times[jobs][form] = round(e0.elapsed_time(e1) / reps, 4)
            best.append(min(times[jobs], key=times[jobs].get))
        if store:
            cache = _load()
            cache[key] = {"best": best, "ms": {str(j): v for j, v in times.items()}}
            _store(cache)
    rows, paired, split = thresholds_from_best(best, cus)
    ctx.set_rows(P.N, rows)  # this ring degree's only: the other keeps its own
    ctx.set_paired(P.N, paired)
    ctx.set_split(P.N, split)
    return (rows, paired, split), times
