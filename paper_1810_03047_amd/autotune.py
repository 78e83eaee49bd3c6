"""Launch-shape autotuner for the trajectory kernels.

* ``pick_team_waves``: the small-dimension dense kernel offers several team shapes
  for one d (how many wavefronts share the row tiles of the real-embedded H_eff);
  which one is fastest depends on d, the operator's tile pattern (banded operators
  have their own single-wave instance), the product precision, the form and the
  number of trajectories.
* ``pick_batch_waves``: the batched launch of a heterogeneous batch runs one
  persistent launch per tile class (d <= 64, 128, 256), each with a team shape
  chosen among those the library offers for the class, or on the sliced-ELL SpMM
  kernel; every class with at least two systems is timed on its own systems.

Every candidate is timed on the workload itself (one warm-up run and ``reps``
timed runs, the trajectory kernel's device time as the library measures it) and
the fastest is kept.  Results are memoised per process and, when ``cache_path``
is given, in a JSON file.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import hashlib

import numpy as np

from . import Opts, batch_tile_candidates, create_batch, create_system, tile_candidates, tile_class

_memo: Dict[str, dict] = {}


def _pattern(system) -> str:
    """Digest of the nonzero pattern of H and of the C_n^dag C_n (the pattern of M, which
    decides whether the banded instance applies)."""
    P = system.H.to_dense() != 0
    for c in system.c_ops:
        C = c.to_dense()
        P = P | ((C.conj().T @ C) != 0)
    return hashlib.sha1(np.packbits(P).tobytes()).hexdigest()[:12]


def _key(system, opts: Opts, device_name: str, ntraj: int) -> str:
    return (f"{device_name}|d={system.dim}|nc={len(system.c_ops)}|prec={opts.precision}|form={opts.form}"
            f"|ntraj={ntraj}|pattern={_pattern(system)}")


def _load(cache_path, key):
    if key in _memo:
        return _memo[key]
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            disk = json.load(f)
        if key in disk:
            _memo[key] = disk[key]
            return disk[key]
    return None


def _store(cache_path, key, res):
    _memo[key] = res
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                disk = json.load(f)
        disk[key] = res
        with open(cache_path, "w") as f:
            json.dump(disk, f, indent=1)


def pick_team_waves(system, opts: Opts, ntraj: int, seed: int = 0x5EED, reps: int = 2,
                    cache_path: Optional[str] = None, proposal=None, device_name: str = "gfx950") -> dict:
    """Returns {"team_waves": w, "kernel_ms": {w: ms, ...}} for the fastest team shape.

    ``team_waves`` is 0 (the library's default) when the dimension offers no
    choice.  ``proposal`` = (params, f_ops) is installed for learned forms.
    """
    key = _key(system, opts, device_name, ntraj)
    hit = _load(cache_path, key)
    if hit is not None:
        return hit
    cands = tile_candidates(system.dim)
    if len(cands) <= 1:
        res = {"team_waves": 0, "kernel_ms": {}}
        _memo[key] = res
        return res
    times = {}
    for w in cands:
        o = Opts(**{**opts.__dict__, "team_waves": int(w)})
        ctx = create_system(system, o)
        if proposal is not None:
            ctx.set_proposal(*proposal)
        ctx.run(ntraj, seed)
        best = float("inf")
        for r in range(reps):
            ctx.run(ntraj, seed + 1 + r)
            best = min(best, ctx.stats()["kernel_ms"])
        ctx.destroy()
        times[int(w)] = best
    w_best = min(times, key=times.get)
    res = {"team_waves": w_best, "kernel_ms": times}
    _store(cache_path, key, res)
    return res


def pick_batch_waves(systems, opts: Opts, ntraj: int, seed: int = 0x5EED, reps: int = 2,
                     cache_path: Optional[str] = None, device_name: str = "gfx950") -> dict:
    """Returns {"class_waves": (w0, w1, w2), "kernel_ms": {class: {w: ms}}}: for every tile
    class of the batch with at least two systems, the fastest team shape on the class's
    own systems (batched form); 0 (the default) for the others."""
    waves, times = [0, 0, 0], {}
    for k in range(3):
        sub = [s for s in systems if tile_class(s.dim) == k]
        cands = batch_tile_candidates(k) + [-1]         # -1: the class on the SpMM kernel
        if len(sub) < 2:
            continue
        digest = hashlib.sha1("|".join(f"{s.dim}:{len(s.c_ops)}:{_pattern(s)}" for s in sub).encode()).hexdigest()[:12]
        key = f"{device_name}|batch-class={k}|systems={digest}|prec={opts.precision}|form={opts.form}|ntraj={ntraj}"
        hit = _load(cache_path, key)
        if hit is None:
            t = {}
            for w in cands:
                cw = [0, 0, 0]
                cw[k] = int(w)
                o = Opts(**{**opts.__dict__, "class_waves": tuple(cw)})
                ctx = create_batch(sub, o)
                ctx.run(ntraj, seed)
                best = float("inf")
                for r in range(reps):
                    ctx.run(ntraj, seed + 1 + r)
                    best = min(best, ctx.stats()["kernel_ms"])
                ctx.destroy()
                t[int(w)] = best
            hit = {"waves": min(t, key=t.get), "kernel_ms": t}
            _store(cache_path, key, hit)
        waves[k] = hit["waves"]
        times[k] = hit["kernel_ms"]
    return {"class_waves": tuple(waves), "kernel_ms": times}
