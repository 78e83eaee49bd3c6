"""Launch-shape autotuner for the trajectory kernels.

The small-dimension dense kernel offers several team shapes for one d (how
many wavefronts share the row tiles of the real-embedded H_eff); which one is
fastest depends on d, the product precision and the form.  ``pick_team_waves``
times every candidate on the workload itself (each candidate one warm-up run
and ``reps`` timed runs of the trajectory kernel, HIP-event timed inside the
library) and returns the fastest.  Results are memoised per process and, when
``cache_path`` is given, in a JSON file keyed by (device, d, precision, form).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

from . import Opts, create_system, tile_candidates

_memo: Dict[str, dict] = {}


def _key(system, opts: Opts, device_name: str) -> str:
    return f"{device_name}|d={system.dim}|nc={len(system.c_ops)}|prec={opts.precision}|form={opts.form}"


def pick_team_waves(system, opts: Opts, ntraj: int, seed: int = 0x5EED, reps: int = 2,
                    cache_path: Optional[str] = None, proposal=None, device_name: str = "gfx950") -> dict:
    """Returns {"team_waves": w, "kernel_ms": {w: ms, ...}} for the fastest team shape.

    ``team_waves`` is 0 (the library's default) when the dimension offers no
    choice.  ``proposal`` = (params, f_ops) is installed for learned forms.
    """
    key = _key(system, opts, device_name)
    if key in _memo:
        return _memo[key]
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            disk = json.load(f)
        if key in disk:
            _memo[key] = disk[key]
            return disk[key]
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
    _memo[key] = res
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                disk = json.load(f)
        disk[key] = res
        with open(cache_path, "w") as f:
            json.dump(disk, f, indent=1)
    return res
