"""Benchmark: trajectories/sec to t_end at rtol 1e-6 on one MI355X.

Workload (one "step" = one qtm_run of the whole hot path over one batch):
Jaynes-Cummings model, Fock cutoff 20 times a two-level atom (d = 40, dense),
g = 1, zero detuning, cavity decay 0.1, atomic decay 0.05, coherent state
alpha = 2 with the atom excited, t in [0, 50] with 501 output times, 10,000
trajectories, rtol 1e-6, atol 1e-8.  Inputs are synthetic and resident on the
device before timing starts.

Forms: "plain" (FP64 products, one block per 16 trajectories, starting-step
rule), and the headline "learned+batched+mixed" (FP32 MFMA products with FP64
state/norms/root finding/averages, persistent blocks with slot refill, and
the trained step proposal).  ``value`` is the headline form's throughput; the
plain form's is reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms plain,best]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trajectories/sec to t_end at rtol 1e-6; learned+batched form vs plain"
PEAK = {"fp64": 78.6, "fp32": 157.3}          # TFLOP/s, MI355X dense matrix peaks
NTRAJ = 10_000


def jcm_flops_per_step(d: int) -> float:
    # six products M w (8 d^2 real flops each, complex) + about 32 complex
    # axpy-type vector operations of 4 d flops (stage sums, error, norms)
    return 6 * 8.0 * d * d + 32 * 4.0 * d


def feature_ops(N: int = 20):
    """Diagonal feature operators of the proposal: atom excited, Fock n = 0..10."""
    import workloads as w
    d = 2 * N
    ops = [w.diag(np.tile([0.0, 1.0], N))]
    for n in range(11):
        v = np.zeros(d)
        v[2 * n:2 * n + 2] = 1.0
        ops.append(w.diag(v))
    return ops


def train_proposal(qtm, system, n_traj_data: int = 170_000, epochs: int = 8, seed: int = 1):
    """Trains the step proposal on segment records produced by the plain GPU solver."""
    f_ops = feature_ops()
    gen = qtm.create_system(system, qtm.Opts(seg_cap=16, form=qtm.FORM_BATCHED))
    feats, tgts = [], []
    chunk = 20_000
    done = 0
    while done < n_traj_data:
        cnt = min(chunk, n_traj_data - done)
        # feature operators must be installed for the records to carry them
        gen.set_proposal(_neutral_params(qtm), f_ops)
        gen.opts.form = qtm.FORM_BATCHED
        gen.run_range(done, cnt, seed)
        seg = gen.segments().reshape(-1, qtm.SEG_REC)
        seg = seg[(seg[:, 19] > 0) & (seg[:, 17] > 0)]
        feats.append(seg[:, :16])
        tau = np.where(seg[:, 18] > 0, 1.0, seg[:, 16])
        tgts.append(np.stack([np.log(seg[:, 17]), np.log(np.maximum(tau, 1e-12)), seg[:, 18]], 1))
        done += cnt
    gen.destroy()
    F = np.concatenate(feats).astype(np.float32)
    T = np.concatenate(tgts).astype(np.float32)
    return F, T, f_ops


def _neutral_params(qtm):
    p = np.zeros(qtm.MLP_NTOTAL, dtype=np.float32)
    p[-16:] = 1.0
    return p


def time_form(qtm, system, opts, steps, warmup, seed0=0, proposal=None):
    import torch
    ctx = qtm.create_system(system, opts)
    if proposal is not None:
        ctx.set_proposal(*proposal)
    for i in range(warmup):
        ctx.run(NTRAJ, seed0 + 1000 + i)
    torch.cuda.synchronize()
    kms, units, acc, rej, seg = [], 0, 0, 0, 0
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.run(NTRAJ, seed0 + i)
        st = ctx.stats()
        kms.append(st["kernel_ms"])
        units += st["accepted"] + st["rejected"]
        acc += st["accepted"]
        rej += st["rejected"]
        seg += st["segments"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean, var = ctx.expect()
    info = ctx.stats()
    ctx.destroy()
    return dict(wall=wall, kernel_ms=float(np.mean(kms)), steps_per_run=units / steps, acc=acc / steps,
                rej=rej / steps, segments=seg / steps, mean=mean, var=var, launch=info)


def cpu_baseline(system, target_s: float = 12.0):
    """The FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    oracle.run(system, 64, seed=0, nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(max(64, min(20000, 64 * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(system, n, seed=0, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "trajectories/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of the {NTRAJ} trajectories (same system, seed 0), FP64 C++ oracle, OpenMP"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="plain,best")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: trajectories are independent and the multi-GPU path "
              "(one all-reduce of the FP64 sums) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1810_03047_amd as qtm
    import workloads as w

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    system = w.jaynes_cummings()
    d = system.dim
    forms = a.forms.split(",")
    res = {}
    if "plain" in forms:
        res["plain"] = time_form(qtm, system, qtm.Opts(precision=qtm.PREC_FP64), a.steps, a.warmup)
    best_name = None
    if "best" in forms:
        proposal = None
        form = qtm.FORM_BATCHED
        if not a.no_learned:
            F, T, f_ops = train_proposal(qtm, system)
            trainer = qtm.create_system(system, qtm.Opts())
            trainer.train_proposal(F, T, epochs=8, batch=4096, lr=2e-3, seed=0)
            proposal = (trainer.get_proposal(), f_ops)
            trainer.destroy()
            form |= qtm.FORM_LEARNED
        res["best"] = time_form(qtm, system, qtm.Opts(precision=qtm.PREC_FP32, form=form), a.steps, a.warmup,
                                proposal=proposal)
        best_name = "learned+batched+mixed" if proposal is not None else "batched+mixed"
    head = res.get("best") or res["plain"]
    prec = "fp32" if "best" in res else "fp64"
    tps = NTRAJ * a.steps / head["wall"]
    flops = head["steps_per_run"] * jcm_flops_per_step(d)
    achieved = flops / (head["kernel_ms"] * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": tps, "unit": "trajectories/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["wall"] / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products, f64 state" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "jaynes_cummings N=20 x atom (d=40, dense), g=1, kappa=0.1, gamma=0.05, alpha=2, "
                               "t in [0,50] (501 points), rtol 1e-6, atol 1e-8",
                   "ntraj": NTRAJ, "form": best_name or "plain", "parallelism": "trajectories (1 GPU)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[prec], "traffic": None,
                     "kernel": "traj_dense_kernel", "kernel_ms": head["kernel_ms"],
                     "flop_per_traj_step": jcm_flops_per_step(d), "traj_steps_per_launch": head["steps_per_run"]},
    }
    if "plain" in res and "best" in res:
        p = res["plain"]
        line["plain"] = {"value": NTRAJ * a.steps / p["wall"], "kernel_ms": p["kernel_ms"],
                         "traj_steps_per_launch": p["steps_per_run"],
                         "tflops": p["steps_per_run"] * jcm_flops_per_step(d) / (p["kernel_ms"] * 1e-3) / 1e12}
        line["speedup_vs_plain"] = line["value"] / line["plain"]["value"]
        line["steps_per_traj"] = {"plain": p["steps_per_run"] / NTRAJ, "best": head["steps_per_run"] / NTRAJ}
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(system)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
