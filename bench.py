"""Benchmark: trajectories/sec to t_end at rtol 1e-6 on one MI355X.

Workload (one "step" = one qtm_run of the whole hot path over one batch):
Jaynes-Cummings model, Fock cutoff 20 times a two-level atom (d = 40, dense),
g = 1, zero detuning, cavity decay 0.1, atomic decay 0.05, coherent state
alpha = 2 with the atom excited, t in [0, 50] with 501 output times, 10,000
trajectories, rtol 1e-6, atol 1e-8.  Inputs are synthetic and resident on the
device before timing starts.

The line also nests, under "secondary", the same measurement (plain FP64 form
against the batched FP32 form, roofline, CPU baseline and oracle check) for the
driven two-level atom (500 trajectories), the transverse-field Ising chain
(L = 10, d = 1024, CSR, 20,000 trajectories), the heterogeneous batch (64
systems, d 8..256, 500 trajectories each), the paper's trilinear Hamiltonian
(d = 512, CSR, 20,000 trajectories), and a stiff Jaynes-Cummings cavity (decay 40,
10,000 trajectories: adaptive DOPRI5 against the exact-propagator form).

Forms: "plain" (FP64 products, the starting-step rule at every segment start)
and the headline "learned+batched+mixed" (FP32 products with FP64 state,
norms, root finding and averages, persistent teams with slot refill, and the
step proposal trained on the device from segment records of the plain
solver).  Both run with the team shape picked by the autotuner.  ``value`` is
the headline form's throughput; the plain form's is reported beside it.

The roofline entry is for the trajectory kernel (traj_team_kernel): algorithmic
FLOPs = attempted steps x (6 complex products 8 d^2 + 32 vector operations 4 d),
divided by the kernel's time.  The Jaynes-Cummings operator is banded: the kernel
multiplies only the 13 of its 25 tiles that lie within one tile of the diagonal (the
others are zero), and executed_flop_per_traj_step and executed_tflops report that
executed work beside the algorithmic figure.  The time is the one the library takes
from device wall-clock stamps written on the launch stream just before and after the kernel (graph
capturable).  HIP events (torch.cuda.Event) on the same stream around each whole
run are reported beside it as run_event_ms (that span also holds the output
clearing, the averaging and the read-back of the sums).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms plain,best] [--no-secondary]
    python bench.py --workload two_level|tfim|hetero|trilinear|stiff     (one configuration alone)
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
# FP32 vector arithmetic without packed (two-wide) FP32 instructions, which this code is
# built without: 256 CUs x 4 SIMDs x 16 FMA lanes per clock x 2 flops x 2.4 GHz
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9 / 1e12       # 78.6 TFLOP/s
NTRAJ = 10_000


# HBM traffic of the headline kernel per launch from two rocprofv3 counter passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
# reads for a 256 MiB device copy (FETCH x 2.0, WRITE x 1.0).  Valid only for the kernel
# sources it was measured on: reported as null once their hash differs.
KERNEL_SOURCES = ["qtm_wave.hip", "qtm_wave_t5x1.hip", "qtm_body.h", "qtm_internal.h"]
TRAFFIC = {"sources_sha256": "d221f7ac68b89c57e8fe328568714a8cec06fc9d132e4deb344122372fe4dfbc",
           "fetch_kib": 1371.7, "write_kib": 162491.7, "fetch_scale": 2.0, "write_scale": 1.0}


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1810_03047_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    t = TRAFFIC
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_sha():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def jcm_flops_per_step(d: int) -> float:
    # six products M w (8 d^2 real flops each, complex) + about 32 complex
    # axpy-type vector operations of 4 d flops (stage sums, error, norms)
    return 6 * 8.0 * d * d + 32 * 4.0 * d


def jcm_executed_flops_per_step(system, single_wave: bool) -> float:
    """FLOPs the matrix cores execute per attempted step.  The team kernel works on
    16x16 real tiles (8x8 complex blocks of M = -iH - 1/2 sum C^dag C).  With
    single-wave teams and an operator whose nonzero blocks lie within one block of the
    diagonal, it multiplies only those 3 RT - 2 of the RT^2 tiles (the rest are zero)."""
    d = system.dim
    M = -1j * system.H.to_dense()
    for c in system.c_ops:
        C = c.to_dense()
        M = M - 0.5 * C.conj().T @ C
    rt = (2 * ((d + 7) // 8 * 8)) // 16
    r, c = np.nonzero(M)
    banded = bool(np.all(np.abs((r >> 3) - (c >> 3)) <= 1))
    tiles = 3 * rt - 2 if (single_wave and banded and rt in (4, 5)) else rt * rt
    return 6 * 8.0 * 64 * tiles + 32 * 4.0 * d


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


def _neutral_params(qtm):
    p = np.zeros(qtm.MLP_NTOTAL, dtype=np.float32)
    p[-16:] = 1.0
    return p


# Training trajectories use their own seed, disjoint from every timed seed (0 .. K-1)
# and warm-up seed (1000 + i), so the learned form is never timed on its training data.
TRAIN_SEED = 1_000_003


def training_data(qtm, system, n_traj_data: int = 170_000, seed: int = TRAIN_SEED):
    """Segment records of the plain FP64 GPU solver -> (features, targets).

    Targets: log of the controller's step after the segment's first accepted
    step, log of the realised jump delay and the censoring flag."""
    f_ops = feature_ops()
    gen = qtm.create_system(system, qtm.Opts(seg_cap=16, form=qtm.FORM_BATCHED))
    gen.set_proposal(_neutral_params(qtm), f_ops)      # installs the feature operators
    feats, tgts = [], []
    chunk, done = 20_000, 0
    while done < n_traj_data:
        cnt = min(chunk, n_traj_data - done)
        gen.run_range(done, cnt, seed)
        seg = gen.segments().reshape(-1, qtm.SEG_REC)
        seg = seg[(seg[:, 19] > 0) & (seg[:, 17] > 0)]
        feats.append(seg[:, :16])
        tau = np.where(seg[:, 18] > 0, 1.0, seg[:, 16])
        tgts.append(np.stack([np.log(seg[:, 17]), np.log(np.maximum(tau, 1e-12)), seg[:, 18]], 1))
        done += cnt
    gen.destroy()
    return np.concatenate(feats).astype(np.float32), np.concatenate(tgts).astype(np.float32), f_ops


def time_form(qtm, system, opts, steps, warmup, seed0=0, proposal=None):
    import torch
    ctx = qtm.create_system(system, opts)
    if proposal is not None:
        ctx.set_proposal(*proposal)
    for i in range(warmup):
        ctx.run(NTRAJ, seed0 + 1000 + i)
    kms, evms, units, acc, rej, seg = [], [], 0, 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        # HIP events on the launch stream (torch's current stream) around the whole run
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.run(NTRAJ, seed0 + i)
        e1.record()
        e1.synchronize()
        evms.append(e0.elapsed_time(e1))
        st = ctx.stats()
        kms.append(st["kernel_ms"])
        units += st["accepted"] + st["rejected"]
        acc += st["accepted"]
        rej += st["rejected"]
        seg += st["segments"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = ctx.stats()
    ctx.destroy()
    return dict(wall=wall, kernel_ms=float(np.mean(kms)), run_event_ms=float(np.mean(evms)), steps_per_run=units / steps, acc=acc / steps,
                rej=rej / steps, segments=seg / steps, launch=info)


def _threads():
    """Host threads for the oracle: the CPU share of this process (at most 16, the share a
    one-GPU machine grants a job), with nproc recorded beside it."""
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        share = os.cpu_count() or 1
    return min(16, share), os.cpu_count() or 1, share


def cpu_baseline(system, mlp=None, f_ops=None, cpu_s: float = 20.0):
    """The FP64 oracle on the host cores over a bounded sample of the workload (the
    headline form: with the proposal weights the GPU uses when ``mlp`` is given).
    Both builds of the oracle are timed (the parity build and the -O3 AVX2/FMA build)
    on all the threads this process may use, and the faster one single-threaded."""
    import oracle
    threads, nproc, share = _threads()
    kw = dict(mlp=mlp, f_ops=f_ops)
    t0 = time.perf_counter()
    oracle.run(system, 64, seed=0, nthreads=threads, **kw)
    dt = time.perf_counter() - t0
    # about cpu_s seconds of CPU work per build at this rate
    n = int(max(64, min(20000, 64 * cpu_s / max(dt * threads, 1e-3))))
    rates = {}
    for name, fast in (("parity_build_O2", False), ("timing_build_O3_avx2", True)):
        t0 = time.perf_counter()
        oracle.run(system, n, seed=0, nthreads=threads, fast=fast, **kw)
        rates[name] = n / (time.perf_counter() - t0)
    best = max(rates, key=rates.get)
    fast_best = best == "timing_build_O3_avx2"
    n1 = max(16, n // threads)
    t0 = time.perf_counter()
    oracle.run(system, n1, seed=0, nthreads=1, fast=fast_best, **kw)
    single = n1 / (time.perf_counter() - t0)
    return {"value": rates[best], "unit": "trajectories/s", "cores": threads, "kind": "oracle",
            "sample": f"trajectories 0..{n - 1} of the same workload (seed 0{', same proposal weights' if mlp is not None else ''}), "
                      f"FP64 C++ oracle, {threads} OpenMP threads (nproc {nproc}, affinity {share}); "
                      f"{best} is the faster build",
            "builds": rates, "nproc": nproc, "single_thread": {"value": single, "build": best, "sample": f"trajectories 0..{n1 - 1}"}}


def oracle_check(qtm, system, opts, proposal, ntraj, seed=0, plain_exact=False):
    """The headline form on trajectories 0..ntraj-1 of one timed seed against the FP64
    oracle (parity build) on the same trajectories and random streams: the largest
    deviation of the averages in units of the oracle's sigma/sqrt(N) (the stated bound is
    3 plus 1e-6/(sigma/sqrt(N))), the fraction of trajectories with the oracle's jump
    counts, and the largest jump-time difference among trajectories whose jump counts
    and channels agree."""
    import dataclasses
    import oracle
    o = dataclasses.replace(opts, record_jumps=32, keep_traj=0)
    ctx = qtm.create_system(system, o)
    if proposal is not None:
        ctx.set_proposal(*proposal)
    ctx.run(ntraj, seed)
    mean, _ = ctx.expect()
    jn = np.zeros(ntraj, dtype=np.int64)
    jt = np.zeros((ntraj, 32))
    jc = np.zeros((ntraj, 32), dtype=np.int32)
    for i in range(ntraj):
        t, c, cnt = ctx.jumps(i)
        jn[i], jt[i, :len(t)], jc[i, :len(c)] = cnt, t, c
    ctx.destroy()
    threads, _, _ = _threads()
    mlp = None
    if proposal is not None:
        mlp = _working_params(proposal[0])
    r = oracle.run(system, ntraj, seed=seed, nthreads=threads, jcap=32, mlp=mlp,
                   f_ops=proposal[1] if proposal is not None else None)
    sig = np.sqrt(np.maximum(r["var"], 0.0) / ntraj)
    dev = np.abs(mean.real - r["mean"].real)
    z = dev / np.maximum(sig, 1e-300)
    bound = 3.0 * sig + 1e-6
    same = jn == r["jump_counts"]
    jtd = 0.0
    for i in np.nonzero(same)[0]:
        m = int(min(jn[i], 32))
        if m and np.array_equal(jc[i, :m], r["jump_channels"][i, :m]):
            jtd = max(jtd, float(np.max(np.abs(jt[i, :m] - r["jump_times"][i, :m]))))
    return {"ntraj": ntraj, "seed": seed, "max_dev_over_sigma": float(np.max(np.where(sig > 0, z, 0.0))),
            "max_dev_over_bound": float(np.max(dev / bound)), "max_abs_dev": float(np.max(dev)),
            "identical_jump_counts": float(np.mean(same)), "max_jump_time_diff": jtd,
            "within_bound": bool(np.all(dev <= bound))}


def _working_params(p32):
    """The values the device computes with: BF16-rounded weight matrices (round to
    nearest even), FP32 biases and standardisation, as FP64 for the oracle."""
    p = np.asarray(p32, dtype=np.float32).copy()
    nf, nh, no = 16, 64, 3
    for a, n in ((0, nh * nf), (nh * nf + nh, nh * nh), (nh * nf + nh + nh * nh + nh, no * nh)):
        u = p[a:a + n].view(np.uint32).copy()
        u += np.uint32(0x7FFF) + ((u >> 16) & 1)
        u &= np.uint32(0xFFFF0000)
        p[a:a + n] = u.view(np.float32)
    return p.astype(np.float64)


def _nnz_M(system) -> int:
    """Stored entries of M = -i H - 1/2 sum C^dag C (the union of the patterns)."""
    M = (system.H.to_dense() != 0)
    for c in system.c_ops:
        C = c.to_dense()
        M = M | ((C.conj().T @ C) != 0)
    return int(M.sum())


def secondary_spec(name, qtm, w):
    """The other configurations: (systems, trajectories per system, label, kernel, roofline
    bound, peak in TFLOP/s or None, flop per trajectory-step of system s or None)."""
    if name == "two_level":
        s = [w.two_level()]
        return dict(systems=s, n=500, batch=False, kernel="traj_team_kernel", bound=None, peak=None, fps=None, check_n=500,
                    label="driven two-level atom, Omega=1, gamma=0.5, t in [0,10] (101 points), sigma_z, "
                          "500 trajectories (latency bound: about 40 dependent steps of a 2x2 system)")
    if name == "tfim":
        s = [w.tfim()]
        nnz = _nnz_M(s[0])
        return dict(systems=s, n=20_000, batch=False, kernel="traj_sparse_kernel", bound="alu", peak=PEAK_FP32_VALU,
                    fps=[6 * 8.0 * nnz + 128.0 * s[0].dim], check_n=2000,
                    label=f"tfim L=10 (d=1024, CSR, nnz(M) {nnz}), J=1, h=0.8, gamma=0.05, t in [0,20] "
                          "(201 points), 20000 trajectories")
    if name == "trilinear":
        s = [w.trilinear()]
        nnz = _nnz_M(s[0])
        return dict(systems=s, n=20_000, batch=False, kernel="traj_sparse_kernel", bound="alu", peak=PEAK_FP32_VALU,
                    fps=[6 * 8.0 * nnz + 128.0 * s[0].dim], check_n=20_000,
                    label=f"trilinear (Sec. 4.2) cutoff 8 per mode (d=512, CSR, nnz(M) {nnz}), K=1, "
                          "gamma=(0.1,0.1,0.4), alpha=sqrt(3), t in [0,4] (100 points), 20000 trajectories")
    if name == "stiff":
        s = [w.jaynes_cummings(kappa=40.0, t_end=10.0, n_t=101)]
        d = s[0].dim
        return dict(systems=s, n=10_000, batch=False, kernel="traj_expo_kernel", bound="mfma", peak=PEAK["fp64"],
                    fps=None, flop_per_pass=16 * 8.0 * d * d, check_n=200,
                    forms=(("plain", dict(precision=0, form=2)), ("best", dict(precision=0, form=2, integrator=1))),
                    label="stiff Jaynes-Cummings N=20 x atom (d=40, dense), g=1, cavity decay 40, atomic decay 0.05, "
                          "alpha=2, t in [0,10] (101 points), 10000 trajectories; adaptive DOPRI5 (FP64, batched) "
                          "against the exact propagator (FP64, batched)")
    if name == "hetero":
        s = w.hetero_batch()
        return dict(systems=s, n=500, batch=True, tune_batch=True, kernel="traj_team_batch_kernel (three tile classes)", bound="mfma",
                    peak=PEAK["fp32"], fps=[6 * 8.0 * x.dim ** 2 + 128.0 * x.dim for x in s], check_n=500,
                    label="hetero_batch 64 systems d~U{8..256}, n_c~U{1..4}, t in [0,20] (101 points), "
                          "500 trajectories each")
    raise ValueError(name)


def run_secondary(name, qtm, w, torch, steps, warmup, cpu=True):
    """Plain FP64 form against the batched FP32 form on one configuration: the same keys
    as the headline line (value = the batched FP32 form's trajectories/s)."""
    sp = secondary_spec(name, qtm, w)
    systems, n = sp["systems"], sp["n"]
    total = n * len(systems)
    make = (lambda o: qtm.create_batch(systems, o)) if sp["batch"] else (lambda o: qtm.create_system(systems[0], o))
    out = {}
    forms = sp.get("forms", (("plain", dict(precision=qtm.PREC_FP64)),
                             ("best", dict(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED))))
    tuned = None
    if sp.get("tune_batch"):
        # team shape of every tile class, timed by the autotuner on the class's own systems
        from paper_1810_03047_amd import autotune
        tuned = autotune.pick_batch_waves(systems, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED), n)
        forms = (forms[0], ("best", dict(forms[1][1], class_waves=tuned["class_waves"])))
    for form_name, kw in forms:
        o = qtm.Opts(**kw)
        ctx = make(o)
        for i in range(warmup):
            ctx.run(n, 1000 + i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, fl, units = [], [], 0
        for i in range(steps):
            ctx.run(n, i)
            st = ctx.stats()
            kms.append(st["kernel_ms"])
            units += st["accepted"] + st["rejected"]
            if sp["fps"] is not None:
                f = 0.0
                for si in range(len(systems)):
                    ts = ctx.traj_stats(si)
                    f += float(ts[:, 0].sum() + ts[:, 1].sum()) * sp["fps"][si]
                fl.append(f)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r = dict(value=total * steps / wall, ms=wall / steps * 1e3, kernel_ms=float(np.mean(kms)),
                 traj_steps_per_launch=units / steps)
        if fl:
            r["tflops"] = float(np.mean(fl)) / (float(np.mean(kms)) * 1e-3) / 1e12
        elif sp.get("flop_per_pass") and o.integrator == qtm.INT_EXPO:
            r["tflops"] = st["passes"] * sp["flop_per_pass"] / (float(np.mean(kms)) * 1e-3) / 1e12
            r["products_per_team"] = st["passes"] / max(1, -(-n // 16))
        else:
            r["kernel_us_per_team_pass"] = 1e3 * float(np.mean(kms)) / max(1, st["max_team_passes"])
        out[form_name] = r
        ctx.destroy()
    b = out["best"]
    line = {
        "metric": METRIC, "value": b["value"], "unit": "trajectories/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": b["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products, f64 state", "data": "synthetic",
        "config": {"workload": sp["label"], "ntraj": total, "form": "batched+mixed", "parallelism": "trajectories (1 GPU)"},
        "plain": out["plain"], "speedup_vs_plain": b["value"] / out["plain"]["value"],
    }
    if tuned is not None:
        line["tuned_class_waves"] = {"class_waves": list(tuned["class_waves"]),
                                     "kernel_ms": {str(k): v for k, v in tuned["kernel_ms"].items()}}
    if name == "stiff":
        line["dtype"] = "f64"
        line["config"]["form"] = "exact propagator (batched)"
    if sp["peak"] is not None and "tflops" in b:
        line["roofline"] = {"bound": sp["bound"], "achieved": b["tflops"], "peak": sp["peak"], "unit": "TFLOP/s",
                            "frac": b["tflops"] / sp["peak"], "traffic": None, "kernel": sp["kernel"],
                            "kernel_ms": b["kernel_ms"]}
    else:
        line["roofline"] = None
        line["latency"] = {"kernel": sp["kernel"], "kernel_ms": b["kernel_ms"],
                           "us_per_team_pass": b["kernel_us_per_team_pass"]}
    if cpu and name == "stiff":
        line["cpu_baseline"], line["oracle_check"] = stiff_cpu_leg(qtm, systems[0], sp["check_n"])
    elif cpu:
        line["cpu_baseline"] = cpu_baseline_systems(systems, n)
        # the oracle on the first trajectories of timed seed 0 of every system, against the
        # batched FP32 form on the same trajectories
        line["oracle_check"] = oracle_check_systems(qtm, systems, sp["batch"], sp["check_n"])
    return line


def cpu_baseline_systems(systems, n, cpu_s: float = 15.0):
    """The oracle (parity build, the faster one on this workload family) on all permitted
    threads over a bounded sample: the first trajectories of seed 0 of every system."""
    import oracle
    threads, nproc, share = _threads()
    t0 = time.perf_counter()
    for si, s in enumerate(systems):
        oracle.run(s, 4, seed=0, sys_id=si, nthreads=threads)
    dt = time.perf_counter() - t0             # 4 trajectories of each system
    per = max(4, min(n, int(4 * cpu_s / max(dt * threads, 1e-3))))
    t0 = time.perf_counter()
    for si, s in enumerate(systems):
        oracle.run(s, per, seed=0, sys_id=si, nthreads=threads)
    wall = time.perf_counter() - t0
    return {"value": per * len(systems) / wall, "unit": "trajectories/s", "cores": threads, "kind": "oracle",
            "sample": f"trajectories 0..{per - 1} of each of the {len(systems)} system(s) (seed 0), FP64 C++ "
                      f"oracle (parity build), {threads} OpenMP threads (nproc {nproc}), {wall:.1f} s"}


def oracle_check_systems(qtm, systems, batch, m):
    """The batched FP32 form against the oracle (parity build) on trajectories 0..m-1 of
    seed 0 of every system: worst deviation of the averages in units of the bound
    3 sigma/sqrt(N) + 1e-6, and the fraction of trajectories with the oracle's jump
    counts."""
    import oracle
    threads, _, _ = _threads()
    o = qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, record_jumps=32)
    ctx = qtm.create_batch(systems, o) if batch else qtm.create_system(systems[0], o)
    ctx.run(m, 0)
    worst, same, tot = 0.0, 0, 0
    for si, s in enumerate(systems):
        mean, _ = ctx.expect(si)
        r = oracle.run(s, m, seed=0, sys_id=si, nthreads=threads, jcap=32)
        bound = 3.0 * np.sqrt(np.maximum(r["var"], 0.0) / m) + 1e-6
        worst = max(worst, float(np.max(np.abs(mean.real - r["mean"].real) / bound)))
        jn = np.array([ctx.jumps(i, system=si)[2] for i in range(m)])
        same += int(np.sum(jn == r["jump_counts"]))
        tot += m
    ctx.destroy()
    return {"ntraj_per_system": m, "seed": 0, "max_dev_over_bound": worst, "within_bound": worst <= 1.0,
            "identical_jump_counts": same / tot}


def stiff_cpu_leg(qtm, system, m):
    """The exact-propagator oracle (Python, scipy's matrix exponential, one thread) timed on
    trajectories 0..m-1 of seed 0, and the same trajectories of the library's
    exact-propagator form compared with it one by one."""
    from oracle import expo
    t0 = time.perf_counter()
    r = expo.run_expo(system, m, seed=0)
    dt = time.perf_counter() - t0
    base = {"value": m / dt, "unit": "trajectories/s", "cores": 1, "kind": "oracle",
            "sample": f"trajectories 0..{m - 1} (seed 0), exact-propagator oracle (numpy/scipy, one thread), {dt:.1f} s"}
    ctx = qtm.create_system(system, qtm.Opts(precision=0, form=qtm.FORM_BATCHED, integrator=qtm.INT_EXPO,
                                             record_jumps=32, keep_traj=1))
    ctx.run(m, 0)
    X = ctx.traj_expect()
    same, jtd = 0, 0.0
    for i in range(m):
        t, c, cnt = ctx.jumps(i)
        if cnt == r["jump_counts"][i]:
            same += 1
            k = min(cnt, 32)
            if k and np.array_equal(c[:k], r["jump_channels"][i, :k]):
                jtd = max(jtd, float(np.max(np.abs(t[:k] - r["jump_times"][i, :k]))))
    ctx.destroy()
    return base, {"ntraj": m, "seed": 0, "identical_jump_counts": same / m, "max_jump_time_diff": jtd,
                  "max_output_diff": float(np.max(np.abs(X - r["X"])))}


def other_workload(a, qtm, w, torch):
    """One secondary configuration as its own JSON line (--workload NAME)."""
    print(json.dumps(run_secondary(a.workload, qtm, w, torch, a.steps, a.warmup, cpu=not a.no_cpu)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="plain,best")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="JSON file for the autotuner's choices")
    ap.add_argument("--counters", action="store_true",
                    help="short run for rocprofv3 counter passes: two launches of the headline kernel "
                         "(FP32 products, batched, 10,000 trajectories; or of --workload's batched form) "
                         "and a 256 MiB device copy for calibration")
    ap.add_argument("--workload", default="jcm", choices=["jcm", "two_level", "tfim", "hetero", "trilinear", "stiff"],
                    help="jcm (default, the headline) or a secondary configuration alone")
    ap.add_argument("--class-waves", default="",
                    help="with --counters --workload hetero: waves per team of the three tile classes, e.g. 4,8,8")
    ap.add_argument("--no-secondary", action="store_true",
                    help="leave out the secondary configurations nested in the headline line")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: trajectories are independent and the multi-GPU path "
              "(one all-reduce of the FP64 sums) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1810_03047_amd as qtm
    from paper_1810_03047_amd import autotune
    import workloads as w

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.counters:
        if a.workload == "hetero":
            # the heterogeneous batch's tile-class launches with the shapes the autotuner picks
            systems = w.hetero_batch()
            cw = tuple(int(x) for x in a.class_waves.split(",")) if a.class_waves else (0, 0, 0)
            ctx = qtm.create_batch(systems, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, class_waves=cw))
            for i in range(2):
                ctx.run(500, i)
        elif a.workload != "jcm":
            sp = secondary_spec(a.workload, qtm, w)
            kw = dict(sp["forms"][1][1]) if "forms" in sp else dict(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED)
            ctx = qtm.create_system(sp["systems"][0], qtm.Opts(**kw))
            for i in range(2):
                ctx.run(sp["n"], i)
        else:
            ctx = qtm.create_system(w.jaynes_cummings(), qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, team_waves=1))
            for i in range(2):
                ctx.run(NTRAJ, i)
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        x.fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "kernel_ms": ctx.stats()["kernel_ms"], "copy_bytes": 4 * x.numel()}), flush=True)
        return
    if a.workload != "jcm":
        other_workload(a, qtm, w, torch)
        return
    system = w.jaynes_cummings()
    d = system.dim
    forms = a.forms.split(",")
    res, tuned = {}, {}
    if "plain" in forms:
        o = qtm.Opts(precision=qtm.PREC_FP64)
        tw = autotune.pick_team_waves(system, o, NTRAJ, cache_path=a.tune_cache)
        tuned["plain"] = tw
        o.team_waves = tw["team_waves"]
        print(f"[bench] plain: team_waves {tw}", file=sys.stderr, flush=True)
        res["plain"] = time_form(qtm, system, o, a.steps, a.warmup)
        opts_plain = o
    best_name, train_info, proposal = None, None, None
    if "best" in forms:
        form = qtm.FORM_BATCHED
        if not a.no_learned:
            t0 = time.perf_counter()
            F, T, f_ops = training_data(qtm, system)
            t1 = time.perf_counter()
            trainer = qtm.create_system(system, qtm.Opts())
            losses = trainer.train_proposal(F, T, epochs=8, batch=4096, lr=2e-3, seed=0)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            proposal = (trainer.get_proposal(), f_ops)
            trainer.destroy()
            form |= qtm.FORM_LEARNED
            train_info = {"samples": int(len(F)), "epochs": 8, "data_s": t1 - t0, "train_s": t2 - t1,
                          "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
            print(f"[bench] proposal trained: {train_info}", file=sys.stderr, flush=True)
        o = qtm.Opts(precision=qtm.PREC_FP32, form=form)
        tw = autotune.pick_team_waves(system, o, NTRAJ, cache_path=a.tune_cache, proposal=proposal)
        tuned["best"] = tw
        o.team_waves = tw["team_waves"]
        print(f"[bench] best: team_waves {tw}", file=sys.stderr, flush=True)
        res["best"] = time_form(qtm, system, o, a.steps, a.warmup, proposal=proposal)
        best_name = "learned+batched+mixed" if proposal is not None else "batched+mixed"
    head = res.get("best") or res["plain"]
    prec = "fp32" if "best" in res else "fp64"
    tps = NTRAJ * a.steps / head["wall"]
    flops = head["steps_per_run"] * jcm_flops_per_step(d)
    achieved = flops / (head["kernel_ms"] * 1e-3) / 1e12
    head_waves = tuned.get("best" if "best" in res else "plain", {}).get("team_waves", 0)
    xflop = jcm_executed_flops_per_step(system, head_waves in (0, 1))
    line = {
        "metric": METRIC, "value": tps, "unit": "trajectories/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["wall"] / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products, f64 state" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "jaynes_cummings N=20 x atom (d=40, dense), g=1, kappa=0.1, gamma=0.05, alpha=2, "
                               "t in [0,50] (501 points), rtol 1e-6, atol 1e-8, 10000 trajectories",
                   "ntraj": NTRAJ, "form": best_name or "plain", "parallelism": "trajectories (1 GPU)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[prec], "traffic": measured_traffic(),
                     "kernel": "traj_team_kernel", "kernel_ms": head["kernel_ms"], "run_event_ms": head["run_event_ms"],
                     "flop_per_traj_step": jcm_flops_per_step(d), "traj_steps_per_launch": head["steps_per_run"],
                     "executed_flop_per_traj_step": xflop,
                     "executed_tflops": head["steps_per_run"] * xflop / (head["kernel_ms"] * 1e-3) / 1e12},
        "tuned_team_waves": {k: v["team_waves"] for k, v in tuned.items()},
    }
    if train_info:
        line["training"] = train_info
    if "plain" in res and "best" in res:
        p = res["plain"]
        line["plain"] = {"value": NTRAJ * a.steps / p["wall"], "kernel_ms": p["kernel_ms"],
                         "traj_steps_per_launch": p["steps_per_run"],
                         "tflops": p["steps_per_run"] * jcm_flops_per_step(d) / (p["kernel_ms"] * 1e-3) / 1e12}
        line["speedup_vs_plain"] = line["value"] / line["plain"]["value"]
        line["per_traj"] = {k: {"accepted": r["acc"] / NTRAJ, "rejected": r["rej"] / NTRAJ,
                                "segments": r["segments"] / NTRAJ} for k, r in res.items()}
    if not a.no_cpu:
        # the CPU leg: the oracle timed on the host, and the same oracle (parity build)
        # checking the timed forms on trajectories 0..NTRAJ-1 of timed seed 0
        line["cpu_baseline"] = cpu_baseline(system, *(
            (_working_params(proposal[0]), proposal[1]) if ("best" in res and proposal is not None) else (None, None)))
        print(f"[bench] cpu baseline: {line['cpu_baseline']}", file=sys.stderr, flush=True)
        checks = {}
        if "best" in res:
            checks["headline"] = oracle_check(qtm, system, o, proposal, NTRAJ, seed=0)
        if "plain" in res:
            checks["plain"] = oracle_check(qtm, system, opts_plain, None, NTRAJ, seed=0)
        line["oracle_check"] = checks
    if not a.no_secondary:
        # the other configurations (two-level atom, Ising chain, heterogeneous batch,
        # trilinear Hamiltonian), each with its plain form, roofline, CPU baseline and
        # oracle check, nested in the one line
        line["secondary"] = {}
        for name in ("two_level", "tfim", "hetero", "trilinear", "stiff"):
            t0 = time.perf_counter()
            line["secondary"][name] = run_secondary(name, qtm, w, torch, max(2, min(a.steps, 3)), 1, cpu=not a.no_cpu)
            print(f"[bench] secondary {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
