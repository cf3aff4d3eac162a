"""Benchmark: stage-parallel Radau IIA on one MI355X.

Workload (the 64^3 mixed-precision batched configuration): unit cube with
64^3 hexahedral cells, Q_4 elements (257^3 = 16,974,593 nodes per stage),
Radau IIA with Q = 4 stages, tau = 5e-4, seeded smooth initial data (16
Fourier modes, amplitudes N(0,1)/|kappa|^2, seed 0), f = 0; FGMRES in fp64 to
rtol 1e-10 with the block preconditioner whose V-cycles, smoother and
transfers run in fp32 with all Q blocks batched into every launch.

Reported:
* value: stage-DoFs/s of the batched fp32 block operator (lam_i M + tau K on
  all Q stages in one launch), stage-DoFs = Q * N^3 (boundary nodes counted,
  as in the paper's DoF table), timed with HIP events on the library stream;
* ms_per_step: wall time of one Radau IIA step (K steps timed after W
  warm-up steps, synchronised on both sides);
* roofline of that operator kernel: it is bound by fp32 vector arithmetic
  (84 flop per stage-DoF for Q_4 against the 78.6 TFLOP/s non-packed fp32
  rate), with the HBM view (8 B per stage-DoF against 8 TB/s) beside it and
  the HBM bytes that the FETCH_SIZE / WRITE_SIZE counters measured;
* plain_fp64_per_stage: the same steps with the preconditioner in fp64 and
  the Q blocks solved one after another (the unbatched, full-precision form);
* uneven_batch: 64 independent problems (the seeded mixed batch of meshes,
  degrees, Q and tau), one step each through rk_step_batch, concurrent on 8
  streams, against the same steps one after another;
* host leg (skipped with --no-cpu), the only part that runs the oracle:
  cpu_baseline, the oracle's assembled block operator (scipy CSR SpMV) on a
  bounded sample (16^3 cells, Q_4, same Q and tau), in the same unit; and
  accuracy_vs_oracle, the error of one GPU step on the 32^3 Q_4 grid against
  the oracle's exact step for FGMRES tolerances 1e-6 .. 1e-10, and
  accuracy_vs_oracle_64cubed, the same on the 64^3 Q_4 grid of the workload.
  The loosest tolerance within 1e-8 on both grids then sets at_1e-8_accuracy:
  s per step of each form at that accuracy.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --mode op [--op-reps R]      (operator launches + one
           device copy of the same size, for counter runs)
       python bench.py --mode deformed [--op-reps R]   (the same for the
           deformed-mesh operator, Q = 4)
       python bench.py --traffic-from FETCH.csv WRITE.csv   (turn two
           rocprofv3 --pmc runs of --mode op into the committed traffic record)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stage-DoFs/s of batched matrix-free operator; s per Radau step at 1e-8 tol"
HBM_PEAK_GBS = 8000.0
# fp32 vector rate without packed instructions: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
OP_KERNEL = "op_kernel<4, float, MIX_DIAG, EPI_STORE>"
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def op_flops_per_stage_dof(k: int) -> float:
    """Arithmetic of the sum-factorised block operator per output node and
    stage (multiply-add = 2 flop): x-pass 2 banded 1D products (2k+3 flop per
    node each) + 4 flop of scaling, y-pass 3 products + 1 add, z-pass
    4(k+1) flop per plane plus the element-start terms (3(k+1)+1)/k."""
    return (2 * (2 * k + 3) + 4) + (3 * (2 * k + 3) + 1) + 4 * (k + 1) + (3 * (k + 1) + 1) / k
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_op_blocks_fp32_64cubed_q4.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2209_06700_amd", "csrc", "op_kernel.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_key(cz, ts=0):
    return str(cz) if ts == 0 else f"ts{ts}_cz{cz}"


def measured_traffic(cz, ts=0):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source with the z-chunk length `cz` and
    tile shape `ts` that the timed launches use."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return rec.get("by_cz", {}).get(traffic_key(cz, ts), {}).get("hbm_bytes_per_launch")


def _counter_rows(path, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 counter_collection.csv."""
    import csv
    out = []
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                out.append((row["Kernel_Name"], float(row["Counter_Value"])))
    return out


def traffic_record(fetch_csv, write_csv, cz, n=64, k=4, Q=4, reps=3, ts=0):
    """HBM bytes per launch of the operator kernel with z-chunk length cz:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one rocprofv3 --pmc run each,
    --cz cz for every launch of the run), averaged over the last `reps`
    (timed) operator dispatches, each scaled by the ratio of the known size of
    a plain device copy to what the same counter read for that copy in the
    same run.  Merged into the record of other chunk lengths."""
    N = n * k + 1
    copy_bytes = 4.0 * Q * N ** 3
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        if rec.get("kernel_source_sha256_16") != kernel_hash() or "by_cz" not in rec:
            rec = {}
    except (OSError, ValueError):
        rec = {}
    rec.update({"kernel": OP_KERNEL, "workload": f"{n}^3 cells Q_{k}, Q={Q}, fp32 block operator",
                "kernel_source_sha256_16": kernel_hash(), "copy_kernel": COPY_KERNEL, "copy_bytes": copy_bytes,
                "algorithmic_bytes_per_launch": 8.0 * Q * N ** 3,
                "commands (per chunk length CZ)": [
                    f"rocprofv3 --pmc {c} -d pmc_{c.split('_')[0].lower()}_czCZ -o op "
                    f"--output-format csv -- python3 bench.py --mode op --cz CZ --tile-shape TS --op-reps {reps}"
                    for c in ("FETCH_SIZE", "WRITE_SIZE")]
                + ["python bench.py --traffic-from pmc_fetch_czCZ/op_counter_collection.csv "
                   "pmc_write_czCZ/op_counter_collection.csv --cz CZ --tile-shape TS"]})
    rec.pop("commands", None)
    entry = {}
    total = 0.0
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _counter_rows(path, counter)
        op = [v for nm, v in rows if f"op_kernel<{k}, float, 0, 0, {ts}>" in nm]
        cp = [v for nm, v in rows if COPY_KERNEL in nm]
        if len(op) < reps or not cp:
            raise SystemExit(f"{path}: no {counter} rows for the operator or the copy kernel")
        op = op[-reps:]
        kib_op = sum(op) / len(op)
        kib_cp = cp[-1]
        scale = copy_bytes / (kib_cp * 1024.0)
        entry[counter] = {"op_kib_per_dispatch": kib_op, "op_dispatches": len(op), "copy_kib": kib_cp,
                          "scale": scale, "op_bytes_per_launch": kib_op * 1024.0 * scale}
        total += kib_op * 1024.0 * scale
    entry["hbm_bytes_per_launch"] = total
    entry["bytes_per_stage_dof"] = total / (Q * N ** 3)
    rec.setdefault("by_cz", {})[traffic_key(cz, ts)] = entry
    return rec


def time_op(torch, R, ctx, form, u, v, reps):
    """Average launch time of rk_apply_operator, HIP events on the context's stream."""
    stream = ctx.stream
    R.rk_apply_operator(ctx, form, u, v)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        R.rk_apply_operator(ctx, form, u, v)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) * 1e-3 / reps


RTOLS = (1e-6, 1e-7, 1e-8, 1e-9, 1e-10)
# the complex method's stopping test is per block in the eigenbasis of A^-1:
# it needs tighter tolerances for the same accuracy of y
RTOLS_COMPLEX = (1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12)


def time_steps(torch, R, n, k, Q, tau, steps, warmup, y0, blocks=None, **opts):
    """Average wall time of `steps` Radau IIA steps after `warmup` steps, from
    the seeded initial data, synchronised on both sides; FGMRES iterations.
    With a list `blocks`, the per-block iteration counts of every step are
    appended to it (complex method)."""
    s = R.RadauIIA(n, k, Q, tau, **opts)
    y = y0.clone()
    t = 0.0
    for _ in range(warmup):
        s.step(t, y)
        t += tau
    torch.cuda.synchronize()
    its, vcs = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = s.step(t, y)
        its.append(st["iterations"])
        vcs.append(st["vcycles"])
        if blocks is not None:
            blocks.append(st["block_iterations"][:(Q + 1) // 2])
        t += tau
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    s.close()
    return dt, its, vcs


def cpu_baseline_leg(torch, R, n=16, k=4, Q=4, tau=5e-4, budget_s=12.0):
    """The host-side leg, the only part of the bench that runs the oracle:
    * the oracle's assembled block operator v_i = (lam_i M + tau K) u_i by CSR
      SpMV (scipy, one thread) on a bounded sample, timed on the host cores;
    * the oracle's exact (modal) Radau IIA step on the 32^3 Q_4 grid and on
      the 64^3 Q_4 grid of the workload itself, the references for the error
      of GPU steps at several FGMRES tolerances."""
    import numpy as np
    from oracle.assemble import Problem
    from oracle.step import ModalSolver
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    p = Problem(n, k, "kron")
    tab = RadauIIA(Q)
    A = [(l * p.M + tau * p.K).tocsr() for l in tab.lam]
    N = n * k + 1
    u = np.random.default_rng(0).standard_normal((Q, p.M.shape[0]))
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < budget_s:
        for i in range(Q):
            A[i] @ u[i]
        reps += 1
        t = time.perf_counter() - t0
    cpu = {"value": Q * N ** 3 * reps / t, "unit": "stage-DoFs/s", "cores": 1, "kind": "oracle",
           "sample": f"assembled block operator (lam_i M + tau K, scipy CSR SpMV, single thread) on "
                     f"{n}^3 cells Q_{k} (N={N}), Q={Q}, {reps} applies in {t:.1f} s",
           "host_cpu_count": os.cpu_count(), "host_cpu_model": host_cpu_model()}
    cpu.update(oracle_runs())
    acc = accuracy_leg(torch, R, 32, k, Q, tau)
    acc64 = accuracy_leg(torch, R, 64, k, Q, tau)
    return cpu, acc, acc64


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_runs():
    """Wall time of whole oracle runs on the host (one thread: SuperLU and
    scipy SpMV are single-threaded):
    * the 8^3 Q_2 manufactured-solution configuration, Q = 2, tau = 0.05, 10
      steps by the direct sparse solve of the stage system;
    * one step of the oracle's FGMRES + block-preconditioned multigrid at
      8^3 Q_4, Q = 4, tau = 5e-4, rtol 1e-10 (set-up timed apart), and its
      linear extrapolation in the number of unknowns to 32^3 Q_4 (64 times as
      many; the iteration count of the multigrid preconditioner does not
      grow with n), since assembling 32^3 Q_4 on the host takes hours."""
    import math
    import numpy as np
    from oracle.assemble import Problem, interpolate, load_separable
    from oracle.fgmres import IterativeStepper
    from oracle.step import DirectStepper
    from oracle.tableau import RadauIIA
    t0 = time.perf_counter()
    n0, k0, Q0, tau0 = 8, 2, 2, 0.05
    p = Problem(n0, k0)
    tab = RadauIIA(Q0)
    G = p.to_int(load_separable(p.mesh, lambda x: np.sin(np.pi * x)))
    y = p.to_int(interpolate(p.mesh, lambda x, y_, z: np.sin(np.pi * x) * np.sin(np.pi * y_) * np.sin(np.pi * z)))
    ds = DirectStepper(p.M, p.K, tab, tau0)
    for st in range(10):
        gam = np.array([(3 * math.pi ** 2 - 1) * math.exp(-(st + c) * tau0) for c in tab.c])
        y, _ = ds.step(y, gam[:, None] * G[None, :])
    t_d0 = time.perf_counter() - t0
    t0 = time.perf_counter()
    it = IterativeStepper(8, 4, RadauIIA(4), 5e-4)
    t_setup = time.perf_counter() - t0
    pp = Problem(8, 4, "kron")
    yy = np.random.default_rng(0).standard_normal(pp.M.shape[0])
    t0 = time.perf_counter()
    _, its, _ = it.step(yy, rtol=1e-10)
    t_step = time.perf_counter() - t0
    return {"d0_manufactured_8cubed_q2_10_steps_s": t_d0,
            "o_iter_8cubed_q4_Q4": {"setup_s": t_setup, "step_s": t_step, "fgmres_iterations": its},
            "o_iter_32cubed_q4_Q4_step_s_extrapolated": t_step * 64,
            "threads": 1}


def accuracy_leg(torch, R, na, k=4, Qa=4, tau=5e-4):
    """Error of one GPU step (seeded Fourier data, every form and FGMRES
    tolerance) against the oracle's exact modal step on the na^3 Q_k grid."""
    import numpy as np
    from oracle.step import ModalSolver
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    Na = na * k + 1
    inner = lambda v: v.reshape(Na, Na, Na)[1:-1, 1:-1, 1:-1].reshape(-1)
    s = R.RadauIIA(na, k, Qa, tau, autotune=0)
    x1 = grid_coords(s.info["nodes"], na)
    s.close()
    y0 = fourier_field(x1, seed=0)
    t0 = time.perf_counter()
    ref = ModalSolver(na, k).step(RadauIIA(Qa), tau, inner(y0))
    t_oracle = time.perf_counter() - t0
    acc = {"grid": f"{na}^3 cells Q_{k}, Q={Qa}, tau={tau:g}, same seeded data", "oracle_modal_step_s": t_oracle,
           "mixed_batched": {}, "fp64_per_stage": {}, "complex_presb_mixed_batched": {}}
    for name, prec, mode, method, rtols in (
            ("mixed_batched", R.RK_PREC_MIXED, R.RK_BATCHED, R.RK_METHOD_CROUT, RTOLS),
            ("fp64_per_stage", R.RK_PREC_FP64, R.RK_PER_STAGE, R.RK_METHOD_CROUT, RTOLS),
            ("complex_presb_mixed_batched", R.RK_PREC_MIXED, R.RK_BATCHED, R.RK_METHOD_COMPLEX, RTOLS_COMPLEX)):
        for rtol in rtols:
            s = R.RadauIIA(na, k, Qa, tau, precision=prec, mode=mode, rtol=rtol, method=method)
            y = torch.tensor(y0, device="cuda")
            st = s.step(0.0, y)
            err = float(np.linalg.norm(inner(y.cpu().numpy()) - ref) / np.linalg.norm(ref))
            acc[name][f"{rtol:.0e}"] = {"rel_l2_error": err, "fgmres_iterations": st["iterations"]}
            s.close()
            del y
    del ref, y0
    torch.cuda.empty_cache()
    return acc


def time_op_rotated(torch, R, ctx, form, us, vs, reps):
    """Average launch time of rk_apply_operator cycling through the buffer
    pairs (us[i], vs[i]) (together larger than the 256 MB Infinity Cache),
    HIP events on the context's stream."""
    stream = ctx.stream
    for u, v in zip(us, vs):
        R.rk_apply_operator(ctx, form, u, v)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for r in range(reps):
        R.rk_apply_operator(ctx, form, us[r % len(us)], vs[r % len(vs)])
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) * 1e-3 / reps


def fp64_32cubed_legs(torch, R, y0_fn, steps=20, reps=40):
    """The 32^3 Q_4 fp64 configurations:
    * the plain per-stage form at Q = 3, tau = 1e-3: `steps` Radau IIA steps
      from the seeded Fourier data (s per step);
    * stage-batched at Q = 3 and Q = 5: the operators RK_OP_CALA and
      RK_OP_BLOCKS in isolation, hot (one buffer pair, which fits in the
      Infinity Cache) and rotated over buffer pairs of more than 512 MB, in
      stage-DoFs/s and as a fraction of the HBM roofline (16 B per stage-DoF
      read + written, fp64); and full steps (s per step)."""
    n, k, tau = 32, 4, 1e-3
    N = n * k + 1
    out = {"grid": f"{n}^3 cells Q_{k} ({N}^3 nodes/stage), tau={tau:g}, fp64, rtol 1e-10"}
    y0 = y0_fn(n, k)
    t_ps, its_ps, _ = time_steps(torch, R, n, k, 3, tau, steps, 1, y0, rtol=1e-10,
                                 precision=R.RK_PREC_FP64, mode=R.RK_PER_STAGE)
    out["per_stage_Q3"] = {"steps": steps, "ms_per_step": t_ps * 1e3, "fgmres_iterations": its_ps}
    for Q in (3, 5):
        sd = Q * N ** 3
        s = R.RadauIIA(n, k, Q, tau, precision=R.RK_PREC_FP64, mode=R.RK_BATCHED, rtol=1e-10)
        nrot = max(2, int(600e6 // (2 * 8 * sd)) + 1)
        us = [torch.randn(sd, dtype=torch.float64, device="cuda") for _ in range(nrot)]
        vs = [torch.empty_like(us[0]) for _ in range(nrot)]
        ops = {}
        for name, form in (("CALA", R.RK_OP_CALA), ("BLOCKS", R.RK_OP_BLOCKS)):
            t_hot = time_op(torch, R, s.ctx, form, us[0], vs[0], reps)
            t_rot = time_op_rotated(torch, R, s.ctx, form, us, vs, reps)
            ops[name] = {"us_hot": t_hot * 1e6, "us_rotated": t_rot * 1e6,
                         "stage_dofs_per_s_hot": sd / t_hot, "stage_dofs_per_s_rotated": sd / t_rot,
                         "hbm_frac_rotated": 16.0 * sd / t_rot / 1e9 / HBM_PEAK_GBS,
                         "rotated_bytes": 2 * 8 * sd * nrot}
        s.close()
        del us, vs
        torch.cuda.empty_cache()
        t_b, its_b, _ = time_steps(torch, R, n, k, Q, tau, min(steps, 10), 1, y0, rtol=1e-10,
                                   precision=R.RK_PREC_FP64, mode=R.RK_BATCHED)
        out[f"batched_Q{Q}"] = {"operators": ops, "ms_per_step": t_b * 1e3, "fgmres_iterations": its_b}
    return out


BATCH_CELLS = (4, 6, 8, 12, 16, 24, 32, 48)


def uneven_batch(torch, R, count=64, seed=1, streams=8, restart=20, autotune=1):
    """The uneven batch: `count` independent heat problems, one Radau IIA step
    each, drawn with numpy.random.default_rng(seed): n^3 cells with n from
    4..48 (values with a multigrid hierarchy: n = 2^j or 3 * 2^j), degree
    U{1..6}, Q U{1..5}, tau log-uniform in [1e-4, 1e-1], mixed precision,
    seeded Fourier data.  The problems are spread over the streams by load
    (largest first, each onto the least loaded stream, the load of a problem
    being max(stage-DoFs, 8M)).
    Timed once concurrently (rk_step_batch, one host thread per stream) and
    once one problem after another."""
    import numpy as np
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(count):
        n = int(rng.choice(BATCH_CELLS))
        k = int(rng.integers(1, 7))
        Q = int(rng.integers(1, 6))
        tau = float(10 ** rng.uniform(-4, -1))
        probs.append((n, k, Q, tau))
    sts = [torch.cuda.Stream() for _ in range(streams)]
    # streams by load: problems largest first, each onto the least loaded
    # stream, by the estimated cost max(stage-DoFs, 8M) (below about 8M
    # stage-DoFs a step is bound by launch and synchronisation latency)
    cost = [max(Q * (n * k + 1) ** 3, 8 << 20) for n, k, Q, _ in probs]
    load, sid = [0] * streams, [0] * count
    for i in sorted(range(count), key=lambda i: -cost[i]):
        s = min(range(streams), key=lambda j: load[j])
        sid[i] = s
        load[s] += cost[i]
    # one V-cycle stream per context (vc_streams = 1): the concurrent
    # contexts already fill the GPU, and split V-cycles measured slower here
    ctxs = [R.RadauIIA(n, k, Q, tau, precision=R.RK_PREC_MIXED, rtol=1e-10, restart=restart,
                       autotune=autotune, vc_streams=1, stream=sts[sid[i]])
            for i, (n, k, Q, tau) in enumerate(probs)]
    y0 = [torch.tensor(fourier_field(grid_coords(c.info["nodes"], n), seed=i), device="cuda")
          for i, (c, (n, _, _, _)) in enumerate(zip(ctxs, probs))]
    handles = [c.ctx for c in ctxs]
    zeros = [0.0] * count

    def run(threads):
        ys = [y.clone() for y in y0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = R.rk_step_batch(handles, zeros, ys, threads=threads)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    run(streams)                                  # warm-up (graph capture, caches)
    t_conc, st = run(streams)
    t_seq, _ = run(1)
    sdofs = sum(Q * (n * k + 1) ** 3 for n, k, Q, _ in probs)
    its = [s["iterations"] for s in st]
    ops = operator_batch_leg(torch, R, ctxs, sdofs)
    for c in ctxs:
        c.close()
    del y0
    torch.cuda.empty_cache()
    return {"problems": count, "recipe": f"default_rng({seed}): n in {list(BATCH_CELLS)}, k U{{1..6}}, "
                                         f"Q U{{1..5}}, tau log-uniform [1e-4, 1e-1], mixed, rtol 1e-10, vc_streams 1, "
                                         f"restart {restart}, streams assigned by load max(stage-DoFs, 8M)",
            "stage_dofs": sdofs, "streams": streams, "autotune": autotune, "s_concurrent": t_conc,
            "s_sequential": t_seq,
            "speedup": t_seq / t_conc, "stage_dof_steps_per_s": sdofs / t_conc,
            "fgmres_iterations": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)},
            "operator_blocks_fp32": ops}


def operator_batch_leg(torch, R, ctxs, sdofs, reps=20):
    """The fp32 block operator (lam_i M + tau K on all Q stages) of every
    problem of the uneven batch: once as one rk_apply_operator launch per
    context (on the contexts' own streams), once as the work-list launches of
    rk_apply_operator_batch on one stream.  Wall time per pass over the batch,
    synchronised on both sides, after a warm-up pass."""
    us = [torch.randn(c.Q * c.N ** 3, dtype=torch.float32, device="cuda") for c in ctxs]
    vs = [torch.empty_like(u) for u in us]

    def measure(sel):
        def per_context():
            for i in sel:
                R.rk_apply_operator(ctxs[i].ctx, R.RK_OP_BLOCKS, us[i], vs[i])

        def work_list():
            R.rk_apply_operator_batch([ctxs[i].ctx for i in sel], R.RK_OP_BLOCKS, [us[i] for i in sel],
                                      [vs[i] for i in sel])

        out = {}
        for name, fn in (("per_context_launches", per_context), ("work_list", work_list)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            out[f"{name}_ms"] = (time.perf_counter() - t0) / reps * 1e3
        # problems of 2^23 stage-DoFs or more take their own launch, the
        # others one work-list launch per degree and group of 12
        alone = [i for i in sel if ctxs[i].Q * ctxs[i].N ** 3 >= 8 << 20]
        deg = [ctxs[i].info["degree"] for i in sel if i not in alone]
        sd = sum(ctxs[i].Q * ctxs[i].N ** 3 for i in sel)
        out.update({"problems": len(sel), "stage_dofs": sd, "own_launches": len(alone),
                    "list_launches": sum((deg.count(d) + 11) // 12 for d in set(deg)),
                    "work_list_stage_dofs_per_s": sd / (out["work_list_ms"] * 1e-3),
                    "speedup": out["per_context_launches_ms"] / out["work_list_ms"]})
        return out

    small = [i for i, c in enumerate(ctxs) if c.Q * c.N ** 3 < 1 << 20]
    out = {"all": measure(list(range(len(ctxs)))), "below_1M_stage_dofs": measure(small)}
    del us, vs
    torch.cuda.empty_cache()
    return out


def deformed_leg(torch, R, n=64, k=4, eps=0.05, qs=(1, 2, 4, 8), reps=10):
    """The deformed-mesh operator (cell-based, per-point geometry) at n^3 Q_k
    in fp32 for several stage counts: the geometry is read once per cell for
    all Q stages, so its share of the traffic per stage-DoF falls as 1/Q."""
    op = R.DeformedOperator(n, k, eps, dtype=torch.float32)
    N = n * k + 1
    geo_bytes = op.geometry.numel() * 4
    nq = k + 1
    flop_cell = 12 * 2 * nq ** 4 + 18 * nq ** 3        # 12 contractions + the point operation
    out = {"mesh": f"{n}^3 cells Q_{k}, eps={eps}, fp32", "geometry_bytes": geo_bytes, "by_Q": {}}
    for Q in qs:
        u = torch.randn(Q * N ** 3, dtype=torch.float32, device="cuda")
        v = torch.empty_like(u)
        alpha, beta = [2.0] * Q, [5e-4] * Q
        op.apply(u, v, alpha, beta)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op.apply(u, v, alpha, beta)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        sd = Q * N ** 3
        alg = 8.0 * sd + geo_bytes
        out["by_Q"][str(Q)] = {"us_per_apply": t * 1e6, "stage_dofs_per_s": sd / t,
                               "algorithmic_bytes_per_stage_dof": alg / sd, "GBps": alg / t / 1e9,
                               "TFLOPs": flop_cell * n ** 3 * Q / t / 1e12}
        del u, v
    del op
    torch.cuda.empty_cache()
    return out


def deformed_step_leg(torch, R, y0, n=64, k=4, Q=4, tau=5e-4, eps=0.05, steps=3):
    """Radau IIA steps on the deformed mesh (mixed, batched, rtol 1e-10): the
    Krylov operator and K y_n read the per-point geometry once per cell for
    all Q stages; the V-cycles run on the deformed levels (deform_mg = 1) or
    on the affine levels (deform_mg = 0)."""
    out = {"eps": eps, "rtol": 1e-10}
    for dmg, name in ((1, "deformed_levels"), (0, "affine_levels")):
        t, its, _ = time_steps(torch, R, n, k, Q, tau, steps, 1, y0, rtol=1e-10, precision=R.RK_PREC_MIXED,
                               mode=R.RK_BATCHED, deform=eps, deform_mg=dmg)
        out[name] = {"ms_per_step": t * 1e3, "fgmres_iterations": its}
    return out


def loosest_rtol(*acc_runs, bound=1e-8):
    """The loosest FGMRES tolerance whose step error is within `bound` on
    every grid given (dicts tolerance -> run)."""
    rtols = set(acc_runs[0])
    ok = [float(r) for r in rtols if all(runs[r]["rel_l2_error"] <= bound for runs in acc_runs)]
    return max(ok) if ok else min(float(r) for r in rtols)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--op-reps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the host leg (oracle)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain fp64 per-stage comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven batch of 64 problems")
    ap.add_argument("--no-fp64-32", action="store_true",
                    help="skip the 32^3 Q_4 fp64 legs (per-stage Q=3 steps, batched Q=3/5 operators and steps)")
    ap.add_argument("--no-deformed", action="store_true", help="skip the deformed-mesh operator leg")
    ap.add_argument("--no-complex", action="store_true",
                    help="skip the direct complex diagonalisation (PRESB) comparison")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--cheb-degree", type=int, default=None, help="smoother degree (library default if unset)")
    ap.add_argument("--cheb-range", type=float, default=None, help="Chebyshev range (library default if unset)")
    ap.add_argument("--mode", choices=["full", "op", "deformed", "cala", "oplist"], default="full",
                    help="op: only the batched fp32 block operator launches; deformed: only the "
                         "deformed-mesh operator; cala: only the fp64 stage operator A^-1 (x) M + tau I (x) K "
                         "(all for counter runs); oplist: only the uneven batch's operator leg (per-context "
                         "and work-list launches, no steps; for kernel traces)")
    ap.add_argument("--cz", type=int, default=None,
                    help="--mode op: fixed z-chunk length (rk_options.z_chunk); --traffic-from: the one the "
                         "counter runs used")
    ap.add_argument("--tile-shape", type=int, default=0,
                    help="with --cz: the tile shape (rk_options.tile_shape) of the op-mode launches and of the "
                         "counter runs (--traffic-from)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record from two rocprofv3 --pmc runs of --mode op")
    args = ap.parse_args()
    if args.traffic_from:
        if args.cz is None:
            raise SystemExit("--traffic-from needs --cz (the z-chunk of the counter runs)")
        rec = traffic_record(*args.traffic_from, cz=args.cz, n=args.n, ts=args.tile_shape)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is a design note only)", file=sys.stderr)
        return 2
    import torch
    from paper_2209_06700_amd import rk as R
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    assert torch.cuda.is_available(), "no GPU"
    n, k, Q, tau = args.n, 4, 4, 5e-4
    N = n * k + 1
    log(f"[bench] creating 64^3-class context n={n} k={k} Q={Q}")
    if args.mode == "op":
        # explicit Chebyshev bounds: no eigenvalue estimation launches at create
        solver = R.RadauIIA(n, k, Q, tau, precision=R.RK_PREC_MIXED, mode=R.RK_BATCHED, restart=1,
                            eig_max=[1.0] * R.n_levels(n), z_chunk=args.cz or 0,
                            tile_shape=args.tile_shape if args.cz else 0)
        u32 = torch.randn(Q * N ** 3, dtype=torch.float32, device="cuda")
        v32 = torch.empty_like(u32)
        t_blk = time_op(torch, R, solver.ctx, R.RK_OP_BLOCKS, u32, v32, args.op_reps)
        # one plain device-to-device copy of the same size: the reference
        # dispatch that scales the byte counters
        with torch.cuda.stream(solver.ctx.stream):
            v32.copy_(u32)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "op", "kernel": OP_KERNEL, "blocks_fp32_us": t_blk * 1e6,
                          "level_cz_store": solver.info["level_cz_store"][0],
                          "level_ts_store": solver.info["level_ts_store"][0], "z_chunk_option": args.cz,
                          "reps": args.op_reps, "GBps": 8.0 * Q * N ** 3 / t_blk / 1e9,
                          "copy_bytes": u32.numel() * 4}), flush=True)
        return 0
    if args.mode == "oplist":
        import numpy as np
        rng = np.random.default_rng(1)
        probs = []
        for _ in range(64):      # the draw of uneven_batch()
            nn = int(rng.choice(BATCH_CELLS))
            kk = int(rng.integers(1, 7))
            QQ = int(rng.integers(1, 6))
            probs.append((nn, kk, QQ, float(10 ** rng.uniform(-4, -1))))
        ctxs = [R.RadauIIA(nn, kk, QQ, tt, precision=R.RK_PREC_MIXED, rtol=1e-10, restart=20, vc_streams=1)
                for nn, kk, QQ, tt in probs]
        torch.cuda.synchronize()
        r = operator_batch_leg(torch, R, ctxs, sum(QQ * (nn * kk + 1) ** 3 for nn, kk, QQ, _ in probs),
                               reps=args.op_reps)
        for c in ctxs:
            c.close()
        print(json.dumps({"mode": "oplist", **r}), flush=True)
        return 0
    if args.mode == "cala":
        # the fp64 stage operator of the Krylov method (mix pass + pair kernel)
        # and one plain device copy of the same size, for counter runs
        solver = R.RadauIIA(n, k, Q, tau, precision=R.RK_PREC_MIXED, mode=R.RK_BATCHED, restart=1,
                            eig_max=[1.0] * R.n_levels(n))
        u64 = torch.randn(Q * N ** 3, dtype=torch.float64, device="cuda")
        v64 = torch.empty_like(u64)
        t_cala = time_op(torch, R, solver.ctx, R.RK_OP_CALA, u64, v64, args.op_reps)
        with torch.cuda.stream(solver.ctx.stream):
            v64.copy_(u64)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "cala", "kernels": ["stage_mix_q_kernel<double, double, 4, false>",
                                                      "op_kernel<4, double, 1, 0, 0>"],
                          "cala_fp64_us": t_cala * 1e6, "krylov_cz": solver.info["krylov_cz"],
                          "reps": args.op_reps, "copy_bytes": u64.numel() * 8}), flush=True)
        return 0
    if args.mode == "deformed":
        # the deformed-mesh operator at Q stages (fp32, eps = 0.05) and one
        # plain device copy of the same size, for counter runs
        op = R.DeformedOperator(n, k, 0.05, dtype=torch.float32)
        u = torch.randn(Q * N ** 3, dtype=torch.float32, device="cuda")
        v = torch.empty_like(u)
        for _ in range(args.op_reps):
            op.apply(u, v, [2.0] * Q, [5e-4] * Q)
        v.copy_(u)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "deformed", "kernel": "deformed_op_kernel<4, float, false>", "Q": Q,
                          "applies": args.op_reps, "launches_per_apply": 8, "copy_bytes": u.numel() * 4,
                          "geometry_bytes": op.geometry.numel() * 4}), flush=True)
        return 0
    smoother = {}
    if args.cheb_degree is not None:
        smoother.update(cheb_degree=args.cheb_degree, coarse_cheb_degree=args.cheb_degree)
    if args.cheb_range is not None:
        smoother["cheb_range"] = args.cheb_range
    solver = R.RadauIIA(n, k, Q, tau, precision=R.RK_PREC_MIXED, mode=R.RK_BATCHED, rtol=1e-10, **smoother)
    ctx = solver.ctx
    # operator throughput: batched fp32 block operator, all Q stages per launch
    u32 = torch.randn(Q * N ** 3, dtype=torch.float32, device="cuda")
    v32 = torch.empty_like(u32)
    t_blk = time_op(torch, R, ctx, R.RK_OP_BLOCKS, u32, v32, args.op_reps)
    log(f"[bench] fp32 block operator {t_blk * 1e6:.1f} us/launch")
    del u32, v32
    u64 = torch.randn(Q * N ** 3, dtype=torch.float64, device="cuda")
    v64 = torch.empty_like(u64)
    t_cala = time_op(torch, R, ctx, R.RK_OP_CALA, u64, v64, max(5, args.op_reps // 2))
    log(f"[bench] fp64 stage operator A^-1 (x) M + tau I (x) K {t_cala * 1e6:.1f} us/launch")
    del u64, v64
    torch.cuda.empty_cache()
    sdofs = Q * N ** 3
    # z-chunk of the timed block-operator launches (tuned at create, or forced)
    cz0 = int(solver.info["level_cz_store"][0])
    ts0 = int(solver.info["level_ts_store"][0])
    x1 = grid_coords(solver.info["nodes"], n)
    y0 = torch.tensor(fourier_field(x1, seed=0), device="cuda")
    opts = solver.opts
    solver.close()
    mixed = dict(precision=R.RK_PREC_MIXED, mode=R.RK_BATCHED, **smoother)
    plain = dict(precision=R.RK_PREC_FP64, mode=R.RK_PER_STAGE, **smoother)
    # Radau IIA steps at FGMRES rtol 1e-10
    t_step, its, vcs = time_steps(torch, R, n, k, Q, tau, args.steps, args.warmup, y0, rtol=1e-10, **mixed)
    log(f"[bench] {t_step * 1e3:.2f} ms/step, FGMRES its {its}")
    # per-component breakdown of one extra step
    s = R.RadauIIA(n, k, Q, tau, rtol=1e-10, timing=1, **mixed)
    y = y0.clone()
    breakdown = s.step(0.0, y)
    s.close()
    del y
    # the plain fp64 per-stage form on the same workload
    ps = max(1, min(3, args.steps))
    t_plain, its_plain = None, None
    if not args.no_plain:
        t_plain, its_plain, _ = time_steps(torch, R, n, k, Q, tau, ps, 1, y0, rtol=1e-10, **plain)
        log(f"[bench] plain fp64 per-stage: {t_plain * 1e3:.2f} ms/step, its {its_plain}")
    # the direct complex diagonalisation with PRESB on the same workload
    cx = None
    if not args.no_complex:
        blk = []
        t_cx, its_cx, vcs_cx = time_steps(torch, R, n, k, Q, tau, args.steps, 1, y0, blocks=blk, rtol=1e-10,
                                          method=R.RK_METHOD_COMPLEX, **mixed)
        cx = {"method": "direct complex diagonalisation, per-block GMRES with PRESB (two V-cycles on "
                        "(Re lam + Im lam) M + tau K per pair)",
              "rtol": 1e-10, "ms_per_step": t_cx * 1e3, "lockstep_iterations": its_cx,
              "block_iterations": blk, "vcycle_sequences": vcs_cx}
        log(f"[bench] complex PRESB: {t_cx * 1e3:.2f} ms/step, block its {blk[-1]}")
    at_acc = None
    cpu = acc = acc64 = None
    if not args.no_cpu:
        log("[bench] host leg: cpu baseline and accuracy against the oracle on 32^3 and 64^3")
        cpu, acc, acc64 = cpu_baseline_leg(torch, R)
        r_mixed = loosest_rtol(acc["mixed_batched"], acc64["mixed_batched"])
        r_plain = loosest_rtol(acc["fp64_per_stage"], acc64["fp64_per_stage"])
        tm, im, _ = time_steps(torch, R, n, k, Q, tau, args.steps, 1, y0, rtol=r_mixed, **mixed)
        at_acc = {"bound": 1e-8, "mixed_batched": {"rtol": r_mixed, "ms_per_step": tm * 1e3, "fgmres_iterations": im}}
        log(f"[bench] at 1e-8 accuracy: mixed batched {tm * 1e3:.2f} ms (rtol {r_mixed:.0e})")
        if not args.no_plain:
            tp, ip, _ = time_steps(torch, R, n, k, Q, tau, ps, 1, y0, rtol=r_plain, **plain)
            at_acc["fp64_per_stage"] = {"rtol": r_plain, "ms_per_step": tp * 1e3, "fgmres_iterations": ip}
            at_acc["speedup"] = tp / tm
            log(f"[bench] at 1e-8 accuracy: plain fp64 per-stage {tp * 1e3:.2f} ms (rtol {r_plain:.0e})")
        if not args.no_complex:
            r_cx = loosest_rtol(acc["complex_presb_mixed_batched"], acc64["complex_presb_mixed_batched"])
            blk = []
            tc, ic, _ = time_steps(torch, R, n, k, Q, tau, args.steps, 1, y0, blocks=blk, rtol=r_cx,
                                   method=R.RK_METHOD_COMPLEX, **mixed)
            at_acc["complex_presb_mixed_batched"] = {"rtol": r_cx, "ms_per_step": tc * 1e3,
                                                     "lockstep_iterations": ic, "block_iterations": blk[-1]}
            log(f"[bench] at 1e-8 accuracy: complex PRESB {tc * 1e3:.2f} ms (rtol {r_cx:.0e})")
    y0d = y0
    del y0
    torch.cuda.empty_cache()
    fp64_32 = None
    if not args.no_fp64_32:
        def y0_fn(nn, kk):
            s_ = R.RadauIIA(nn, kk, 1, 1e-3, autotune=0, restart=1, eig_max=[1.0] * R.n_levels(nn))
            x = grid_coords(s_.info["nodes"], nn)
            s_.close()
            return torch.tensor(fourier_field(x, seed=0), device="cuda")
        fp64_32 = fp64_32cubed_legs(torch, R, y0_fn)
        log(f"[bench] 32^3 Q_4 fp64: per-stage Q=3 {fp64_32['per_stage_Q3']['ms_per_step']:.2f} ms/step; batched "
            f"Q=3 {fp64_32['batched_Q3']['ms_per_step']:.2f}, Q=5 {fp64_32['batched_Q5']['ms_per_step']:.2f} ms/step")
    batch = None
    if not args.no_batch:
        batch = uneven_batch(torch, R)
        log(f"[bench] uneven batch of {batch['problems']}: {batch['s_concurrent'] * 1e3:.1f} ms concurrent, "
            f"{batch['s_sequential'] * 1e3:.1f} ms one after another")
    deformed = None
    if not args.no_deformed:
        deformed = deformed_leg(torch, R, n=n, k=k)
        deformed["step"] = deformed_step_leg(torch, R, y0d, n=n, k=k, Q=Q, tau=tau)
        for name in ("deformed_levels", "affine_levels"):
            st = deformed["step"][name]
            log(f"[bench] deformed mesh step, V-cycles on {name}: {st['ms_per_step']:.2f} ms, "
                f"its {st['fgmres_iterations']}")
        log("[bench] deformed operator: " + ", ".join(
            f"Q={q} {v['us_per_apply']:.0f} us ({v['stage_dofs_per_s']:.3g} sDoF/s)" for q, v in deformed["by_Q"].items()))
    flop = op_flops_per_stage_dof(k)
    achieved = flop * sdofs / t_blk / 1e12
    hbm_gbs = 8.0 * sdofs / t_blk / 1e9
    out = {
        "metric": METRIC,
        "value": sdofs / t_blk,
        "unit": "stage-DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (operator); f32 V-cycle + f64 FGMRES (step)",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 hex cells, Q_4 ({N}^3 nodes/stage), Radau IIA Q={Q}, tau={tau}, "
                               f"mixed precision, batched stages",
                   "n_cells": n, "degree": k, "Q": Q, "tau": tau, "stage_dofs": sdofs,
                   "precision": "mixed", "mode": "batched", "rtol": 1e-10,
                   "cheb_degree": opts.cheb_degree, "cheb_range": opts.cheb_range},
        "s_per_step": t_step,
        "fgmres_iterations_per_step": its,
        "vcycles_per_step": vcs,
        "plain_fp64_per_stage": None if t_plain is None else {
            "ms_per_step": t_plain * 1e3, "fgmres_iterations": its_plain, "rtol": 1e-10,
            "speedup_of_mixed_batched": t_plain / t_step},
        "complex_presb": cx,
        "deformed_operator": deformed,
        "at_1e-8_accuracy": at_acc,
        "uneven_batch": batch,
        "fp64_32cubed": fp64_32,
        "step_breakdown_s": {k2: breakdown[k2] for k2 in ("t_rhs", "t_vmult", "t_basis", "t_blocks", "t_rest")},
        "operators": {
            "blocks_fp32_us": t_blk * 1e6,
            "blocks_fp32_stage_dofs_per_s": sdofs / t_blk,
            "cala_fp64_us": t_cala * 1e6,
            "cala_fp64_stage_dofs_per_s": sdofs / t_cala,
            "cala_fp64_GBps": 16.0 * sdofs / t_cala / 1e9,
        },
        "roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(cz0, ts0),
                     "algorithmic_bytes_per_launch": 8 * sdofs, "bytes_per_stage_dof": 8,
                     "z_chunk": cz0, "tile_shape": ts0,
                     "kernel": OP_KERNEL + " (batched block operator, all Q stages per launch)",
                     "avg_launch_us": t_blk * 1e6,
                     "alu": {"achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / ALU_PEAK_TFLOPS, "flop_per_stage_dof": flop,
                             "algorithmic_flop_per_launch": flop * sdofs}},
    }
    if cpu is not None:
        out["accuracy_vs_oracle"] = acc
        out["accuracy_vs_oracle_64cubed"] = acc64
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
