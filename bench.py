"""Benchmark of the batched forward model + ABC on one MI355X.

Workload ("batch"): 4096 ABC parameter sets drawn from the uniform prior
alpha in [0, 10], S_b in [0.01, 1], S_s in [1e2, 1e4] (Philox seed 1); every
swimmer has N = 128 points and runs to T = 0.25 in 10000 forward-Euler
steps of dt = 2.5e-5, its head observed every 200 steps (the data's 50
times); FP32; the paper's blob (eq. eqnblob, the library's default).  The
workload as first stated takes 5000 steps of 5e-5: with the paper's blob
the data's own parameters (2, 0.1, 1e3) are beyond forward Euler's
stability bound there and blow up at step 40, so the step is halved over
the same time.  One bench step is one pass of the hot path over that
batch: the per-system set-up (constants and the FP32 kernel tables of the
paper's blob), then preferred curvature, elastic forces, dense
regularized-Brinkmanlet velocity sum, Euler update and observations for all
4096 swimmers (one persistent kernel), then the ABC distances against the
observed data, the 5th-percentile tolerance and the accept mask.  Inputs are
resident in device memory before the timed region.

Prints one JSON line.  value = Brinkmanlet pair evaluations per second
(ordered pairs i, j of one system, self included, per completed Euler step;
runs that blow up count only the steps they computed).  The line also
carries the surrogate-prescreened ABC comparison (accepted samples per
second of both methods on the same 1M prior draws; --no-surrogate skips it).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the dominant kernel (the persistent forward kernel), in FP32
# FLOP against the FP32 vector peak of 157.3 TFLOP/s.  Algorithmic work per
# ordered pair evaluation of eq. (BrV) in its FP32 form: per distinct pair
# (one evaluation serves both ends, symmetric schedule) the difference
# vector (2), v = |d|^2 + 1 (2 FMA), the two cubics of the table (6 FMA),
# and for each end F.d times H2 (MUL, FMA, MUL) and the two accumulations
# (4 FMA): 42 FLOP (FMA = 2) per distinct pair, 21 per ordered pair.  The
# kernel is bound by VALU instruction issue, not FLOP: integer and float
# operations share the issue slots.  rocprofv3's SQ_INSTS_VALU over the
# launch gives 17.8 VALU lane-operations per ordered pair evaluation, all
# work of the step included (the symmetric pair loop alone is 14.75 in the
# ISA); the issue peak without packed FP32 is 256 CUs x 4 SIMDs x 16 lanes
# per clock x 2.4 GHz = 39.3e12 lane-operations/s, i.e. 78.6 TFLOP/s of FMA
# (the build keeps packed FP32 off).
# (profiles/k_forward_batch_4096x128_counters.md)
VALU_OPS_PER_PAIR = 17.8
PAIR_LOOP_VALU_OPS = 15.75  # the sperm kernel's symmetric pair loop alone (ISA, per ordered pair)
FP32_FLOP_PER_PAIR = 21
NONPACKED_FP32_PEAK_TFLOPS = 78.6
# the FP32 large-system step, k_big_pairs (every pair once for both points,
# FP64 accumulation) and k_big_update: 26.2 VALU lane-operations per ordered
# pair evaluation from SQ_INSTS_VALU
# (profiles/k_big_pairs_dense_64x8x512_counters.md; the one-sided
# k_big_step<float, 1> it replaced took 39.9)
VALU_OPS_PER_PAIR_BIG = 26.2
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3
# HBM bytes of one launch of that kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch: 46324.6 and 2227.1) scaled by
# the same counters over a 256 MiB device copy (x2.0 and x1.0), for the
# kernel as it stands (profiles/k_forward_batch_4096x128_counters.md): almost
# all of it the 4096 kernel tables (22.5 KiB each) read once into LDS; set
# it to None whenever the kernel changes until the counters are taken again
TRAFFIC_BYTES = (46324.6 * 2.00 + 2227.1 * 1.00) * 1024


def load_data():
    path = os.path.join(ROOT, "tests", "golden", "abc_data_batch.txt")
    a = np.loadtxt(path)
    return a[:, :2]


def cpu_model():
    """The host CPU model (lscpu), or the platform's processor string."""
    import platform
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or "unknown"


def cpu_baseline(steps_cpu):
    """The FP64 oracle as it stands, timed on the host cores on bounded
    samples of the workloads (its paper-blob kernel integrates every pair at
    alpha > 0, about 1 ms per pair on one core):
      batch  one swimmer of the batched workload at the data's parameters
             (alpha = 2), N = 128, the paper's blob, steps_cpu of its 10000
             steps, all threads: the reported value;
      single the single-swimmer workload on one core: N = 64, alpha = 1
             (quadrature) for 3 of its 2000 steps (extrapolated to 2000),
             and alpha = 0 (closed forms) in full;
      dense  one velocity evaluation of the dense workload's sample 0
             (8 x 512 points, its alpha), at 32 of its 4096 targets, all
             threads.
    The batched workload's 64-particle subset (10000 steps each) would take
    about 1e10 pair quadratures, days on these cores: the batch sample's rate
    stands for it."""
    from oracle import core
    from paper_1910_12007_amd import inputs
    core.lib()
    threads = core.num_threads()
    out = {"kind": "oracle", "cores": threads, "cpu_model": cpu_model(), "legs": {}}
    P = inputs.theta_rows(inputs.TRUE_THETA)
    t0 = time.perf_counter()
    core.forward(P, 128, steps_cpu, inputs.BATCH_DT, 100)
    sec = time.perf_counter() - t0
    out["value"] = 128 * 128 * steps_cpu / sec
    out["unit"] = "pair-evals/s"
    out["sample"] = (f"1 swimmer of the batched workload (alpha, S_b, S_s = 2, 0.1, 1e3), N=128, paper's blob, "
                     f"{steps_cpu} of {inputs.BATCH_STEPS} steps, FP64, {sec:.1f} s on {threads} threads")
    core.set_threads(1)
    try:
        single = {}
        for alpha, k in ((1.0, 3), (0.0, 2000)):
            Ps = inputs.param_rows(1, alpha=alpha)
            t0 = time.perf_counter()
            core.forward(Ps, 64, k, 1e-4, 100)
            sec = time.perf_counter() - t0
            single[f"alpha_{alpha:g}"] = {"steps": k, "seconds": sec, "pair_evals_per_s": 64 * 64 * k / sec,
                                          "run_2000_steps_s_extrapolated": sec * 2000 / k}
        out["legs"]["single_1_core"] = single
    finally:
        core.set_threads(threads)
    lay = inputs.dense_layout(n_samples=1, seed=3)[0]
    x = np.concatenate([lay[m, 7] + np.arange(512) / 511.0 for m in range(8)])
    y = np.concatenate([np.full(512, lay[m, 8]) for m in range(8)])
    F = [core.forces(x[512 * m:512 * (m + 1)], y[512 * m:512 * (m + 1)], lay[m, 1], lay[m, 2],
                     core.kappa0(512, lay[m, 3], lay[m, 5], lay[m, 4], lay[m, 6], 0.0)) for m in range(8)]
    fx, fy = np.concatenate([f[0] for f in F]), np.concatenate([f[1] for f in F])
    idx = np.arange(0, 4096, 128)
    t0 = time.perf_counter()
    core.velocity_at(x, y, fx, fy, lay[0, 0], 1.5 / 511, idx)
    sec = time.perf_counter() - t0
    out["legs"]["dense_sample0"] = {"targets": int(idx.size), "sources": 4096, "alpha": float(lay[0, 0]),
                                    "seconds": sec, "pair_evals_per_s": idx.size * 4096 / sec,
                                    "one_step_s_extrapolated": sec * 4096 / idx.size}
    return out


# weights of the surrogate MLP 5 -> 256 x 4 -> 33 (multiply-adds per row)
MLP_MACS = 5 * 256 + 3 * 256 * 256 + 256 * 33
BF16_PEAK_TFLOPS = 2500.0


def mlp_leg(ctx, stream, rows=1 << 20, train_rows=65536, batch=1024, epochs=2):
    """BF16 MFMA throughput of the surrogate kernels: a forward pass over
    `rows` inputs (the prescreen's GEMMs) and Adam training steps of
    `batch` rows, timed with HIP events on the library's stream.
    Algorithmic FLOP: 2 per multiply-add of the unpadded layers; a training
    step is a forward and a backward pass (3x the forward's GEMM work)."""
    import torch
    from paper_1910_12007_amd import inputs, swim
    g = torch.Generator().manual_seed(7)
    X = torch.randn(rows, 5, generator=g).to("cuda")
    Y = torch.empty(rows, 33, device="cuda")
    Xt = X[:train_rows].contiguous()
    Tt = torch.randn(train_rows, 33, generator=g).to("cuda")
    params = torch.from_numpy(inputs.mlp_init(0)[1]).to("cuda")
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    perm = torch.from_numpy(inputs.epoch_permutations(train_rows, epochs, 7)).to("cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    swim.surrogate_forward(ctx, X, params, Y, stream=stream)  # warm-up
    ev[0].record(stream)
    swim.surrogate_forward(ctx, X, params, Y, stream=stream)
    ev[1].record(stream)
    ev[2].record(stream)
    swim.surrogate_train(ctx, Xt, Tt, perm, epochs, batch, 1e-3, params, m, v, stream=stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    fwd_ms, train_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    steps = epochs * (train_rows // batch)
    fwd_tf = 2.0 * MLP_MACS * rows / (fwd_ms * 1e-3) / 1e12
    train_tf = 6.0 * MLP_MACS * batch * steps / (train_ms * 1e-3) / 1e12
    return {"forward_rows": rows, "forward_ms": fwd_ms, "forward_tflops": fwd_tf,
            "train_steps": steps, "train_batch": batch, "train_ms": train_ms, "train_tflops": train_tf,
            "peak_tflops": BF16_PEAK_TFLOPS, "forward_frac": fwd_tf / BF16_PEAK_TFLOPS,
            "train_frac": train_tf / BF16_PEAK_TFLOPS, "dtype": "bf16 operands, fp32 accumulation"}


def dense_leg(ctx, stream, samples=64, steps=1000, dt_div=64):
    """Large-N dense workload: `samples` independent systems of 8 interacting
    swimmers of N = 512 (4096 points) on a 2 x 4 grid of spacing 1.5, random
    beat phases, alpha ~ U[0, 10] (seed 3), FP32.  The stated dt = 2e-5 is
    beyond forward Euler's stability bound at N = 512 (dt * rho ~ 51 with the
    other blob, ~1.4 times more with the paper's, whose H1(0) - H1(ds) is
    larger), so the run uses a stable power-of-two fraction: dt / 64 (with
    the paper's blob 56 of 64 samples blow up within 50 steps at dt / 32,
    none in 1000 at dt / 48 or dt / 64); the work per step does not depend
    on dt.  Runs on the FP32 large-system step (per step: the tile-pair
    kernel, every pair once for both points, then the update kernel).
    (The parity of one full-size velocity evaluation against the FP64
    oracle is a test: test_dense_sample_velocity_at_full_size.)"""
    import torch
    from paper_1910_12007_amd import inputs, swim
    lay = inputs.dense_layout(n_samples=samples, seed=3)
    P = torch.from_numpy(lay.reshape(-1, 9)).to("cuda")
    N = np.full(samples, 512, np.int32)
    nsw = np.full(samples, 8, np.int32)
    dt = 2e-5 / dt_div
    nfil = samples * 8
    oe = min(100, steps)
    obs = torch.empty((nfil, steps // oe, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(nfil, dtype=torch.float32, device="cuda")
    status = torch.empty(samples, dtype=torch.int32, device="cuda")
    done = torch.empty(samples, dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    warm = torch.empty((nfil, 1, 2), dtype=torch.float32, device="cuda")
    swim.swim_forward(ctx, N, nsw, P, 10, dt, 10, 1.5, warm, speed, status, done, stream=stream)  # warm-up
    ev[0].record(stream)
    swim.swim_forward(ctx, N, nsw, P, steps, dt, oe, 1.5, obs, speed, status, done, stream=stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    d = done.cpu().numpy().astype(np.int64)
    pairs = float(np.sum(d * 4096 * 4096))
    out = {"workload": f"{samples} samples x 8 swimmers x N=512 (2x4 grid, spacing 1.5), {steps} Euler steps of "
                       f"dt=2e-5/{dt_div} (stability), FP32, symmetric large-system step (k_big_pairs + k_big_update)",
           "ms": ms, "pair_evals_per_s": pairs / (ms * 1e-3), "swimmer_steps_per_s": float(np.sum(d)) * 8 / (ms * 1e-3),
           "runs_stopped": int(np.sum(status.cpu().numpy() != 0)),
           "fp32_tflops": FP32_FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12,
           "fp32_frac": FP32_FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
           "valu_tops": VALU_OPS_PER_PAIR_BIG * pairs / (ms * 1e-3) / 1e12, "valu_peak_tops": VALU_PEAK_TOPS,
           "valu_issue_frac": VALU_OPS_PER_PAIR_BIG * pairs / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS,
           "valu_ops_per_pair": VALU_OPS_PER_PAIR_BIG}
    return out


def per_sample_leg(ctx, stream, P_all, n=256, N=128, steps=None, dt=None):
    """The batched generation's first n draws as one fused persistent launch
    against one launch per sample (each a batch of one system), both on the
    library's path with inputs resident; HIP events on the same stream."""
    import torch
    from paper_1910_12007_amd import inputs, swim
    steps = steps or inputs.BATCH_STEPS
    dt = dt or inputs.BATCH_DT
    oe = inputs.BATCH_OBS_EVERY
    P = P_all[:n].contiguous()
    obs = torch.empty((n, steps // oe, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    graph_mode = swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH)
    swim.swim_set_option(ctx, swim.SWIM_OPT_GRAPH, 0)
    try:
        swim.swim_forward(ctx, np.full(n, N, np.int32), None, P, steps, dt, oe, 1.5, obs, speed, status,
                          stream=stream)
        ev[0].record(stream)
        swim.swim_forward(ctx, np.full(n, N, np.int32), None, P, steps, dt, oe, 1.5, obs, speed, status,
                          stream=stream)
        ev[1].record(stream)
        ev[2].record(stream)
        for i in range(n):
            swim.swim_forward(ctx, np.full(1, N, np.int32), None, P[i:i + 1], steps, dt, oe, 1.5, obs[i:i + 1],
                              speed[i:i + 1], status[i:i + 1], stream=stream)
        ev[3].record(stream)
        torch.cuda.synchronize()
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_GRAPH, graph_mode)
    fused, single = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    return {"draws": n, "fused_ms": fused, "per_sample_launches_ms": single, "speedup": single / fused}


def pmc_leg(ctx, data, n=16384, steps=None, dt=None, quantiles=(0.5, 0.25, 0.1)):
    """Uneven batching with population Monte Carlo: n particles, each with
    its own filament size N ~ U{64, 96, ..., 512} (seed 2) and the batched
    workload's priors, steps and dt; three generations at the 50th, 25th and
    10th percentile tolerances (Philox seed 2).  The launch shapes come from
    the autotuner run on generation 0's draws; each generation is one
    abc_step (host proposals and weights in FP64, FP32 forward runs, device
    distances and percentile), its forward runs replayed from a captured
    graph once the layout repeats."""
    import torch
    from paper_1910_12007_amd import inputs, swim, surrogate_abc
    steps = steps or inputs.BATCH_STEPS
    dt = dt or inputs.BATCH_DT
    N = inputs.uneven_sizes(n, seed=2)
    model = surrogate_abc.batch_model(steps=steps, dt=dt)
    theta0 = swim.abc_prior_draw(2, n, inputs.PRIOR_LO, inputs.PRIOR_HI)
    t0 = time.perf_counter()
    chosen = swim.swim_autotune(ctx, swim.SWIM_F32, N, None, torch.from_numpy(inputs.theta_rows(theta0)).cuda(),
                                50, dt)
    tune_s = time.perf_counter() - t0
    gens = []
    prev_theta = prev_w = None
    for g, q in enumerate(quantiles):
        t0 = time.perf_counter()
        r = swim.abc_step(ctx, model, data, N, 2, g, q, prev_theta, prev_w)
        sec = time.perf_counter() - t0
        steps_done = r["steps"].astype(np.int64)
        pairs = float(np.sum(steps_done * N.astype(np.int64) ** 2))
        acc = r["accept"]
        gens.append({"generation": g, "quantile": q, "seconds": sec, "tolerance": r["tol"],
                     "completed": int(np.isfinite(r["dist"]).sum()), "accepted": int(acc.sum()),
                     "pair_evals_per_s": pairs / sec, "swimmer_steps_per_s": float(np.sum(steps_done)) / sec,
                     "posterior_mean": [float(x) for x in np.average(r["theta"][acc], axis=0, weights=r["w"][acc])]
                     if acc.any() else None})
        prev_theta, prev_w = r["theta"][acc], r["w"][acc]
    return {"workload": f"{n} particles, N ~ U{{64..512 step 32}} (seed 2), {steps} steps dt={dt}, PMC generations "
                        f"at quantiles {list(quantiles)}, FP32",
            "autotune_s": tune_s, "tuned_waves_per_system": {str(k): v for k, v in chosen["wps"].items() if v},
            "graph_launches": swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_LAUNCHES), "generations": gens}


def tmcmc_leg(ctx, data, n=2048, seed=7):
    """TMCMC (the paper's sampler) on the batched workload's model and data:
    n samples per stage (the paper takes 2000), (alpha, S_b, S_s) on the
    batched workload's prior box and the noise standard deviation sigma on
    [1e-4, 1e-2]; FP32 forward runs, one batched launch per Metropolis step
    across all chains.  Reports the stages, forward runs and their rate, and
    the final-stage posterior against the parameters the data were made
    with (2, 0.1, 1e3, sigma = 1e-3)."""
    from paper_1910_12007_amd import inputs, swim, surrogate_abc
    model = surrogate_abc.batch_model()
    lo = np.append(inputs.PRIOR_LO, 1e-4)
    hi = np.append(inputs.PRIOR_HI, 1e-2)
    t0 = time.perf_counter()
    r = swim.tmcmc_run(ctx, model, lo, hi, data, 128, n, seed, cv_target=1.0, cov_scale=0.2, max_stages=60)
    wall = time.perf_counter() - t0
    th = r["theta"]
    truth = np.append(inputs.TRUE_THETA, 1e-3)
    return {"workload": f"TMCMC, {n} samples per stage, N=128, {model.steps} steps dt={model.dt}, FP32, "
                        "theta = (alpha, S_b, S_s, sigma), data of the batched workload",
            "stages": r["n_stages"], "q": [float(x) for x in r["q"]], "forward_runs": r["runs"],
            "seconds": wall, "forward_seconds": r["seconds"], "forward_runs_per_s": r["runs"] / r["seconds"],
            "accepted_per_stage": [int(x) for x in r["accepted"]], "log_evidence": r["log_evidence"],
            "posterior_mean": th.mean(0).tolist(), "posterior_std": th.std(0).tolist(),
            "true": truth.tolist(),
            "z_scores_of_truth": ((truth - th.mean(0)) / th.std(0)).tolist()}


def sperm_leg(ctx, stream, n=2000, steps=20000, dt=1e-5):
    """Full sperm model (Appendix, Table Tab:param): one TMCMC stage's batch
    of the paper's experiments, n = 2000 systems with (alpha, K_C) ~
    U[0,2] x U[0,16] (seed 11), FP32, dt = 1e-5 (the Table's stiffnesses
    diverge at the Table's dt).  The paper's run to T = 20 is 2M steps; the
    leg times `steps` of them, all identical in work, and states the
    extrapolation to a whole stage.  Configurations: one swimmer (74 points)
    and two swimmers with head centres 0.5 apart (148 points).

    Roofline: VALU issue bound.  Algorithmic work is n_pts^2 ordered pairs
    per system step at PAIR_LOOP_VALU_OPS lane-operations each (the
    symmetric pair loop's cost per ordered pair; the point phase of the
    step, with its head and neck terms, comes on top)."""
    import torch
    from paper_1910_12007_amd import inputs, swim
    rows = torch.from_numpy(inputs.sperm_rows(n, seed=11)).to("cuda")
    out = {"workload": f"full sperm model, {n} systems (alpha, K_C) ~ U[0,2]xU[0,16], FP32, {steps} Euler steps "
                       f"of dt={dt} (T = 20 needs {int(round(20 / dt))})"}
    for n_swim in (1, 2):
        sw = torch.from_numpy(inputs.sperm_swimmers(n, n_swim, 0.5)).to("cuda")
        oe = steps // 50
        head = torch.empty((n * n_swim, 51, 2), dtype=torch.float32, device="cuda")
        tail = torch.empty_like(head)
        status = torch.empty(n, dtype=torch.int32, device="cuda")
        shape = swim.sperm_shape(n_swim=n_swim)
        swim.swim_sperm_forward(ctx, swim.SWIM_F32, shape, rows, sw, 100, dt, 2, head, tail, status,
                                stream=stream)  # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        swim.swim_sperm_forward(ctx, swim.SWIM_F32, shape, rows, sw, steps, dt, oe, head, tail, status, stream=stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        npts = n_swim * 74
        st = status.cpu().numpy()
        pairs = float(n) * npts * npts * steps
        tops = PAIR_LOOP_VALU_OPS * pairs / (ms * 1e-3) / 1e12
        tflops = FP32_FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12
        out[f"{n_swim}_swimmer" + ("s" if n_swim > 1 else "")] = {
            "points_per_system": npts, "ms": ms, "us_per_step": 1e3 * ms / steps,
            "pair_evals_per_s": pairs / (ms * 1e-3), "swimmer_steps_per_s": float(n) * n_swim * steps / (ms * 1e-3),
            "runs_stopped": int(np.sum(st != 0)),
            "stage_seconds_to_T20": ms * 1e-3 * (20 / dt) / steps,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP32_PEAK_TFLOPS,
                         "kernel": "k_sperm_forward<float,%d,2>" % (1 if npts <= 64 else 2 if npts <= 128 else 3),
                         "fp32_flop_per_pair": FP32_FLOP_PER_PAIR, "pair_loop_valu_ops": PAIR_LOOP_VALU_OPS,
                         "pair_loop_valu_issue_frac": tops / VALU_PEAK_TOPS}}
    return out


def sperm_tmcmc_leg(ctx, n=2000, steps=10000, obs_every=200, dt=1e-5, seed=17, noise=0.01):
    """The paper's Sec. 4.1 experiment on the full sperm model: TMCMC with
    n = 2000 samples per stage over theta = (alpha, sigma/beta), prior
    [0, 2] x [0, 0.5], 50 head-centre velocity pairs as data, 1 % noise,
    FP32 forward runs.  The horizon is shortened to T = steps * dt = 0.1
    (the paper runs to T = 20, 2M steps at this dt).  The synthetic data
    are the library's FP64 run of the nominal model (alpha = 1, K_C = 8)
    plus seeded Gaussian noise of sigma = noise * |mean of the outputs|."""
    import torch
    from paper_1910_12007_amd import inputs, swim
    shape = swim.sperm_shape()
    row = inputs.sperm_rows(1)[0]
    sw = inputs.sperm_swimmers(1)
    n_obs = steps // obs_every
    head = torch.empty((1, n_obs + 1, 2), dtype=torch.float64, device="cuda")
    tail = torch.empty_like(head)
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    g = torch.empty((1, n_obs, 2), dtype=torch.float64, device="cuda")
    swim.swim_sperm_forward(ctx, swim.SWIM_F64, shape, torch.from_numpy(row[None].copy()).cuda(),
                            torch.from_numpy(sw).cuda(), steps, dt, obs_every, head, tail, status)
    swim.swim_sperm_observables(ctx, swim.SWIM_F64, swim.SWIM_OBS_HEAD_VELOCITY, 1, obs_every * dt, head, tail,
                                status, g)
    torch.cuda.synchronize()
    xi = g.cpu().numpy()[0]
    beta = abs(float(xi.mean()))
    data = xi + noise * beta * np.random.Generator(np.random.PCG64(seed)).normal(size=xi.shape)
    m = swim.sperm_model(shape, row, ("alpha",), 1, swim.SWIM_OBS_HEAD_VELOCITY, (beta, beta), steps, obs_every, dt,
                         swim.SWIM_F32)
    t0 = time.perf_counter()
    r = swim.tmcmc_sperm_run(ctx, m, sw, [0.0, 0.0], [2.0, 0.5], data, n, seed, max_stages=40)
    wall = time.perf_counter() - t0
    th = r["theta"]
    mean, std = th.mean(0), th.std(0)
    truth = np.array([1.0, noise])
    return {"workload": f"TMCMC over the full sperm model (Sec. 4.1): {n} samples per stage, theta = (alpha, "
                        f"sigma/beta) on [0,2]x[0,0.5], {n_obs} head-centre velocity pairs, {noise:.0%} noise, "
                        f"T = {steps * dt:g} ({steps} steps of dt = {dt}), FP32 forward runs",
            "stages": r["n_stages"], "q": [float(x) for x in r["q"]], "forward_runs": r["runs"], "seconds": wall,
            "forward_seconds": r["seconds"], "forward_runs_per_s": r["runs"] / r["seconds"],
            "swimmer_steps_per_s": r["runs"] * steps / r["seconds"],
            "accepted_per_stage": [int(x) for x in r["accepted"]], "log_evidence": r["log_evidence"],
            "posterior_mean": [float(x) for x in mean], "posterior_std": [float(x) for x in std],
            "true": [float(x) for x in truth], "z_scores_of_truth": [float(x) for x in (truth - mean) / std]}


def field_leg(ctx, stream, grid=1024):
    """Flow and pressure picture (Sec. 2.1, eqs. BrV, BrP; Figs. 1 and 3):
    velocity and pressure of two swimmers' point forces (2 x 128 points,
    forces of a bent configuration, alpha = 1) on a grid x grid lattice of
    targets, FP32 pair kernel from the system's table, FP64 sums and
    pressure weights."""
    import torch
    from paper_1910_12007_amd import inputs, swim
    N = 128
    x, y = inputs.filament_geometry(N, 5, n_swim=2, spacing=0.5)
    rng = np.random.Generator(np.random.PCG64(5))
    f = rng.normal(size=(2, x.size))
    f -= f.mean(axis=1, keepdims=True)
    gx, gy = np.meshgrid(np.linspace(-0.5, 1.5, grid), np.linspace(-0.5, 1.0, grid))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")
    X, Y, FX, FY, TX, TY = map(d, (x, y, f[0], f[1], gx.ravel(), gy.ravel()))
    u = torch.empty(grid * grid, dtype=torch.float32, device="cuda")
    v, p = torch.empty_like(u), torch.empty_like(u)
    swim.swim_flow_field(ctx, X, Y, FX, FY, 1.0, 1.5 / (N - 1), TX, TY, u, v, p, stream=stream)  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    swim.swim_flow_field(ctx, X, Y, FX, FY, 1.0, 1.5 / (N - 1), TX, TY, u, v, p, stream=stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    pairs = float(grid * grid) * x.size
    return {"workload": f"velocity and pressure of 2 x {N} point forces on a {grid}x{grid} grid, alpha = 1, FP32",
            "ms": ms, "target_source_pairs_per_s": pairs / (ms * 1e-3)}


def reading_blob_leg(ctx, stream, Ns, P, steps, dt, obs_every, paper_ms):
    """The headline generation with the other blob of the library, the
    reading's unit-mass blob (closed forms for every alpha), at the same
    prior draws, for comparison with the default (the paper's blob, eq.
    eqnblob).  Both read per-system FP32 tables, so a run step costs the
    same; the difference is the per-system set-up: a one-step run with each
    blob.  Also the FP64 direct evaluation with each blob (the paper's
    integrates every pair: a reference mode)."""
    import torch
    from paper_1910_12007_amd import swim
    n = len(Ns)
    speed = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    one = torch.empty((n, 1, 2), dtype=torch.float32, device="cuda")
    obs = torch.empty((n, steps // obs_every, 2), dtype=torch.float32, device="cuda")

    def timed(blob, k, every, o):
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, blob)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        swim.swim_forward(ctx, Ns, None, P, k, dt, every, 1.5, o, speed, status, done, stream=stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])

    m = 512
    rng = np.random.Generator(np.random.PCG64(11))
    pts = [torch.from_numpy(a).to("cuda") for a in (rng.uniform(0, 1, m), rng.uniform(0, 0.3, m),
                                                   rng.normal(size=m), rng.normal(size=m))]
    ux, uy = torch.empty_like(pts[0]), torch.empty_like(pts[0])

    def timed_f64(blob):
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, blob)
        swim.swim_pair_velocity(ctx, np.array([0, m]), [1.0], [0.02], *pts, ux, uy, stream=stream)  # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        swim.swim_pair_velocity(ctx, np.array([0, m]), [1.0], [0.02], *pts, ux, uy, stream=stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])

    try:
        timed(swim.SWIM_BLOB_READING, 1, 1, one)  # warm-up
        one_reading = min(timed(swim.SWIM_BLOB_READING, 1, 1, one) for _ in range(2))
        one_paper = min(timed(swim.SWIM_BLOB_PAPER, 1, 1, one) for _ in range(2))
        ms = timed(swim.SWIM_BLOB_READING, steps, obs_every, obs)
        f64_paper = timed_f64(swim.SWIM_BLOB_PAPER)
        f64_reading = timed_f64(swim.SWIM_BLOB_READING)
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_PAPER)
    done_h = done.cpu().numpy().astype(np.int64)
    pairs = float(np.sum(done_h * Ns.astype(np.int64) ** 2))
    return {"workload": f"the headline generation ({n} prior draws, N={int(Ns[0])}, {steps} steps) with the "
                        "reading's blob (closed forms)",
            "ms": ms, "paper_blob_ms": paper_ms, "one_step_ms": one_reading, "one_step_paper_ms": one_paper,
            "paper_setup_extra_ms": one_paper - one_reading,
            "pair_evals_per_s": pairs / (ms * 1e-3), "runs_stopped": int((status != 0).sum().item()),
            "fp64_direct": {"workload": f"one FP64 velocity sum of {m} points, alpha = 1, eps = 0.02",
                            "paper_ms": f64_paper, "reading_ms": f64_reading,
                            "paper_pair_evals_per_s": m * m / (f64_paper * 1e-3),
                            "reading_pair_evals_per_s": m * m / (f64_reading * 1e-3)}}


def surrogate_leg(ctx, data):
    """Surrogate-prescreened ABC against plain batched ABC on the same 1M
    prior draws (tolerance: the 5th percentile of the completed runs of the
    4096-draw batch; MLP trained on 65536 completed runs)."""
    from paper_1910_12007_amd import surrogate_abc
    r = surrogate_abc.run(ctx, data)
    s, p, t = r["surrogate"], r["plain"], r["training"]
    return {
        "tolerance": r["tol"], "prescreen_factor": r["factor"], "proposals": s["proposals"],
        "plain_accepted": p["accepted"], "plain_seconds": p["seconds"], "plain_accepts_per_s": p["accepts_per_s"],
        "survivors": s["survivors"], "surrogate_accepted": s["accepted"], "prescreen_ms": s["ms_prescreen"],
        "rerun_ms": s["ms_rerun"], "surrogate_accepts_per_s": s["accepts_per_s"], "gain": r["gain"],
        "recall": s["recall"], "accepted_not_in_plain": s["not_in_plain"],
        "posterior_mean_rel_err": [float(x) for x in r["mean_rel_err"]],
        "intervals_overlap": [bool(x) for x in r["intervals_overlap"]],
        "posterior_mean_plain": [float(x) for x in p["post"]["mean"]],
        "posterior_mean_surrogate": [float(x) for x in s["post"]["mean"]],
        "training_rows": t["rows"], "training_draws": t["draws"], "training_steps": t["steps"],
        "training_set_s": t["t_data"], "training_s": t["t_train"],
        "surrogate_accepts_per_s_with_training": s["accepts_per_s_with_training"],
        "gain_with_training": r["gain_with_training"],
        "stopped_early": s["stopped_early"], "rerun_ms_without_early_stop": s["ms_rerun_without_early_stop"],
        "gain_without_early_stop": r["gain_without_early_stop"],
        "same_accepted_without_early_stop": s["same_accepted_without_early_stop"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--euler-steps", type=int, default=0, help="0: the workload's 10000 steps")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--wps", type=int, default=0, help="waves per system (0: library default)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-prescreened ABC comparison")
    ap.add_argument("--no-dense", action="store_true", help="skip the large-N dense workload")
    ap.add_argument("--no-pmc", action="store_true", help="skip the uneven-N PMC workload")
    ap.add_argument("--no-tmcmc", action="store_true", help="skip the TMCMC run")
    ap.add_argument("--no-sperm", action="store_true", help="skip the full sperm-model workload")
    ap.add_argument("--sperm-tmcmc", action="store_true",
                    help="also run TMCMC over the full sperm model on synthetic head-velocity data (the paper's "
                         "Sec. 4.1 set-up; its FP64 data run takes ~15 s)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (3 times), the reference "
                         "for scaling the HBM byte counters, and exit")
    ap.add_argument("--dense-only", type=int, default=0, metavar="STEPS",
                    help="only run the large-N dense workload for this many Euler steps (for profiling "
                         "its kernel), print its record and exit")
    ap.add_argument("--dense-div", type=int, default=64, help="the dense workload's dt is 2e-5 / this")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the swimmer batches are "
              "independent, so the workload is measured as one GPU's share of it.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}), flush=True)
        return

    from paper_1910_12007_amd import inputs, swim

    ctx = swim.Context(0)
    # a stream of our own: the library runs on it and the events time it
    stream = torch.cuda.Stream()
    if args.dense_only:
        print(json.dumps(dense_leg(ctx, stream, steps=args.dense_only, dt_div=args.dense_div)), flush=True)
        ctx.close()
        return
    n, N = args.n, 128
    steps, dt, obs_every = inputs.BATCH_STEPS, inputs.BATCH_DT, inputs.BATCH_OBS_EVERY
    if args.euler_steps:
        steps = args.euler_steps
        obs_every = min(obs_every, steps)
    n_obs = steps // obs_every
    theta = swim.abc_prior_draw(1, n, inputs.PRIOR_LO, inputs.PRIOR_HI)
    P = torch.from_numpy(inputs.theta_rows(theta)).to("cuda")
    Ns = np.full(n, N, np.int32)
    data = torch.from_numpy(np.ascontiguousarray(load_data()[:n_obs])).to("cuda")
    obs = torch.empty((n, n_obs, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    dist = torch.empty(n, dtype=torch.float64, device="cuda")
    tol = torch.empty(1, dtype=torch.float64, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")

    ev = []

    def step(record):
        if record:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
        swim.swim_forward(ctx, Ns, None, P, steps, dt, obs_every, 1.5, obs, speed, status, done, stream=stream)
        if record:
            b.record(stream)
            ev.append((a, b))
        swim.abc_distance(ctx, obs, data, status, dist, stream=stream)
        swim.abc_select(ctx, dist, 0.05, tol, acc, stream=stream)

    if args.wps:
        swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, args.wps)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    done_h = done.cpu().numpy().astype(np.int64)
    pairs = float(np.sum(done_h * N * N))
    swimmer_steps = float(np.sum(done_h))
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    n_acc = int(acc.sum().item())
    st = status.cpu().numpy()
    # the forward call = per-system set-up + the persistent kernel.  The
    # kernel's own launch time: the same calls again with the library's
    # timing events recorded right before and after the persistent launch,
    # on the stream it runs on (SWIM_OPT_TIME_KERNEL; those calls launch
    # eagerly instead of replaying the captured graph)
    # The set-up is the whole call less the launch, both taken on these
    # same calls (the launch alone varies by a few percent between calls)
    swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, 1)
    kus, calls = [], []
    for _ in range(max(3, args.steps)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        swim.swim_forward(ctx, Ns, None, P, steps, dt, obs_every, 1.5, obs, speed, status, done, stream=stream)
        b.record(stream)
        kus.append(swim.swim_get_option(ctx, swim.SWIM_OPT_KERNEL_US))
        calls.append((a, b))
    swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, 0)
    torch.cuda.synchronize()
    kernel_ms = float(np.mean(kus)) * 1e-3
    setup_ms = float(np.mean([a.elapsed_time(b) for a, b in calls])) - kernel_ms
    tflops = FP32_FLOP_PER_PAIR * pairs / (kernel_ms * 1e-3) / 1e12
    issue = VALU_OPS_PER_PAIR * pairs / (kernel_ms * 1e-3) / 1e12
    out = {
        "metric": "swimmer steps/s & Brinkmanlet pair-evals/s; ABC accepts/s surrogate vs plain",
        "value": pairs * args.steps / wall,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched ABC forward generation with the paper's blob (eq. eqnblob): {n} prior "
                               f"draws, N={N}, {steps} Euler steps dt={dt}, head every {obs_every} steps, RMS "
                               "distance, 5th-percentile tolerance",
                   "particles": n, "N": N, "euler_steps": steps, "blob": "paper (eq. eqnblob)"},
        "swimmer_steps_per_s": swimmer_steps * args.steps / wall,
        "abc_accepts_per_s": n_acc * args.steps / wall,
        "abc_accepted": n_acc,
        "abc_tolerance": tol.item(),
        "runs_stopped": int(np.sum(st != 0)),
        "forward_call_ms": fwd_ms, "setup_ms": setup_ms,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_PEAK_TFLOPS, "traffic": TRAFFIC_BYTES,
                     "kernel": "k_forward<float,2,8> (persistent forward run, the default launch shape of 128-point FP32 systems)", "kernel_ms": kernel_ms,
                     "kernel_ms_source": "HIP events around the persistent launch (SWIM_OPT_TIME_KERNEL), "
                                         f"mean of {len(kus)} calls",
                     "fp32_flop_per_pair": FP32_FLOP_PER_PAIR, "pair_evals_per_launch": pairs,
                     "nonpacked_fp32_peak_tflops": NONPACKED_FP32_PEAK_TFLOPS,
                     "frac_of_nonpacked": tflops / NONPACKED_FP32_PEAK_TFLOPS,
                     "valu_ops_per_pair": VALU_OPS_PER_PAIR, "valu_issue_tops": issue,
                     "valu_issue_peak_tops": VALU_PEAK_TOPS, "valu_issue_frac": issue / VALU_PEAK_TOPS},
    }
    out["reading_blob"] = reading_blob_leg(ctx, stream, Ns, P, steps, dt, obs_every, fwd_ms)
    out["surrogate_mfma"] = mlp_leg(ctx, stream)
    out["fused_vs_per_sample"] = per_sample_leg(ctx, stream, P)
    if not args.no_dense:
        out["dense"] = dense_leg(ctx, stream, dt_div=args.dense_div)
    if not args.no_pmc:
        # a context of its own: the autotuner's launch shapes for this
        # workload stay out of the other legs
        pctx = swim.Context(0)
        out["pmc_uneven"] = pmc_leg(pctx, load_data())
        pctx.close()
    if not args.no_tmcmc:
        out["tmcmc"] = tmcmc_leg(ctx, load_data())
    if not args.no_sperm:
        out["sperm"] = sperm_leg(ctx, stream)
        if args.sperm_tmcmc:
            out["sperm_tmcmc"] = sperm_tmcmc_leg(ctx)
        out["flow_field"] = field_leg(ctx, stream)
    if not args.no_surrogate:
        out["surrogate_abc"] = surrogate_leg(ctx, load_data())
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
