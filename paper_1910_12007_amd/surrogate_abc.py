"""Surrogate-prescreened rejection ABC against plain batched ABC.

Every step runs in the library's kernels through its C ABI; this module
only sequences the calls, times them and summarizes the accepted sets.

The experiment:

1. plain batched ABC on the batched generation's draws (4096 prior draws,
   seed 1, N = 128, 10000 steps of dt = 2.5e-5): its 5th-percentile
   tolerance ``tol`` over the completed runs;
2. training set: ``n_train_runs`` prior draws (seed 4) run on the forward
   model; the first ``train_cap`` completed ones whose head stays within
   1.5 beat amplitudes of its start give (alpha,
   ln S_b, ln S_s, b, omega) -> 16 head displacements and the mean speed
   (about 8 % of the draws qualify, so 65536 training runs take about
   0.8M draws);
3. training: Adam (lr 1e-3, batch 1024, ``epochs`` epochs) on the GPU with
   the library's BF16 MFMA forward and backward kernels;
4. prescreen ``n_prop`` fresh prior draws at ``factor * tol`` with the
   surrogate, re-run the survivors on the plain forward model, accept
   d <= tol (a re-run stops once its running squared head deviation has
   passed the tolerance: its distance can only grow; the same pass without
   that stop is timed too, and gives the same accepted set);
5. plain batched ABC on the same ``n_prop`` proposals at the same ``tol``,
   for the accepted-samples rate and the reference posterior.

Accepted samples per second of each method = accepted / device time of the
work that produced them (the surrogate's one-off training-set and training
time are reported separately and folded into a second rate).
"""
import time

import numpy as np

from . import inputs, swim

# observation indices of the 16 summary times (every 3rd head sample, 3..48
# in 1-based sample numbers)
SUM_IDX = np.arange(2, 50, 3, dtype=np.int32)

# training-set bound on the head displacement at the summary times, in beat
# amplitudes b: within the observed quarter beat a stable swimmer's head
# moves about one amplitude, so a completed run beyond 1.5 b is an Euler
# instability below the blow-up bound.  Such a run is far outside any
# useful tolerance (one summary off by 0.05 already gives an RMS distance
# of about 0.009), and its erratic values would dominate the MSE.
MAX_DISP_PER_B = 1.5


def batch_model(steps=inputs.BATCH_STEPS, dt=inputs.BATCH_DT, obs_every=inputs.BATCH_OBS_EVERY,
                dtype=swim.SWIM_F32):
    m = swim.abc_model()
    for d in range(3):
        m.lo[d] = float(inputs.PRIOR_LO[d])
        m.hi[d] = float(inputs.PRIOR_HI[d])
    m.b, m.omega, m.k = 0.1, 2 * np.pi, 2 * np.pi
    m.steps, m.obs_every, m.dt, m.eps_over_ds = steps, obs_every, dt, 1.5
    m.dtype, m.use_graph = dtype, 1
    return m


def _sync():
    import torch
    torch.cuda.synchronize()


def train(ctx, model, N=128, n_train_runs=65536, seed=4, epochs=20, batch=1024, lr=1e-3, init_seed=0,
          cap=None, max_disp=None):
    """Generate the training set and train the surrogate; device tensors in
    the returned dict."""
    import torch
    cap = n_train_runs if cap is None else cap
    max_disp = MAX_DISP_PER_B * model.b if max_disp is None else max_disp
    dev = "cuda"
    X = torch.empty((cap, 5), dtype=torch.float32, device=dev)
    T = torch.empty((cap, 33), dtype=torch.float32, device=dev)
    st = {k: torch.empty(n, dtype=torch.float32, device=dev)
          for k, n in (("in_mu", 5), ("in_sd", 5), ("out_mu", 33), ("out_sd", 33))}
    _sync()
    t0 = time.perf_counter()
    n = swim.surrogate_dataset(ctx, model, N, n_train_runs, seed, SUM_IDX, max_disp, X, T, st["in_mu"], st["in_sd"],
                               st["out_mu"], st["out_sd"])
    _sync()
    t_data = time.perf_counter() - t0
    if n < batch:
        raise RuntimeError(f"only {n} completed training runs (batch {batch})")
    X, T = X[:n].contiguous(), T[:n].contiguous()
    _, flat = inputs.mlp_init(init_seed)
    params = torch.from_numpy(flat).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    perm = torch.from_numpy(inputs.epoch_permutations(n, epochs, seed)).to(dev)
    spe = n // batch
    loss = torch.empty(epochs * spe, dtype=torch.float32, device=dev)
    _sync()
    t0 = time.perf_counter()
    swim.surrogate_train(ctx, X, T, perm, epochs, batch, lr, params, m, v, loss)
    _sync()
    t_train = time.perf_counter() - t0
    lh = loss.cpu().numpy() / (33.0 * batch)
    return dict(params=params, X=X, T=T, n_rows=n, t_data=t_data, t_train=t_train, loss=lh, steps=epochs * spe,
                **st)


def plain_abc(ctx, model, data, N=128, n=4096, seeds=(1,), q=0.05, tol=None):
    """Plain batched ABC: one abc_step per seed (n prior draws each).  With
    tol given, acceptance is d <= tol on the returned distances; otherwise
    each batch's own percentile tolerance."""
    Nv = np.full(n, N, np.int32)
    thetas, dists, accs, secs, tols = [], [], [], [], []
    for s in seeds:
        t0 = time.perf_counter()
        r = swim.abc_step(ctx, model, data, Nv, s, 0, q)
        secs.append(time.perf_counter() - t0)
        acc = r["accept"] if tol is None else (np.isfinite(r["dist"]) & (r["dist"] <= tol))
        thetas.append(r["theta"])
        dists.append(r["dist"])
        accs.append(acc)
        tols.append(r["tol"])
    theta = np.concatenate(thetas)
    acc = np.concatenate(accs)
    return dict(theta=theta, dist=np.concatenate(dists), accept=acc, seconds=float(np.sum(secs)),
                tols=tols, n_accept=int(acc.sum()), n_completed=int(np.isfinite(np.concatenate(dists)).sum()))


def posterior_summary(theta):
    """Mean and the 5 % / 95 % quantiles (90 % interval) per parameter."""
    theta = np.asarray(theta)
    if theta.shape[0] == 0:
        nan = np.full(3, np.nan)
        return dict(mean=nan, lo=nan, hi=nan)
    return dict(mean=theta.mean(0), lo=np.quantile(theta, 0.05, axis=0), hi=np.quantile(theta, 0.95, axis=0))


def run(ctx, data, N=128, n_c1=4096, n_train_runs=1_000_000, train_cap=65536, epochs=20, n_prop=1 << 20,
        factor=2.0, prop_seed=5, model=None, keep_surrogate=False):
    """The whole comparison.  Plain ABC runs on the same n_prop proposals
    (same Philox seed) as the prescreen, so the surrogate's accepted set is
    a subset of the plain one and their difference is the surrogate's false
    negatives."""
    model = batch_model() if model is None else model
    # 1. tolerance: 5th percentile of the completed runs of the batched
    #    generation (n_c1 draws, seed 1)
    c1 = plain_abc(ctx, model, data, N, n_c1, seeds=(1,))
    tol = c1["tols"][0]
    # 2-3. surrogate
    S = train(ctx, model, N, n_train_runs, epochs=epochs, cap=train_cap)
    # 4. prescreened ABC
    t0 = time.perf_counter()
    P = swim.abc_prescreened(ctx, model, N, S["params"], S["in_mu"], S["in_sd"], S["out_mu"], S["out_sd"], SUM_IDX,
                             data, tol, factor, n_prop, prop_seed, n_prop)
    wall_s = time.perf_counter() - t0
    acc_s = int(P["accept"].sum())
    sec_s = (P["ms_prescreen"] + P["ms_rerun"]) * 1e-3
    # 4b. the same pass with every survivor run to the end (no early stop)
    swim.swim_set_option(ctx, swim.SWIM_OPT_EARLY_STOP, 0)
    try:
        Pf = swim.abc_prescreened(ctx, model, N, S["params"], S["in_mu"], S["in_sd"], S["out_mu"], S["out_sd"],
                                  SUM_IDX, data, tol, factor, n_prop, prop_seed, n_prop)
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_EARLY_STOP, 1)
    sec_f = (Pf["ms_prescreen"] + Pf["ms_rerun"]) * 1e-3
    # 5. plain ABC on the same proposals at the same tolerance
    R = plain_abc(ctx, model, data, N, n_prop, seeds=(prop_seed,), tol=tol)
    th_p = R["theta"][R["accept"]]
    th_s = P["theta"][P["accept"]]
    plain_set = {tuple(t) for t in th_p}
    surr_set = {tuple(t) for t in th_s}
    post_p = posterior_summary(th_p)
    post_s = posterior_summary(th_s)
    rate_p = R["n_accept"] / R["seconds"]
    rate_s = acc_s / sec_s
    rate_s_all = acc_s / (sec_s + S["t_data"] + S["t_train"])
    mean_err = np.abs(post_s["mean"] - post_p["mean"]) / np.abs(post_p["mean"])
    overlap = (post_s["lo"] <= post_p["hi"]) & (post_p["lo"] <= post_s["hi"])
    out = dict(
        tol=tol, factor=factor,
        plain=dict(proposals=n_prop, completed=R["n_completed"], accepted=R["n_accept"], seconds=R["seconds"],
                   accepts_per_s=rate_p, post=post_p),
        surrogate=dict(proposals=n_prop, survivors=P["n_surv"], accepted=acc_s,
                       completed=int(np.isfinite(P["dist"]).sum()), ms_prescreen=P["ms_prescreen"],
                       ms_rerun=P["ms_rerun"], wall_s=wall_s, accepts_per_s=rate_s,
                       stopped_early=int(np.sum(~np.isfinite(P["dist"]) & np.isfinite(Pf["dist"]))),
                       ms_rerun_without_early_stop=Pf["ms_rerun"],
                       accepts_per_s_without_early_stop=acc_s / sec_f,
                       same_accepted_without_early_stop=bool(np.array_equal(Pf["accept"], P["accept"])),
                       accepts_per_s_with_training=rate_s_all, post=post_s,
                       recall=len(surr_set & plain_set) / max(len(plain_set), 1),
                       not_in_plain=len(surr_set - plain_set)),
        training=dict(draws=n_train_runs, rows=S["n_rows"], steps=S["steps"], t_data=S["t_data"],
                      t_train=S["t_train"], loss_first=float(np.mean(S["loss"][:8])),
                      loss_last=float(np.mean(S["loss"][-8:]))),
        gain=rate_s / rate_p if rate_p > 0 else float("inf"),
        gain_without_early_stop=(acc_s / sec_f) / rate_p if rate_p > 0 else float("inf"),
        gain_with_training=rate_s_all / rate_p if rate_p > 0 else float("inf"),
        mean_rel_err=mean_err, intervals_overlap=overlap,
    )
    if keep_surrogate:
        out["S"] = S
        out["P"] = P
    return out
