"""The paper's experiments over the full sperm model on the GPU (Sec. 4):
observables (head-centre velocities, Sec. 4.1; tail and head distances of two
swimmers, Secs. 4.2-4.3), the two-level Gaussian likelihood (Sec. 4.3), and
TMCMC over the model (tmcmc_sperm_run) against the oracle's TMCMC driven by
the oracle's sperm model, stage by stage.

Both sides share only the seeded Philox streams.  In FP64 their
log-likelihoods agree to ~1e-13, so every tempering, resampling and
Metropolis decision coincides.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("reading_blob_module")]

torch = pytest.importorskip("torch")

from paper_1910_12007_amd import inputs, swim  # noqa: E402

EPS, HR = 0.045, 0.05


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = swim.Context(0)
    swim.swim_set_option(c, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_READING)
    yield c
    c.close()


def gpu_run(ctx, dtype, shape, rows, sw, steps, dt, oe):
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    n_sys = rows.shape[0]
    head = torch.empty((n_sys * shape.n_swim, steps // oe + 1, 2), dtype=td, device="cuda")
    tail = torch.empty_like(head)
    status = torch.empty(n_sys, dtype=torch.int32, device="cuda")
    swim.swim_sperm_forward(ctx, dtype, shape, torch.from_numpy(rows).cuda(), torch.from_numpy(sw).cuda(), steps, dt,
                            oe, head, tail, status)
    return head, tail, status


@pytest.mark.parametrize("dtype", [swim.SWIM_F64, swim.SWIM_F32])
def test_observables_match_oracle(ctx, oracle_core, dtype):
    """Both observables from the same GPU run (3 systems of two swimmers,
    one of them stopped by a bad row), GPU kernel against the oracle's
    definitions applied to the run's stored samples."""
    shape = swim.sperm_shape(n_swim=2)
    rows = inputs.sperm_rows(3, alpha=0.7)
    rows[1, 0] = -1.0
    sw = inputs.sperm_swimmers(3, 2, 0.5, phases=[0.0, 0.9])
    steps, dt, oe = 80, 1e-5, 20
    head, tail, status = gpu_run(ctx, dtype, shape, rows, sw, steps, dt, oe)
    n_obs = steps // oe
    for kind in (swim.SWIM_OBS_HEAD_VELOCITY, swim.SWIM_OBS_PAIR_DISTANCES):
        g = torch.empty((3, n_obs, 2), dtype=torch.float64, device="cuda")
        swim.swim_sperm_observables(ctx, dtype, kind, 2, oe * dt, head, tail, status, g)
        torch.cuda.synchronize()
        got = g.cpu().numpy()
        H = head.cpu().double().numpy().reshape(3, 2, n_obs + 1, 2)
        T = tail.cpu().double().numpy().reshape(3, 2, n_obs + 1, 2)
        assert np.all(np.isnan(got[1]))
        for s in (0, 2):
            ref = oracle_core.sperm_head_velocity(H[s], oe * dt) if kind == 0 else \
                oracle_core.sperm_pair_distances(H[s], T[s])
            np.testing.assert_allclose(got[s], ref, rtol=1e-13, atol=0)


def test_loglik2_matches_oracle(ctx):
    from oracle import tmcmc as otm
    rng = np.random.Generator(np.random.PCG64(41))
    n, n_obs = 500, 50
    data = rng.normal(size=(n_obs, 2))
    g = data[None] + rng.normal(scale=0.05, size=(n, n_obs, 2))
    s2 = rng.uniform(1e-3, 0.2, size=(n, 2))
    s2[7, 1] = 0.0
    g[11, 4, 0] = np.nan
    status = np.zeros(n, np.int32)
    status[::13] = 1
    logl = torch.empty(n, dtype=torch.float64, device="cuda")
    swim.tmcmc_loglik2(ctx, torch.from_numpy(g).cuda(), torch.from_numpy(data).cuda(), torch.from_numpy(s2).cuda(),
                       torch.from_numpy(status).cuda(), logl)
    torch.cuda.synchronize()
    got = logl.cpu().numpy()
    gg = g.reshape(n, -1).copy()
    gg[status != 0] = np.nan
    ref = otm.gauss_loglik2(gg, data.ravel(), s2[:, 0], s2[:, 1])
    assert np.array_equal(np.isneginf(got), np.isneginf(ref))
    ok = np.isfinite(ref)
    np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-12, atol=0)


def oracle_loglik_fn(core, otm, shape, sys_row, fields, n_sigma, kind, beta, sw, steps, dt, oe, data):
    idx = [inputs.SPERM_FIELDS.index(f) for f in fields]
    nf = len(fields)

    def fn(th):
        th = np.atleast_2d(th)
        out = np.empty(th.shape[0])
        for i, t in enumerate(th):
            row = np.array(sys_row, dtype=np.float64)
            row[idx] = t[:nf]
            r = core.sperm_forward(row, sw, shape.n_flag, shape.n_head, shape.eps, shape.head_radius,
                                   shape.neck_gap, steps, dt, oe)
            if r["status"] != 0:
                out[i] = -np.inf
                continue
            g = core.sperm_head_velocity(r["head"], oe * dt) if kind == 0 else \
                core.sperm_pair_distances(r["head"], r["tail"])
            ga, gb = t[nf], t[-1]
            out[i] = otm.gauss_loglik2(g.reshape(1, -1), data.ravel(), [ga * beta[0]], [gb * beta[1]])[0]
        return out
    return fn


CASES = {
    # Sec. 4.1: one swimmer, theta = (alpha, sigma/beta), head velocities
    "one_swimmer_alpha_sigma": dict(shape=dict(n_flag=50, n_head=24, n_swim=1), fields=("alpha",), n_sigma=1,
                                    kind=swim.SWIM_OBS_HEAD_VELOCITY, steps=60, oe=20,
                                    lo=[0.0, 0.01], hi=[2.0, 0.5], noise=0.05),
    # Sec. 4.3 (reduced swimmer): two swimmers, theta = (alpha, K_C,
    # sigma_t/beta_t, sigma_h/beta_h), tail and head distances
    "two_swimmers_two_sigma": dict(shape=dict(n_flag=20, n_head=8, n_swim=2), fields=("alpha", "KC"), n_sigma=2,
                                   kind=swim.SWIM_OBS_PAIR_DISTANCES, steps=60, oe=20,
                                   lo=[0.0, 0.0, 0.01, 0.01], hi=[2.0, 16.0, 0.5, 0.5], noise=0.02),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_tmcmc_sperm_run_matches_oracle(ctx, oracle_core, case):
    from oracle import tmcmc as otm
    cf = CASES[case]
    shp = cf["shape"]
    shape = swim.sperm_shape(shp["n_flag"], shp["n_head"], shp["n_swim"], EPS, HR, 1.0 / (shp["n_flag"] - 1))
    dt, steps, oe = 1e-5, cf["steps"], cf["oe"]
    sys_row = inputs.sperm_rows(1)[0]
    sw = inputs.sperm_swimmers(1, shp["n_swim"], 0.5)
    # synthetic data: the nominal model (alpha = 1, K_C = 8) plus relative noise
    r = oracle_core.sperm_forward(sys_row, sw, shape.n_flag, shape.n_head, EPS, HR, shape.neck_gap, steps, dt, oe)
    assert r["status"] == 0
    xi = oracle_core.sperm_head_velocity(r["head"], oe * dt) if cf["kind"] == 0 else \
        oracle_core.sperm_pair_distances(r["head"], r["tail"])
    if cf["n_sigma"] == 1:
        beta = [abs(xi.mean())] * 2
    else:
        beta = [abs(xi[:, 0].mean()), abs(xi[:, 1].mean())]
    rng = np.random.Generator(np.random.PCG64(5))
    data = xi + cf["noise"] * np.array(beta)[None, :] * rng.normal(size=xi.shape)
    n, seed = 16, 303
    fn = oracle_loglik_fn(oracle_core, otm, shape, sys_row, cf["fields"], cf["n_sigma"], cf["kind"], beta, sw,
                          steps, dt, oe, data)
    ref = otm.tmcmc(fn, cf["lo"], cf["hi"], n, seed, cv_target=1.0, b=0.2, max_stages=12)
    m = swim.sperm_model(shape, sys_row, cf["fields"], cf["n_sigma"], cf["kind"], beta, steps, oe, dt,
                         swim.SWIM_F64)
    got = swim.tmcmc_sperm_run(ctx, m, sw, cf["lo"], cf["hi"], data, n, seed, max_stages=12)
    print(case, {"stages": got["n_stages"], "q": got["q"], "accepted": got["accepted"], "runs": got["runs"],
                 "log_evidence": (got["log_evidence"], ref["log_evidence"]), "mean": got["theta"].mean(0)})
    assert got["n_stages"] == len(ref["q"]) - 1 >= 1
    np.testing.assert_allclose(got["q"], ref["q"], rtol=1e-9, atol=1e-15)
    assert np.array_equal(got["accepted"], ref["accepted"])
    assert got["runs"] == ref["evaluations"]
    span = np.max(np.array(cf["hi"]) - np.array(cf["lo"]))
    np.testing.assert_allclose(got["theta"], ref["theta"], rtol=1e-9, atol=1e-12 * span)
    np.testing.assert_allclose(got["logl"], ref["logl"], rtol=1e-9)
    assert abs(got["log_evidence"] - ref["log_evidence"]) <= 1e-9 * abs(ref["log_evidence"]) + 1e-9


def test_tmcmc_sperm_argument_errors(ctx):
    shape = swim.sperm_shape(20, 8, 2)
    row = inputs.sperm_rows(1)[0]
    sw = inputs.sperm_swimmers(1, 2, 0.5)
    data = np.zeros((3, 2))
    good = dict(fields=("alpha",), n_sigma=1, kind=swim.SWIM_OBS_PAIR_DISTANCES, beta=(1.0, 1.0))
    lo, hi = [0.0, 0.01], [2.0, 0.5]

    def call(shape=shape, fields=good["fields"], n_sigma=1, kind=good["kind"], beta=(1.0, 1.0), lo=lo, hi=hi,
             data=data, n=8, sw=sw):
        m = swim.sperm_model(shape, row, fields, n_sigma, kind, beta, 60, 20, 1e-5)
        return swim.tmcmc_sperm_run(ctx, m, sw, lo, hi, data, n, 1, max_stages=2)
    for kw in (dict(n_sigma=3), dict(fields=()), dict(fields=("alpha", "KC", "KT", "a")), dict(kind=7),
               dict(beta=(0.0, 1.0)), dict(lo=[0.0, -0.1]), dict(hi=[2.0, 0.005]), dict(data=np.zeros((2, 2))),
               dict(n=1), dict(shape=swim.sperm_shape(20, 8, 1), sw=sw[:1])):
        with pytest.raises(swim.SwimError):
            call(**kw)


def test_fp32_sperm_run_agrees_with_fp64_in_distribution(ctx, oracle_core):
    """FP32 forward runs change the likelihoods at the rounding level, so the
    chains take other decisions.  The FP32 run is compared in distribution:
    one swimmer, theta = (alpha, sigma/beta), 256 samples per stage.  Same
    number of stages within one, posterior means within one FP64 posterior
    standard deviation, evidence within 1 in log."""
    shape = swim.sperm_shape()
    dt, steps, oe = 1e-5, 60, 20
    sys_row = inputs.sperm_rows(1)[0]
    sw = inputs.sperm_swimmers(1)
    r = oracle_core.sperm_forward(sys_row, sw, shape.n_flag, shape.n_head, EPS, HR, shape.neck_gap, steps, dt, oe)
    xi = oracle_core.sperm_head_velocity(r["head"], oe * dt)
    beta = [abs(xi.mean())] * 2
    data = xi + 0.05 * beta[0] * np.random.Generator(np.random.PCG64(6)).normal(size=xi.shape)
    out = {}
    for dt_ in (swim.SWIM_F64, swim.SWIM_F32):
        m = swim.sperm_model(shape, sys_row, ("alpha",), 1, swim.SWIM_OBS_HEAD_VELOCITY, beta, steps, oe, dt, dt_)
        out[dt_] = swim.tmcmc_sperm_run(ctx, m, sw, [0.0, 0.01], [2.0, 0.5], data, 256, 41, max_stages=20)
    a, b = out[swim.SWIM_F64], out[swim.SWIM_F32]
    print({"stages": (a["n_stages"], b["n_stages"]), "mean64": a["theta"].mean(0), "mean32": b["theta"].mean(0),
           "std64": a["theta"].std(0), "logZ": (a["log_evidence"], b["log_evidence"])})
    assert a["q"][-1] == 1.0 and b["q"][-1] == 1.0
    assert abs(a["n_stages"] - b["n_stages"]) <= 1
    assert np.all(np.abs(a["theta"].mean(0) - b["theta"].mean(0)) <= a["theta"].std(0))
    assert abs(a["log_evidence"] - b["log_evidence"]) < 1.0
