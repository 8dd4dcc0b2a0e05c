"""The paper's blob (eq. eqnblob), the library's and the oracle's default
(SWIM_OPT_BLOB = SWIM_BLOB_PAPER), against the oracle with the same blob:
one velocity evaluation, forward runs of the filament and of the full sperm
model, and the flow and pressure field, in the Stokes limit (closed forms)
and for alpha > 0 (quadrature; FP32 from the tables built from it by the
node sweep).  Bars: FP64 1e-12 (per evaluation, norm-wise and point by
point, and on displacement series), FP32 1e-5 per evaluation and 1e-4 on
displacement series.  The oracle integrates every pair at alpha > 0 (~1 ms
each), so those cases are small systems over few steps; the batched
workload's size (N = 128, 1000 steps) checks FP32 against the library's
FP64 run of the same system, which the FP64 cases here pin to the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1910_12007_amd import inputs, swim  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = swim.Context(0)
    yield c
    c.close()


@pytest.fixture
def paper(ctx):
    """The context at its default blob (the paper's)."""
    assert swim.swim_get_option(ctx, swim.SWIM_OPT_BLOB) == swim.SWIM_BLOB_PAPER
    yield ctx
    assert swim.swim_get_option(ctx, swim.SWIM_OPT_BLOB) == swim.SWIM_BLOB_PAPER


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def rel_max(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: no single point hides in the norm."""
    return float(np.max(np.abs(np.ravel(a) - np.ravel(b))) / np.max(np.abs(np.ravel(b))))


@pytest.mark.parametrize("alpha,N", [(0.0, 100), (2.0, 24), (12.0, 24), (3.7, 128)])
@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-5)])
def test_pair_velocity(paper, oracle_core, dtype, tol, alpha, N):
    x, y = inputs.filament_geometry(N, 4, n_swim=2, spacing=0.3)
    fx, fy = [], []
    for m in range(2):
        f = oracle_core.forces(x[m * N:(m + 1) * N], y[m * N:(m + 1) * N], 0.1, 1e3,
                               oracle_core.kappa0(N, 0.1, 2 * np.pi, 2 * np.pi, 0.0, 0.02))
        fx.append(f[0])
        fy.append(f[1])
    fx, fy = np.concatenate(fx), np.concatenate(fy)
    eps = 1.5 / (N - 1)
    npd = np.float32 if dtype == swim.SWIM_F32 else np.float64
    arr = [np.asarray(a, npd) for a in (x, y, fx, fy)]
    dev = [torch.from_numpy(a).cuda() for a in arr]
    ux, uy = torch.empty_like(dev[0]), torch.empty_like(dev[0])
    swim.swim_pair_velocity(paper, np.array([0, 2 * N]), [alpha], [eps], *dev, ux, uy)
    torch.cuda.synchronize()
    ox, oy = oracle_core.velocity(*[a.astype(np.float64) for a in arr], alpha, eps)
    with oracle_core.paper_blob():
        rx, ry = oracle_core.velocity(*[a.astype(np.float64) for a in arr], alpha, eps)
    # the two blobs differ (the default is the paper's)
    with oracle_core.reading_blob():
        kx, ky = oracle_core.velocity(*[a.astype(np.float64) for a in arr], alpha, eps)
    assert rel(np.r_[kx, ky], np.r_[ox, oy]) > 1e-3
    got = np.r_[ux.cpu().double().numpy(), uy.cpu().double().numpy()]
    err, emax = rel(got, np.r_[ox, oy]), rel_max(got, np.r_[ox, oy])
    print({"dtype": dtype, "err": err, "max": emax})
    assert err <= tol and emax <= tol and np.array_equal(ox, rx)


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
def test_filament_forward_and_graph_key(ctx, oracle_core, dtype, tol):
    """A forward run with the other blob (twice: the second call captures a
    graph), then the same layout with the paper's blob: the captured graph
    of the first blob must not be replayed."""
    N, steps, dt, oe = 64, 200, 1e-4, 50
    P = inputs.param_rows(1, alpha=0.0)
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    obs = torch.empty((1, steps // oe, 2), dtype=td, device="cuda")
    speed = torch.empty(1, dtype=td, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    Pd = torch.from_numpy(P).cuda()
    outs = []
    try:
        for blob in (0, 0, 1):
            swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, blob)
            swim.swim_forward(ctx, [N], None, Pd, steps, dt, oe, 1.5, obs, speed, st)
            torch.cuda.synchronize()
            assert st.item() == 0
            outs.append(obs.cpu().double().numpy()[0].copy())
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_PAPER)
    x0 = np.array([1.0, 0.0])
    with oracle_core.reading_blob():
        ref0 = oracle_core.forward(P, N, steps, dt, oe)["obs"][0]
    ref1 = oracle_core.forward(P, N, steps, dt, oe)["obs"][0]
    floor = 4 * np.finfo(np.float32 if dtype == swim.SWIM_F32 else np.float64).eps * np.sqrt(steps) * 4
    for got, ref in ((outs[0], ref0), (outs[1], ref0), (outs[2], ref1)):
        err = np.linalg.norm(got - ref)
        allow = tol * np.linalg.norm(ref - x0) + floor
        print({"err": err, "allow": allow})
        assert err <= allow
    assert rel(ref1 - x0, ref0 - x0) > 1e-4


def test_sperm_forward(paper, oracle_core):
    rows = inputs.sperm_rows(1, alpha=0.0)
    sw = inputs.sperm_swimmers(1)
    shape = swim.sperm_shape()
    steps, dt, oe = 60, 1e-5, 20
    head = torch.empty((1, 4, 2), dtype=torch.float64, device="cuda")
    tail = torch.empty_like(head)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    swim.swim_sperm_forward(paper, swim.SWIM_F64, shape, torch.from_numpy(rows).cuda(), torch.from_numpy(sw).cuda(),
                            steps, dt, oe, head, tail, st)
    torch.cuda.synchronize()
    assert st.item() == 0
    with oracle_core.paper_blob():
        ref = oracle_core.sperm_forward(rows[0], sw, shape.n_flag, shape.n_head, shape.eps, shape.head_radius,
                                        shape.neck_gap, steps, dt, oe)
    for k, g in (("head", head), ("tail", tail)):
        got = g.cpu().numpy()[0]
        r = ref[k][0]
        err = rel(got - got[0], r - r[0])
        print(k, err)
        assert err <= 1e-11


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-5)])
def test_field(paper, oracle_core, dtype, tol):
    rng = np.random.Generator(np.random.PCG64(12))
    x, y = rng.uniform(0, 1, 80), rng.uniform(0, 0.3, 80)
    fx, fy = rng.normal(size=80), rng.normal(size=80)
    gx, gy = np.meshgrid(np.linspace(-0.2, 1.2, 30), np.linspace(-0.2, 0.5, 20))
    tx, ty = np.r_[gx.ravel(), x[:10]], np.r_[gy.ravel(), y[:10] + 0.003]
    npd = np.float32 if dtype == swim.SWIM_F32 else np.float64
    arr = [np.asarray(a, npd) for a in (x, y, fx, fy, tx, ty)]
    dev = [torch.from_numpy(a).cuda() for a in arr]
    u = torch.empty(tx.size, dtype=dev[0].dtype, device="cuda")
    v, p = torch.empty_like(u), torch.empty_like(u)
    swim.swim_flow_field(paper, *dev[:4], 0.0, 0.02, dev[4], dev[5], u, v, p)
    torch.cuda.synchronize()
    with oracle_core.paper_blob():
        ou, ov, op = oracle_core.field(*[a.astype(np.float64) for a in arr[:4]], 0.0, 0.02,
                                       arr[4].astype(np.float64), arr[5].astype(np.float64))
    e1 = rel(np.r_[u.cpu().double().numpy(), v.cpu().double().numpy()], np.r_[ou, ov])
    e2 = rel(p.cpu().double().numpy(), op)
    print({"velocity": e1, "pressure": e2})
    assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
def test_filament_forward_brinkman(paper, oracle_core, dtype, tol):
    """Two systems in one batch, alpha = 0 (closed forms) and alpha = 2
    (quadrature), each against the oracle's run with the paper's blob."""
    N, steps, dt, oe = 32, 20, 1e-4, 10
    P = inputs.param_rows(2, alpha=0.0)
    P[1, 0] = 2.0
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    obs = torch.empty((2, steps // oe, 2), dtype=td, device="cuda")
    speed = torch.empty(2, dtype=td, device="cuda")
    st = torch.empty(2, dtype=torch.int32, device="cuda")
    swim.swim_forward(paper, [N, N], None, torch.from_numpy(P).cuda(), steps, dt, oe, 1.5, obs, speed, st)
    torch.cuda.synchronize()
    assert list(st.cpu().numpy()) == [0, 0]
    got = obs.cpu().double().numpy()
    x0 = np.array([1.0, 0.0])
    floor = 4 * np.finfo(np.float32 if dtype == swim.SWIM_F32 else np.float64).eps * np.sqrt(steps) * 4
    with oracle_core.paper_blob():
        refs = [oracle_core.forward(P[i:i + 1], N, steps, dt, oe)["obs"][0] for i in range(2)]
    for i in range(2):
        err = np.linalg.norm(got[i] - refs[i])
        allow = tol * np.linalg.norm(refs[i] - x0) + floor
        print({"alpha": P[i, 0], "err": err, "allow": allow})
        assert err <= allow
    assert rel(refs[1] - x0, refs[0] - x0) > 1e-4


@pytest.mark.parametrize("dtype", [swim.SWIM_F64, swim.SWIM_F32])
def test_sperm_forward_brinkman(paper, oracle_core, dtype):
    """A small sperm model (12-point flagellum, 8-point head) at alpha = 0.9,
    with the bars of the default blob's sperm runs: FP64 within 4e-12 of the
    oracle's path length sum dt |u|, FP32 within 1e-4 of the displacement
    plus the FP32 spacing of the positions."""
    import test_gpu_sperm as tgs
    nf, nh, steps, dt, oe = 12, 8, 40, 1e-5, 10
    eps, hr, dn = 0.09, 0.05, 1.0 / 11
    shape = swim.sperm_shape(nf, nh, 1, eps, hr, dn)
    rows = inputs.sperm_rows(1, alpha=0.9, KC=5.0)
    sw = inputs.sperm_swimmers(1)
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    head = torch.empty((1, steps // oe + 1, 2), dtype=td, device="cuda")
    tail = torch.empty_like(head)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    swim.swim_sperm_forward(paper, dtype, shape, torch.from_numpy(rows).cuda(), torch.from_numpy(sw).cuda(), steps,
                            dt, oe, head, tail, st)
    torch.cuda.synchronize()
    assert st.item() == 0
    path = 0.0
    with oracle_core.paper_blob():
        ref = oracle_core.sperm_forward(rows[0], sw, nf, nh, eps, hr, dn, steps, dt, oe)
        x, y = oracle_core.sperm_initial(nf, nh, hr, dn, sw[0, 0], sw[0, 1])
        for k in range(steps):
            fx, fy = oracle_core.sperm_forces(nf, nh, hr, dn, rows[0], sw[0, 2], k * dt, x, y)
            ux, uy = oracle_core.velocity(x, y, fx, fy, rows[0][0], eps)
            path += dt * np.sqrt(np.sum(ux * ux + uy * uy))
            x, y = x + dt * ux, y + dt * uy
    assert ref["status"] == 0
    tgs.check(dtype, head.cpu().double().numpy(), ref["head"], path, steps, "head")
    tgs.check(dtype, tail.cpu().double().numpy(), ref["tail"], path, steps, "tail")


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-5)])
def test_field_brinkman(paper, oracle_core, dtype, tol):
    rng = np.random.Generator(np.random.PCG64(13))
    x, y = rng.uniform(0, 1, 40), rng.uniform(0, 0.3, 40)
    fx, fy = rng.normal(size=40), rng.normal(size=40)
    gx, gy = np.meshgrid(np.linspace(-0.2, 1.2, 15), np.linspace(-0.2, 0.5, 10))
    tx, ty = np.r_[gx.ravel(), x[:10]], np.r_[gy.ravel(), y[:10] + 0.003]
    npd = np.float32 if dtype == swim.SWIM_F32 else np.float64
    arr = [np.asarray(a, npd) for a in (x, y, fx, fy, tx, ty)]
    dev = [torch.from_numpy(a).cuda() for a in arr]
    u = torch.empty(tx.size, dtype=dev[0].dtype, device="cuda")
    v, p = torch.empty_like(u), torch.empty_like(u)
    swim.swim_flow_field(paper, *dev[:4], 2.0, 0.02, dev[4], dev[5], u, v, p)
    torch.cuda.synchronize()
    with oracle_core.paper_blob():
        ou, ov, op = oracle_core.field(*[a.astype(np.float64) for a in arr[:4]], 2.0, 0.02,
                                       arr[4].astype(np.float64), arr[5].astype(np.float64))
    e1 = rel(np.r_[u.cpu().double().numpy(), v.cpu().double().numpy()], np.r_[ou, ov])
    e2 = rel(p.cpu().double().numpy(), op)
    print({"velocity": e1, "pressure": e2})
    assert e1 <= tol and e2 <= tol


def test_graph_replay_rebuilds_quadrature_tables(paper, oracle_core):
    """FP32 runs with the paper's blob through a captured graph: the
    per-system constants (g(0) by quadrature) and the quadrature-built tables
    are set-up kernels inside the graph, so a replay with new alpha values in
    the same parameter buffer must equal the eager run at those values, bit
    for bit, and the oracle within the FP32 bar."""
    N, steps, dt, oe = 32, 20, 1e-4, 10
    P = inputs.param_rows(2, alpha=2.0)
    P[1, 0] = 5.0
    P2 = P.copy()
    P2[:, 0] = [0.7, 9.0]
    Pd = torch.from_numpy(P).cuda()
    obs = torch.empty((2, steps // oe, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(2, dtype=torch.float32, device="cuda")
    st = torch.empty(2, dtype=torch.int32, device="cuda")

    def run():
        swim.swim_forward(paper, [N, N], None, Pd, steps, dt, oe, 1.5, obs, speed, st)
        torch.cuda.synchronize()
        assert list(st.cpu().numpy()) == [0, 0]
        return obs.cpu().numpy().copy()

    try:
        swim.swim_set_option(paper, swim.SWIM_OPT_GRAPH, 0)
        ref = run()
        Pd.copy_(torch.from_numpy(P2))
        torch.cuda.synchronize()
        ref2 = run()
        Pd.copy_(torch.from_numpy(P))
        torch.cuda.synchronize()
        swim.swim_set_option(paper, swim.SWIM_OPT_GRAPH, 1)
        captures0 = swim.swim_get_option(paper, swim.SWIM_OPT_GRAPH_CAPTURES)
        launches0 = swim.swim_get_option(paper, swim.SWIM_OPT_GRAPH_LAUNCHES)
        for _ in range(3):
            assert np.array_equal(run(), ref)
        Pd.copy_(torch.from_numpy(P2))
        torch.cuda.synchronize()
        for _ in range(2):
            assert np.array_equal(run(), ref2)
        assert swim.swim_get_option(paper, swim.SWIM_OPT_GRAPH_CAPTURES) - captures0 == 1
        assert swim.swim_get_option(paper, swim.SWIM_OPT_GRAPH_LAUNCHES) - launches0 == 4
    finally:
        swim.swim_set_option(paper, swim.SWIM_OPT_GRAPH, 1)
    x0 = np.array([1.0, 0.0])
    floor = 4 * np.finfo(np.float32).eps * np.sqrt(steps) * 4
    with oracle_core.paper_blob():
        for i in range(2):
            r = oracle_core.forward(P2[i:i + 1], N, steps, dt, oe)["obs"][0]
            err = np.linalg.norm(ref2[i] - r)
            allow = 1e-4 * np.linalg.norm(r - x0) + floor
            print({"alpha": P2[i, 0], "err": err, "allow": allow})
            assert err <= allow


@pytest.mark.parametrize("dtype", [swim.SWIM_F64, swim.SWIM_F32])
def test_edge_cases(paper, oracle_core, dtype):
    """The paper's blob at alpha > 0: a field of no sources is zero, a field
    of no targets is a no-op, and at the domain's edge alpha * eps = 1 the
    velocity still meets its bar."""
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    none = torch.empty(0, dtype=td, device="cuda")
    tx = torch.linspace(0, 1, 5, dtype=td, device="cuda")
    u = torch.full((5,), 7.0, dtype=td, device="cuda")
    v, p = u.clone(), u.clone()
    swim.swim_flow_field(paper, none, none, none, none, 2.0, 0.05, tx, tx, u, v, p)
    torch.cuda.synchronize()
    assert torch.all(u == 0) and torch.all(v == 0) and torch.all(p == 0)
    swim.swim_flow_field(paper, tx, tx, tx, tx, 2.0, 0.05, none, none, none, none, none)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(21))
    pts = [rng.uniform(0, 1, 24), rng.uniform(0, 0.3, 24), rng.normal(size=24), rng.normal(size=24)]
    npd = np.float32 if dtype == swim.SWIM_F32 else np.float64
    arr = [a.astype(npd) for a in pts]
    dev = [torch.from_numpy(a).cuda() for a in arr]
    ux, uy = torch.empty_like(dev[0]), torch.empty_like(dev[0])
    swim.swim_pair_velocity(paper, np.array([0, 24]), [20.0], [0.05], *dev, ux, uy)
    torch.cuda.synchronize()
    with oracle_core.paper_blob():
        ox, oy = oracle_core.velocity(*[a.astype(np.float64) for a in arr], 20.0, 0.05)
    got = np.r_[ux.cpu().double().numpy(), uy.cpu().double().numpy()]
    err, emax = rel(got, np.r_[ox, oy]), rel_max(got, np.r_[ox, oy])
    print({"dtype": dtype, "err": err, "max": emax})
    bar = 1e-12 if dtype == swim.SWIM_F64 else 1e-5
    assert err <= bar and emax <= bar


def test_tmcmc_sperm_run_fp32(paper):
    """TMCMC over a small sperm model with the paper's blob at alpha > 0,
    FP32: every chain step relaunches the forward runs, whose set-up (g(0)
    and the quadrature-built tables) follows each sample's alpha.  The data
    come from an FP64 run at alpha = 1 plus 2 % noise.  The run completes
    with samples inside the prior box, finite likelihoods and evidence, and
    a posterior on alpha that covers the truth.  (The oracle, integrating
    every pair, is too slow for the hundreds of runs a TMCMC run takes.)"""
    nf, nh, steps, dt, oe = 12, 8, 60, 1e-5, 20
    shape = swim.sperm_shape(nf, nh, 1, 0.09, 0.05, 1.0 / 11)
    row = inputs.sperm_rows(1, alpha=1.0, KC=5.0)
    sw = inputs.sperm_swimmers(1)
    head = torch.empty((1, steps // oe + 1, 2), dtype=torch.float64, device="cuda")
    tail = torch.empty_like(head)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    swim.swim_sperm_forward(paper, swim.SWIM_F64, shape, torch.from_numpy(row).cuda(), torch.from_numpy(sw).cuda(),
                            steps, dt, oe, head, tail, st)
    g = torch.empty((1, steps // oe, 2), dtype=torch.float64, device="cuda")
    swim.swim_sperm_observables(paper, swim.SWIM_F64, swim.SWIM_OBS_HEAD_VELOCITY, 1, oe * dt, head, tail, st, g)
    torch.cuda.synchronize()
    assert st.item() == 0
    xi = g.cpu().numpy()[0]
    beta = [abs(xi.mean())] * 2
    rng = np.random.Generator(np.random.PCG64(9))
    data = xi + 0.02 * beta[0] * rng.normal(size=xi.shape)
    m = swim.sperm_model(shape, row[0], ("alpha",), 1, swim.SWIM_OBS_HEAD_VELOCITY, beta, steps, oe, dt,
                         swim.SWIM_F32)
    lo, hi = [0.0, 0.001], [2.0, 0.2]
    got = swim.tmcmc_sperm_run(paper, m, sw, lo, hi, data, 128, 77, max_stages=12)
    th = got["theta"]
    print({"stages": got["n_stages"], "runs": got["runs"], "log_evidence": got["log_evidence"],
           "mean": th.mean(0), "std": th.std(0)})
    assert got["n_stages"] >= 1 and np.isfinite(got["log_evidence"])
    assert np.all(np.isfinite(got["logl"]))
    assert np.all(th >= np.array(lo)) and np.all(th <= np.array(hi))
    a = th[:, 0]
    assert a.min() <= 1.0 <= a.max()
    assert abs(a.mean() - 1.0) <= 4 * a.std() + 0.05


def test_batched_size_fp32_against_fp64(paper):
    """The batched workload's filament (N = 128, dt = 5e-5) with the paper's
    blob at alpha > 0, 1000 steps: the FP32 run (tables from the node sweep)
    against the library's FP64 run of the same system (quadrature per pair;
    the FP64 cases above pin it to the oracle), at 1e-4 on the displacement
    series and the mean speed.  The draws are picked on the FP64 runs of the
    batch's first 256 prior draws alone: of those that complete and swim at
    a physical speed (mean head speed below one body length per unit time;
    the gait drives about 0.4), the two with the softest stretching springs.
    A completed run is not necessarily a stable one: with the paper's
    stiffer near field, some draws settle into a bounded oscillation of
    forward Euler (e.g. (7.92, 0.54, 179): mean speed 25, and whether it
    leaves the position bound within 1000 steps depends on rounding), in
    which the two precisions drift apart by a few percent and which carries
    no parity information.  Picking on FP32 completion let the FP32 sum
    order decide which draws the test compares."""
    N, steps, dt, oe = 128, 1000, 5e-5, 100
    theta = swim.abc_prior_draw(1, 256, inputs.PRIOR_LO, inputs.PRIOR_HI)
    Pa = torch.from_numpy(inputs.theta_rows(theta)).cuda()
    ob = torch.empty((256, steps // oe, 2), dtype=torch.float64, device="cuda")
    sp = torch.empty(256, dtype=torch.float64, device="cuda")
    st = torch.empty(256, dtype=torch.int32, device="cuda")
    swim.swim_forward(paper, np.full(256, N, np.int32), None, Pa, steps, dt, oe, 1.5, ob, sp, st)
    torch.cuda.synchronize()
    ok = np.flatnonzero((st.cpu().numpy() == 0) & (sp.cpu().numpy() < 1.0))
    assert ok.size >= 2
    pick = list(ok[np.argsort(theta[ok, 2], kind="stable")[:2]])
    P = inputs.theta_rows(theta[pick])
    Pd = torch.from_numpy(P).cuda()
    out = {}
    for dtype, td in ((swim.SWIM_F32, torch.float32), (swim.SWIM_F64, torch.float64)):
        obs = torch.empty((2, steps // oe, 2), dtype=td, device="cuda")
        speed = torch.empty(2, dtype=td, device="cuda")
        st = torch.empty(2, dtype=torch.int32, device="cuda")
        swim.swim_forward(paper, [N, N], None, Pd, steps, dt, oe, 1.5, obs, speed, st)
        torch.cuda.synchronize()
        assert list(st.cpu().numpy()) == [0, 0], dtype
        out[dtype] = (obs.cpu().double().numpy(), speed.cpu().double().numpy())
    x0 = np.array([1.0, 0.0])
    for i, bar in ((0, 1e-4), (1, 1e-4)):
        o32, s32 = out[swim.SWIM_F32][0][i], out[swim.SWIM_F32][1][i]
        o64, s64 = out[swim.SWIM_F64][0][i], out[swim.SWIM_F64][1][i]
        floor = np.linalg.norm(np.spacing(np.abs(o64).astype(np.float32)))
        err = np.linalg.norm(o32 - o64)
        print({"draw": pick[i], "theta": theta[pick[i]], "series": err / np.linalg.norm(o64 - x0),
               "speed": abs(s32 / s64 - 1)})
        assert err <= bar * np.linalg.norm(o64 - x0) + floor
        assert abs(s32 / s64 - 1) <= bar


def test_dense_sample_as_benchmarked(paper, oracle_core):
    """The dense workload's sample 0 (8 swimmers x 512 points on the 2 x 4
    grid, its alpha) with the paper's blob, as the benchmark runs it.  One
    velocity evaluation at the initial configuration, all 4096 sources, on
    16 sampled targets (both ends of every swimmer) against the oracle's
    quadrature, which takes ~0.5 s per target: FP32 within 1e-5 and FP64
    within 1e-12 of the largest sampled velocity.  Then the run at the
    benchmark's dt = 2e-5/64: FP32 against the FP64 run over 100 steps,
    head of every swimmer every 10, at 1e-4 of the displacement (plus one
    FP32 spacing of the stored positions), both runs completing."""
    lay = inputs.dense_layout(n_samples=1, seed=3)[0]
    s = np.arange(512) / 511.0
    X = np.concatenate([lay[m, 7] + s for m in range(8)])
    Y = np.concatenate([np.full(512, lay[m, 8]) for m in range(8)])
    F = [oracle_core.forces(X[512 * m:512 * (m + 1)], Y[512 * m:512 * (m + 1)], lay[m, 1], lay[m, 2],
                            oracle_core.kappa0(512, lay[m, 3], lay[m, 5], lay[m, 4], lay[m, 6], 0.0))
         for m in range(8)]
    FX = np.concatenate([f[0] for f in F])
    FY = np.concatenate([f[1] for f in F])
    eps = 1.5 / 511
    idx = np.concatenate([[512 * m, 512 * m + 511] for m in range(8)])
    for dtype, tol, npd, td in ((swim.SWIM_F32, 1e-5, np.float32, torch.float32),
                                (swim.SWIM_F64, 1e-12, np.float64, torch.float64)):
        # both sides take the same (rounded) positions and forces
        arr = [a.astype(npd) for a in (X, Y, FX, FY)]
        ux = torch.empty(4096, dtype=td, device="cuda")
        uy = torch.empty_like(ux)
        swim.swim_pair_velocity(paper, np.array([0, 4096]), [lay[0, 0]], [eps],
                                *[torch.from_numpy(a).cuda() for a in arr], ux, uy)
        torch.cuda.synchronize()
        ox, oy = oracle_core.velocity_at(*[a.astype(np.float64) for a in arr], lay[0, 0], eps, idx)
        got = np.r_[ux.cpu().double().numpy()[idx], uy.cpu().double().numpy()[idx]]
        ref = np.r_[ox, oy]
        print({"dtype": dtype, "max": rel_max(got, ref)})
        assert rel_max(got, ref) <= tol, (dtype, rel_max(got, ref))
    P = torch.from_numpy(lay).cuda()
    dt = 2e-5 / 64
    out = {}
    for dtype, td in ((swim.SWIM_F64, torch.float64), (swim.SWIM_F32, torch.float32)):
        P_t = P.to(torch.float64)
        obs = torch.empty((8, 10, 2), dtype=td, device="cuda")
        speed = torch.empty(8, dtype=td, device="cuda")
        st = torch.empty(1, dtype=torch.int32, device="cuda")
        swim.swim_forward(paper, [512], [8], P_t, 100, dt, 10, 1.5, obs, speed, st)
        torch.cuda.synchronize()
        assert st.item() == swim.SWIM_ST_OK, dtype
        out[dtype] = obs.cpu().double().numpy()
    o64, o32 = out[swim.SWIM_F64], out[swim.SWIM_F32]
    x0 = lay[:, 7:9] + np.array([1.0, 0.0])
    disp = np.linalg.norm(o64 - x0[:, None, :])
    floor = np.linalg.norm(np.spacing(np.abs(o64).astype(np.float32)))
    err = np.linalg.norm(o32 - o64)
    print({"fp32_vs_fp64": err / disp})
    assert err <= 1e-4 * disp + floor


def test_batched_workload_as_benchmarked(paper):
    """The batched workload in the launch configuration the benchmark times:
    4096 prior draws (Philox seed 1), N = 128, the paper's blob, 10000 steps
    of dt = 2.5e-5, head every 200 steps, FP32, default launch shapes, one
    swim_forward call; then the ABC distance, tolerance and accept mask.
    The tolerance and mask follow the oracle's definitions applied to the
    GPU distances.  The oracle integrates every pair of the paper's blob
    (~10 s per step of this system on one core), so the sampled runs, the
    first completed run in draw order and the one closest to the data, are
    held against the library's FP64 run of the same system over all 10000
    steps (the FP64 path is pinned to the oracle above), at 1e-4 on the mean
    speed, the ABC distance and the displacement series; the two earliest
    blow-ups blow up in FP64 too."""
    import os
    from oracle import abc
    n, N = 4096, 128
    steps, dt, oe = inputs.BATCH_STEPS, inputs.BATCH_DT, inputs.BATCH_OBS_EVERY
    n_obs = steps // oe
    theta = swim.abc_prior_draw(1, n, inputs.PRIOR_LO, inputs.PRIOR_HI)
    P = inputs.theta_rows(theta)
    obs = torch.empty((n, n_obs, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    swim.swim_forward(paper, np.full(n, N, np.int32), None, torch.from_numpy(P).cuda(), steps, dt, oe, 1.5, obs,
                      speed, status, done)
    data = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "abc_data_batch.txt"))[:n_obs, :2]
    dist = torch.empty(n, dtype=torch.float64, device="cuda")
    tol = torch.empty(1, dtype=torch.float64, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")
    swim.abc_distance(paper, obs, torch.from_numpy(data).cuda(), status, dist)
    swim.abc_select(paper, dist, 0.05, tol, acc)
    torch.cuda.synchronize()
    st, d, sd = status.cpu().numpy(), dist.cpu().numpy(), done.cpu().numpy()
    assert tol.item() == abc.tolerance(d, 0.05)
    assert np.array_equal(acc.cpu().numpy().astype(bool), abc.accept(d, tol.item()))
    ok, bad = np.flatnonzero(st == 0), np.flatnonzero(st != 0)
    assert 100 < ok.size < n
    samples = [ok[0], ok[np.argmin(d[ok])]]
    P2 = torch.from_numpy(P[samples]).cuda()
    o64 = torch.empty((2, n_obs, 2), dtype=torch.float64, device="cuda")
    s64 = torch.empty(2, dtype=torch.float64, device="cuda")
    t64 = torch.empty(2, dtype=torch.int32, device="cuda")
    swim.swim_forward(paper, [N, N], None, P2, steps, dt, oe, 1.5, o64, s64, t64)
    torch.cuda.synchronize()
    assert list(t64.cpu().numpy()) == [0, 0]
    o32 = obs.cpu().double().numpy()
    x0 = np.array([1.0, 0.0])
    for k, i in enumerate(samples):
        r, rs = o64[k].cpu().numpy(), s64[k].item()
        dr = abc.distance(r[None], data)[0]
        floor = np.linalg.norm(np.spacing(np.abs(r).astype(np.float32)))
        err = np.linalg.norm(o32[i] - r)
        print({"draw": int(i), "theta": theta[i], "series": err / np.linalg.norm(r - x0),
               "speed": abs(speed[i].item() / rs - 1), "dist": abs(d[i] / dr - 1)})
        assert abs(speed[i].item() / rs - 1) <= 1e-4
        assert abs(d[i] / dr - 1) <= 1e-4
        assert err <= 1e-4 * np.linalg.norm(r - x0) + floor
    # the two earliest blow-ups blow up in FP64 too
    early = bad[np.argsort(sd[bad], kind="stable")[:2]]
    k = int(sd[early].max()) + 50
    Pb = torch.from_numpy(P[early]).cuda()
    ob = torch.empty((2, 1, 2), dtype=torch.float64, device="cuda")
    sb = torch.empty(2, dtype=torch.float64, device="cuda")
    tb = torch.empty(2, dtype=torch.int32, device="cuda")
    swim.swim_forward(paper, [N, N], None, Pb, k, dt, k, 1.5, ob, sb, tb)
    torch.cuda.synchronize()
    assert np.all(tb.cpu().numpy() != 0), (theta[early], sd[early])
