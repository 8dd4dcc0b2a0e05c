"""GPU parity of libswim against the FP64 oracle (run on an MI355X).

Tolerances (norm-wise relative, over the whole vector of one evaluation):
  velocity sum, FP64 build  1e-12;  FP32 build 1e-5
  head-displacement series of a forward run, FP64 1e-12;  FP32 1e-4, plus
  the rounding floor of the state (eps |X| sqrt(steps)) and, for FP32, one
  ulp of each stored head position (see check_traj)
  elastic forces from FP32 positions: 1e-4 (the strain l/ds - 1 of a spring
  is a difference of O(1) numbers; at strains ~1e-3 a few ulp of l become
  ~1e-4 of the tension), FP64 1e-11.
Inputs are rounded to the kernel's precision first and the oracle gets the
same rounded values.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("reading_blob_module")]

torch = pytest.importorskip("torch")

from paper_1910_12007_amd import inputs, swim  # noqa: E402

DT = {swim.SWIM_F32: torch.float32, swim.SWIM_F64: torch.float64}
NP = {swim.SWIM_F32: np.float32, swim.SWIM_F64: np.float64}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = swim.Context(0)
    swim.swim_set_option(c, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_READING)
    yield c
    c.close()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def rel_max(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: point by point, so that a few wrong
    points (near contact, a block's tail) cannot hide in a norm."""
    return float(np.max(np.abs(np.ravel(a) - np.ravel(b))) / np.max(np.abs(np.ravel(b))))


def _systems():
    """(N, n_swim, alpha) of one multi-system call: ragged sizes across the
    256-point tiles, several swimmers in one fluid, Stokes to alpha = 10."""
    return [(64, 1, 1.0), (128, 1, 0.0), (300, 1, 2.0), (96, 3, 1e-3), (200, 2, 10.0), (520, 1, 5.0)]


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-5)])
def test_pair_velocity_matches_oracle(ctx, oracle_core, dtype, tol):
    xs, ys, fxs, fys, off, alphas, epss = [], [], [], [], [0], [], []
    for k, (N, nsw, a) in enumerate(_systems()):
        x, y = inputs.filament_geometry(N, seed=10 + k, n_swim=nsw)
        fx, fy = inputs.force_pattern(N, seed=20 + k, n_swim=nsw)
        xs.append(x); ys.append(y); fxs.append(fx); fys.append(fy)
        off.append(off[-1] + N * nsw)
        alphas.append(a)
        epss.append(1.5 / (N - 1))
    X, Y, FX, FY = (np.concatenate(v).astype(NP[dtype]) for v in (xs, ys, fxs, fys))
    td = DT[dtype]
    ux = torch.empty(len(X), dtype=td, device="cuda")
    uy = torch.empty_like(ux)
    swim.swim_pair_velocity(ctx, np.array(off), alphas, epss, dev(X, td), dev(Y, td), dev(FX, td), dev(FY, td), ux, uy)
    torch.cuda.synchronize()
    gx, gy = ux.cpu().double().numpy(), uy.cpu().double().numpy()
    for s in range(len(alphas)):
        sl = slice(off[s], off[s + 1])
        ox, oy = oracle_core.velocity(X[sl], Y[sl], FX[sl], FY[sl], alphas[s], epss[s])
        g, r = np.concatenate([gx[sl], gy[sl]]), np.concatenate([ox, oy])
        e, em = rel(g, r), rel_max(g, r)
        assert e < tol and em < tol, (s, _systems()[s], e, em)


@pytest.mark.parametrize("alpha", [0.0, 0.7])
def test_pair_velocity_far_pairs(ctx, oracle_core, alpha):
    """FP32 pairs beyond the kernel table (r^2/eps^2 >= 2^24, here two
    filaments about 60 body lengths apart at eps = 1.5/127) take the direct
    evaluation; near pairs in the same system still use the table."""
    N = 128
    x1, y1 = inputs.filament_geometry(N, seed=41, n_swim=1)
    x2, y2 = inputs.filament_geometry(N, seed=42, n_swim=1)
    X = np.concatenate([x1, x2 + 60.0]).astype(np.float32)
    Y = np.concatenate([y1, y2 + 5.0]).astype(np.float32)
    fx1, fy1 = inputs.force_pattern(N, seed=43, n_swim=1)
    fx2, fy2 = inputs.force_pattern(N, seed=44, n_swim=1)
    # a net force on each filament makes the far pairs' share of the
    # velocity large (a dropped or wrong far term fails the tolerance)
    FX = np.concatenate([fx1 + 2.0, fx2 - 3.0]).astype(np.float32)
    FY = np.concatenate([fy1 - 1.0, fy2 + 4.0]).astype(np.float32)
    eps = 1.5 / (N - 1)
    assert ((60.0 - 1.0) / eps) ** 2 > 2.0 ** 24
    ux = torch.empty(2 * N, dtype=torch.float32, device="cuda")
    uy = torch.empty_like(ux)
    swim.swim_pair_velocity(ctx, np.array([0, 2 * N]), [alpha], [eps], dev(X, torch.float32), dev(Y, torch.float32),
                            dev(FX, torch.float32), dev(FY, torch.float32), ux, uy)
    torch.cuda.synchronize()
    ox, oy = oracle_core.velocity(X, Y, FX, FY, alpha, eps)
    g = np.concatenate([ux.cpu().double().numpy(), uy.cpu().double().numpy()])
    assert rel(g, np.concatenate([ox, oy])) < 1e-5 and rel_max(g, np.concatenate([ox, oy])) < 1e-5


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-11), (swim.SWIM_F32, 1e-4)])
def test_elastic_forces_match_oracle(ctx, oracle_core, dtype, tol):
    Ns = [5, 64, 127, 300]
    rows, xs, ys = [], [], []
    for k, N in enumerate(Ns):
        x, y = inputs.filament_geometry(N, seed=30 + k)
        xs.append(x); ys.append(y)
        rows.append(inputs.param_rows(1, Sb=0.1 * (k + 1), Ss=300.0 * (k + 1), phase=0.3 * k)[0])
    P = np.array(rows)
    X, Y = (np.concatenate(v).astype(NP[dtype]) for v in (xs, ys))
    td = DT[dtype]
    fx = torch.empty(len(X), dtype=td, device="cuda")
    fy = torch.empty_like(fx)
    t = 0.0123
    swim.swim_elastic_forces(ctx, Ns, P, t, dev(X, td), dev(Y, td), fx, fy)
    torch.cuda.synchronize()
    gx, gy = fx.cpu().double().numpy(), fy.cpu().double().numpy()
    o = 0
    for k, N in enumerate(Ns):
        sl = slice(o, o + N)
        k0 = oracle_core.kappa0(N, P[k, 3], P[k, 5], P[k, 4], P[k, 6], t)
        ox, oy = oracle_core.forces(X[sl], Y[sl], P[k, 1], P[k, 2], k0)
        assert rel(np.concatenate([gx[sl], gy[sl]]), np.concatenate([ox, oy])) < tol, (N,)
        o += N


def run_forward(ctx, dtype, N, n_swim, P, steps, dt, obs_every):
    td = DT[dtype]
    N = np.atleast_1d(np.asarray(N, np.int32))
    nfil = P.shape[0]
    n_obs = steps // obs_every
    obs = torch.full((nfil, n_obs, 2), float("nan"), dtype=td, device="cuda")
    speed = torch.empty(nfil, dtype=td, device="cuda")
    status = torch.empty(len(N), dtype=torch.int32, device="cuda")
    swim.swim_forward(ctx, N, n_swim, dev(P, torch.float64), steps, dt, obs_every, 1.5, obs, speed, status)
    torch.cuda.synchronize()
    return obs.cpu().double().numpy(), speed.cpu().double().numpy(), status.cpu().numpy()


def disp_err(obs, ref, x0):
    """relative error of the head-displacement series (positions minus the
    initial head position)."""
    return rel(obs - x0, ref - x0)


def check_traj(obs, ref, x0, tol, dtype, steps, xmax):
    """|obs - ref| <= tol |ref - x0| + floor.  The floor is the rounding of the
    state itself: positions of size xmax updated `steps` times carry
    ~eps xmax sqrt(steps) of rounding whatever the arithmetic (it matters only
    for runs whose displacement is tiny), and FP32 outputs add one ulp of
    every stored position."""
    err = np.linalg.norm(np.ravel(obs - ref))
    eps = np.finfo(np.float32 if dtype == swim.SWIM_F32 else np.float64).eps
    allow = tol * np.linalg.norm(np.ravel(ref - x0)) + 4 * eps * xmax * np.sqrt(steps) * np.sqrt(ref.size)
    if dtype == swim.SWIM_F32:
        allow += np.linalg.norm(np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64))
    assert err <= allow, (err, allow, disp_err(obs, ref, x0))


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
@pytest.mark.parametrize("alpha", [1.0, 0.0])
def test_single_swimmer_run_matches_oracle(ctx, oracle_core, dtype, tol, alpha):
    """N = 64, 2000 steps of dt = 1e-4, S_b = 0.1, S_s = 1e3, b = 0.1, k = omega = 2 pi."""
    P = inputs.param_rows(1, alpha=alpha)
    obs, speed, st = run_forward(ctx, dtype, [64], None, P, 2000, 1e-4, 100)
    ref = oracle_core.forward(P, 64, 2000, 1e-4, 100)
    assert st[0] == 0 and ref["status"] == 0
    check_traj(obs[0], ref["obs"][0], np.array([1.0, 0.0]), tol, dtype, 2000, 1.0)
    assert abs(speed[0] / ref["speed"][0] - 1) < tol


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
def test_uneven_batch_matches_oracle(ctx, oracle_core, dtype, tol):
    """Systems of 64 to 512 points (every persistent-kernel bucket), 60 steps,
    with 1, 2 and 4 wavefronts per system (one wave only for the systems of
    up to 256 points: larger ones need at least two, and asking for one is
    an error).  The heads start at the origin (x0 = -1): the run is short
    enough for the head to move ~1e-5, which FP32 outputs resolve only near
    zero."""
    Ns = [64, 96, 160, 200, 256, 320, 448, 512, 128, 64]
    rng = np.random.Generator(np.random.PCG64(41))
    P = inputs.param_rows(len(Ns), Sb=0.01, Ss=100.0, x0=-1.0)
    P[:, 0] = rng.uniform(0, 10, len(Ns))
    P[1, 0] = 0.0
    steps, dt = 60, 2e-6
    refs = [oracle_core.forward(P[i:i + 1], N, steps, dt, 20) for i, N in enumerate(Ns)]
    try:
        for wps in (1, 2, 4):
            swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, wps)
            sel = [i for i, N in enumerate(Ns) if wps > 1 or N <= 256]
            Ns_w = [Ns[i] for i in sel]
            obs, speed, st = run_forward(ctx, dtype, Ns_w, None, P[sel], steps, dt, 20)
            for k, i in enumerate(sel):
                assert st[k] == 0 and refs[i]["status"] == 0
                check_traj(obs[k], refs[i]["obs"][0], np.array([0.0, 0.0]), tol, dtype, steps, 1.0)
            again = run_forward(ctx, dtype, Ns_w, None, P[sel], steps, dt, 20)
            assert np.array_equal(again[0], obs), "runs are not bit-reproducible"
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, 0)


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
def test_multi_swimmer_systems_match_oracle(ctx, oracle_core, dtype, tol):
    """Interacting swimmers: a 3 x 64 system (persistent kernel) and an
    8 x 80 system (per-step kernel with targets split over workgroups), on a
    grid centred at the origin, 100 steps of dt = 5e-5."""
    lay = inputs.dense_layout(n_samples=2, seed=5)
    P1 = lay[0][:3].copy()
    P1[:, 0] = 2.5
    P2 = lay[1].copy()
    P2[:, 0] = 0.7
    for Q in (P1, P2):
        Q[:, 7] -= 2.75
        Q[:, 8] -= 0.75
    P = np.vstack([P1, P2])
    steps, dt = 100, 5e-5
    obs, speed, st = run_forward(ctx, dtype, [64, 80], [3, 8], P, steps, dt, 50)
    assert list(st) == [0, 0]
    r1 = oracle_core.forward(P1, 64, steps, dt, 50)
    r2 = oracle_core.forward(P2, 80, steps, dt, 50)
    for m in range(3):
        check_traj(obs[m], r1["obs"][m], np.array([P1[m, 7] + 1.0, P1[m, 8]]), tol, dtype, steps, 3.0)
    for m in range(8):
        check_traj(obs[3 + m], r2["obs"][m], np.array([P2[m, 7] + 1.0, P2[m, 8]]), tol, dtype, steps, 3.0)


def oracle_velocity_path(oracle_core, P, N, steps, dt):
    """Sum over the steps of dt |u|_2, u the velocity of all points of the
    system at that step, along the oracle's own run (forces, velocity sum
    and Euler update of the oracle, step by step)."""
    ds = 1.0 / (N - 1)
    x = np.concatenate([p[7] + np.arange(N) * ds for p in P])
    y = np.concatenate([np.full(N, p[8]) for p in P])
    total = 0.0
    for k in range(steps):
        F = [oracle_core.forces(x[m * N:(m + 1) * N], y[m * N:(m + 1) * N], p[1], p[2],
                                oracle_core.kappa0(N, p[3], p[5], p[4], p[6], k * dt)) for m, p in enumerate(P)]
        ux, uy = oracle_core.velocity(x, y, np.concatenate([f[0] for f in F]), np.concatenate([f[1] for f in F]),
                                      P[0, 0], 1.5 * ds)
        total += dt * np.sqrt(np.sum(ux * ux + uy * uy))
        x, y = x + dt * ux, y + dt * uy
    return total


@pytest.mark.parametrize("dtype,tol", [(swim.SWIM_F64, 1e-12), (swim.SWIM_F32, 1e-4)])
def test_large_system_over_several_tiles_matches_oracle(ctx, oracle_core, dtype, tol):
    """8 interacting swimmers of N = 140 (1120 points: the per-step
    large-system kernel with two LDS tiles of sources), 20 steps of dt = 5e-5,
    heads every 10 steps.

    FP64: the bar is the per-evaluation one (1e-12 of the velocity norm of
    the whole system, test_pair_velocity_matches_oracle) carried through the
    run: a head may be off by 4e-12 sum_k dt |u_k|_2 (the factor 4 covers the
    feedback of position errors through the forces over 20 steps).  Some
    heads move only a few 1e-3 here while the snapping filaments carry
    velocities of ~70, so a bar relative to each head's own displacement
    would ask for more than the evaluation bar (measured 3.6e-13 absolute
    against 2.4e-13 for 1e-12 sum_k dt |u_k|_2).  FP32: 1e-4 of each head's
    displacement series plus the rounding floor (check_traj)."""
    lay = inputs.dense_layout(n_samples=2, seed=5)
    P = lay[1].copy()
    P[:, 0] = 0.7
    P[:, 7] -= 2.75
    P[:, 8] -= 0.75
    steps, dt = 20, 5e-5
    obs, speed, st = run_forward(ctx, dtype, [140], [8], P, steps, dt, 10)
    assert list(st) == [0]
    ref = oracle_core.forward(P, 140, steps, dt, 10)
    assert ref["status"] == 0
    if dtype == swim.SWIM_F64:
        allow = 4.0 * tol * oracle_velocity_path(oracle_core, P, 140, steps, dt)
        err = [float(np.max(np.linalg.norm(obs[m] - ref["obs"][m], axis=-1))) for m in range(8)]
        print({"allow": allow, "err": err})
        assert max(err) <= allow, (err, allow)
    else:
        for m in range(8):
            check_traj(obs[m], ref["obs"][m], np.array([P[m, 7] + 1.0, P[m, 8]]), tol, dtype, steps, 3.0)


def _forward_eps(ctx, dtype, N, nsw, P, steps, dt, oe, eps_over_ds):
    td = DT[dtype]
    nfil = P.shape[0]
    obs = torch.full((nfil, steps // oe, 2), float("nan"), dtype=td, device="cuda")
    speed = torch.empty(nfil, dtype=td, device="cuda")
    status = torch.empty(len(N), dtype=torch.int32, device="cuda")
    swim.swim_forward(ctx, np.asarray(N, np.int32), nsw, dev(P, torch.float64), steps, dt, oe, eps_over_ds, obs,
                      speed, status)
    torch.cuda.synchronize()
    return obs.cpu().double().numpy(), status.cpu().numpy()


def test_large_system_symmetric_step_matches_one_sided(ctx):
    """The FP32 large-system step at its automatic choice (every pair once for
    both points, tile pairs of 256 points, partial sums reduced in a fixed
    order) against the one-sided kernel (every ordered pair, one target per
    lane): both accumulate in FP64 from the same FP32 table, so they differ
    by FP64 rounding of differently ordered sums; 1e-6 of each head's
    displacement.  Cases: 8 swimmers of N = 140 (1120 points, five tiles, the
    last partly filled; 40 steps of 5e-5); 8 swimmers of N = 80 in two groups
    at opposite corners of the position bound with eps = 0.05 ds, whose
    cross pairs (r ~ 2800 > 2^22 eps) lie beyond the FP32 table and take the
    direct pass (20 steps of 2e-6, stable at this eps on the oracle; the
    FP32 run also against the FP64 one at 1e-4); and one N = 128 swimmer at
    eps = 0.08 ds, which the host sends to the large-system step because its
    pairs could leave the table (40 steps of 5e-7, against FP64 at 1e-4).
    The far pairs' contributions are tiny here (each filament's forces sum
    to zero), so these cases check that the direct pass and the routing run
    and agree, not the far field's size.  The symmetric runs repeat bit for
    bit."""
    lay = inputs.dense_layout(n_samples=2, seed=5)
    P1 = lay[1].copy()
    P1[:, 0] = 0.7
    P1[:, 7] -= 2.75
    P1[:, 8] -= 0.75
    P2 = inputs.dense_layout(n_samples=1, seed=5)[0].copy()
    P2[:, 0] = 0.7
    P2[:, 7] -= 2.75
    P2[:, 8] -= 0.75
    P2[:4, 7:9] -= 985.0
    P2[4:, 7:9] += 985.0
    P3 = inputs.param_rows(1, alpha=1.0)
    try:
        for Nn, nsw, P, steps, dt, oe, e in ((140, 8, P1, 40, 5e-5, 10, 1.5), (80, 8, P2, 20, 2e-6, 5, 0.05),
                                             (128, 1, P3, 40, 5e-7, 10, 0.08)):
            out = {}
            x0 = P[:, 7:9] + np.array([1.0, 0.0])
            for big in ((0, 1, 0) if nsw > 1 else (0,)):
                swim.swim_set_option(ctx, swim.SWIM_OPT_BIG_TPL, big)
                obs, st = _forward_eps(ctx, swim.SWIM_F32, [Nn], [nsw], P, steps, dt, oe, e)
                assert list(st) == [0], (Nn, big, st)
                if big in out:
                    assert np.array_equal(obs, out[big]), "symmetric runs are not bit-reproducible"
                out[big] = obs
            if 1 in out:
                for m in range(nsw):
                    disp = np.linalg.norm(out[1][m] - x0[m])
                    err = np.linalg.norm(out[0][m] - out[1][m])
                    floor = np.linalg.norm(np.spacing(np.abs(out[1][m]).astype(np.float32)))
                    assert err <= 1e-6 * disp + floor, (Nn, m, err, disp)
            if e < 1.0:
                o64, st = _forward_eps(ctx, swim.SWIM_F64, [Nn], [nsw], P, steps, dt, oe, e)
                assert list(st) == [0]
                for m in range(nsw):
                    disp = np.linalg.norm(o64[m] - x0[m])
                    err = np.linalg.norm(out[0][m] - o64[m])
                    floor = np.linalg.norm(np.spacing(np.abs(o64[m]).astype(np.float32)))
                    print({"N": Nn, "m": m, "fp32_vs_fp64": err / disp})
                    assert err <= 1e-4 * disp + floor, (Nn, m, err, disp)
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_BIG_TPL, 0)


def test_dense_sample_velocity_at_full_size(ctx, oracle_core):
    """One velocity evaluation of the large-N dense workload at its full size:
    sample 0 (8 swimmers x 512 points on the 2 x 4 grid, alpha from seed 3)
    at its initial configuration, forces of the oracle at t = 0, all 4096
    velocities against the FP64 oracle in FP32 and FP64."""
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
    for dtype, tol in ((swim.SWIM_F32, 1e-5), (swim.SWIM_F64, 1e-12)):
        # both sides take the same inputs: the FP32 run's positions and
        # forces rounded to FP32 (at |x| ~ 5 that rounding alone moves
        # neighbouring points by 1e-4 of their spacing)
        Xd, Yd, FXd, FYd = (a.astype(NP[dtype]).astype(np.float64) for a in (X, Y, FX, FY))
        ox, oy = oracle_core.velocity(Xd, Yd, FXd, FYd, lay[0, 0], eps)
        td = DT[dtype]
        ux = torch.empty(4096, dtype=td, device="cuda")
        uy = torch.empty_like(ux)
        swim.swim_pair_velocity(ctx, np.array([0, 4096]), [lay[0, 0]], [eps], dev(Xd, td), dev(Yd, td),
                                dev(FXd, td), dev(FYd, td), ux, uy)
        torch.cuda.synchronize()
        g = np.concatenate([ux.cpu().double().numpy(), uy.cpu().double().numpy()])
        ref = np.concatenate([ox, oy])
        assert rel(g, ref) < tol and rel_max(g, ref) < tol, (dtype, rel(g, ref), rel_max(g, ref))


def test_dense_sample_run(ctx, oracle_core):
    """The dense workload's sample 0 (8 swimmers x 512 points, its alpha) as
    a run at the benchmark's dt = 2e-5/32: the FP64 run against the oracle
    over its first 3 steps (the oracle sums 4096^2 pairs per step on the host
    cores), head of every swimmer every step, at 1e-12 of the displacement;
    the FP32 run against the FP64 run over 100 steps, every 10, at 1e-4 of
    the displacement (plus one FP32 spacing of the stored positions)."""
    lay = inputs.dense_layout(n_samples=1, seed=3)[0]
    P = dev(lay, torch.float64)
    dt = 2e-5 / 32
    x0 = lay[:, 7:9] + np.array([1.0, 0.0])
    out = {}
    for dtype, steps, oe in ((swim.SWIM_F64, 3, 1), (swim.SWIM_F64, 100, 10), (swim.SWIM_F32, 100, 10)):
        td = DT[dtype]
        obs = torch.empty((8, steps // oe, 2), dtype=td, device="cuda")
        speed = torch.empty(8, dtype=td, device="cuda")
        st = torch.empty(1, dtype=torch.int32, device="cuda")
        swim.swim_forward(ctx, [512], [8], P, steps, dt, oe, 1.5, obs, speed, st)
        torch.cuda.synchronize()
        assert st.item() == 0
        out[(dtype, steps)] = obs.cpu().double().numpy()
    ref = oracle_core.forward(lay, 512, 3, dt, 1)
    assert ref["status"] == 0
    got = out[(swim.SWIM_F64, 3)]
    disp = np.linalg.norm(ref["obs"] - x0[:, None, :])
    err = np.linalg.norm(got - ref["obs"])
    print({"fp64_vs_oracle": err / disp})
    assert err <= 1e-12 * disp
    o64, o32 = out[(swim.SWIM_F64, 100)], out[(swim.SWIM_F32, 100)]
    disp = np.linalg.norm(o64 - x0[:, None, :])
    floor = np.linalg.norm(np.spacing(np.abs(o64).astype(np.float32)))
    err = np.linalg.norm(o32 - o64)
    print({"fp32_vs_fp64": err / disp})
    assert err <= 1e-4 * disp + floor


def test_blowup_and_bad_parameters_are_statuses(ctx):
    P = inputs.param_rows(3, alpha=2.0)
    P[0, 1], P[0, 2] = 1.0, 1e4      # beyond the explicit-Euler bound at N = 128
    P[2, 0] = 1000.0                  # alpha * eps > 1
    obs, speed, st = run_forward(ctx, swim.SWIM_F32, [128, 128, 128], None, P, 400, 5e-5, 100)
    assert st[0] in (swim.SWIM_ST_NONFINITE, swim.SWIM_ST_BOUND)
    assert st[1] == swim.SWIM_ST_OK
    assert st[2] == swim.SWIM_ST_BADPARAM
    assert np.isnan(speed[0]) and np.isnan(speed[2]) and np.isfinite(speed[1])
    assert np.all(np.isnan(obs[2])) and np.all(np.isfinite(obs[1]))


def test_argument_errors(ctx):
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(swim.SwimError):
        swim.swim_pair_velocity(ctx, [0, 4], [1.0], [-0.1], x, x, x, x, x, x)
    with pytest.raises(swim.SwimError):
        swim.swim_pair_velocity(ctx, [0, 4], [100.0], [0.1], x, x, x, x, x, x)
    P = dev(inputs.param_rows(1), torch.float64)
    with pytest.raises(swim.SwimError):
        swim.swim_forward(ctx, [2], None, P, 10, 1e-4, 1, 1.5, x, x[:1], torch.zeros(1, dtype=torch.int32,
                                                                                         device="cuda"))
    with pytest.raises(swim.SwimError):
        swim.swim_forward(ctx, [64], None, P, 0, 1e-4, 1, 1.5, x, x[:1], torch.zeros(1, dtype=torch.int32,
                                                                                          device="cuda"))
    # one wave per system for a 512-point system would carry nine point
    # windows per lane: that shape is not built, and asking for it is an error
    obs = torch.empty((1, 1, 2), dtype=torch.float32, device="cuda")
    swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, 1)
    try:
        with pytest.raises(swim.SwimError, match="SWIM_OPT_WPS"):
            swim.swim_forward(ctx, [512], None, P, 1, 1e-6, 1, 1.5, obs, x[:1], torch.zeros(1, dtype=torch.int32,
                                                                                            device="cuda"))
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, 0)


def test_abc_distance_and_select_match_oracle(ctx):
    from oracle import abc
    rng = np.random.Generator(np.random.PCG64(8))
    n, n_obs = 5000, 50
    data = rng.standard_normal((n_obs, 2))
    obs = (data[None] + rng.standard_normal((n, n_obs, 2)) * rng.uniform(0.01, 1, (n, 1, 1))).astype(np.float32)
    status = np.zeros(n, np.int32)
    status[::97] = 1
    obs[5, 3, 0] = np.nan
    dist = torch.empty(n, dtype=torch.float64, device="cuda")
    swim.abc_distance(ctx, dev(obs, torch.float32), dev(data, torch.float64), dev(status, torch.int32), dist)
    tol = torch.empty(1, dtype=torch.float64, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")
    swim.abc_select(ctx, dist, 0.05, tol, acc)
    torch.cuda.synchronize()
    ref = abc.distance(np.where(status[:, None, None] != 0, np.nan, obs.astype(np.float64)), data)
    got = dist.cpu().numpy()
    np.testing.assert_allclose(got[np.isfinite(ref)], ref[np.isfinite(ref)], rtol=1e-14)
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    # the tolerance is an order statistic of the GPU distances: compare exactly
    assert tol.item() == abc.tolerance(got, 0.05)
    assert np.array_equal(acc.cpu().numpy().astype(bool), abc.accept(got, tol.item()))
