"""Pins of the full sperm-model oracle (Appendix: tapered beat, eqs. EFB,
curva, EFT for flagellum and head, the neck springs and angle energy, eq.
Fenergy) against what the geometry and the mathematics fix:

* the preferred curvature is the second s-derivative of the tapered beat
  (finite differences of the printed beat form);
* each energy term in closed form on a configuration built for it: a
  uniformly stretched flagellum, a flagellum bent into a circular arc, a
  scaled head circle (ring and diameter springs, discrete curvature of a
  regular polygon 2/(R (1 + cos dth))), a rigidly shifted head (neck
  springs), a rigidly rotated head (neck angle);
* forces are minus the gradient of the energy (central differences), term
  by term;
* internal forces carry no net force or torque;
* a passive swimmer (no beat) only loses energy along its run;
* two swimmers placed as mirror images (phases 0 and pi) stay mirror images.
"""
import numpy as np
import pytest

from oracle import core

pytestmark = pytest.mark.usefixtures("reading_blob_module")

NF, NH = 50, 24
DS = 1.0 / (NF - 1)
HR, DN = 0.05, DS
DTH = 2 * np.pi / NH
CH = 2 * HR * np.sin(DTH / 2)
TABLE = dict(alpha=1.0, KC=8.0, KT=1e4, KHT=1e4, KHC=0.8, KNT=500.0, KNA=1e4, a=0.1, eta=2 * np.pi,
             omega=4 * np.pi)


def row(**kw):
    d = dict(TABLE)
    d.update(kw)
    return np.array([d[f] for f in core.SPERM_FIELDS])


def only(term, **kw):
    """A system row with every stiffness zero except `term`."""
    z = dict(KC=0.0, KT=0.0, KHT=0.0, KHC=0.0, KNT=0.0, KNA=0.0)
    z[term] = TABLE[term]
    z.update(kw)
    return row(**z)


def energy(r, x, y, phase=0.0, t=0.0):
    return core.sperm_energy(NF, NH, HR, DN, r, phase, t, x, y)


def test_zhat_is_the_second_derivative_of_the_tapered_beat():
    rng = np.random.Generator(np.random.PCG64(1))
    s = rng.uniform(0, 1, 40)
    a, eta, om = 0.1, 2 * np.pi, 4 * np.pi
    for t, ph in ((0.0, 0.0), (0.37, 1.1), (3.2, -2.0)):
        def yhat(u):
            return a * (1 - u) * np.sin(eta * u - om * t + ph)
        h = 1e-4
        fd = (yhat(s + h) - 2 * yhat(s) + yhat(s - h)) / h ** 2
        got = core.sperm_zhat(s, a, eta, om, ph, t)
        assert np.max(np.abs(got - fd)) < 1e-5
        # taper: the beat amplitude vanishes at the head end s = 1, where
        # only the -2 a eta cos term of the curvature remains
        assert core.sperm_zhat([1.0], a, eta, om, ph, t)[0] == pytest.approx(-2 * a * eta * np.cos(eta - om * t + ph))


def test_initial_geometry():
    x, y = core.sperm_initial(NF, NH, HR, DN, 0.3, -0.2)
    assert np.allclose(x[:NF], 0.3 + DS * np.arange(NF), atol=1e-15) and np.all(y[:NF] == -0.2)
    c = np.array([0.3 + 1.0 + DN + HR, -0.2])
    hx, hy = x[NF:], y[NF:]
    assert np.allclose(np.hypot(hx - c[0], hy - c[1]), HR, atol=1e-15)
    # the head point at angle pi sits dN right of the last flagellum point
    assert hx[NH // 2] - x[NF - 1] == pytest.approx(DN, abs=1e-15)
    assert abs(np.mean(hx) - c[0]) < 1e-15 and abs(np.mean(hy) - c[1]) < 1e-15


def test_energy_terms_in_closed_form():
    x0, y0 = core.sperm_initial(NF, NH, HR, DN)
    c = np.array([1.0 + DN + HR, 0.0])
    # at rest every spring is at its rest length and the flagellum is straight
    for term in ("KT", "KHT", "KNT", "KNA"):
        assert abs(energy(only(term), x0, y0)) < 1e-20 * TABLE[term] + 1e-18
    # straight flagellum against the preferred curvature: K_C sum zhat^2 ds
    s = DS * np.arange(1, NF - 1)
    for t in (0.0, 0.21):
        zh = core.sperm_zhat(s, 0.1, 2 * np.pi, 4 * np.pi, 0.4, t)
        assert energy(only("KC"), x0, y0, 0.4, t) == pytest.approx(8.0 * np.sum(zh ** 2) * DS, rel=1e-13)
    # regular polygon: discrete curvature 2/(R (1 + cos dth)) at every node
    kap = 2.0 / (HR * (1 + np.cos(DTH)))
    assert energy(only("KHC"), x0, y0) == pytest.approx(0.8 * NH * (kap - 1 / HR) ** 2 * CH, rel=1e-12)
    # flagellum uniformly stretched by lam: K_T (lam - 1)^2 (nf - 1) ds
    lam = 1.003
    xs = x0.copy()
    xs[:NF] = lam * x0[:NF]
    assert energy(only("KT"), xs, y0) == pytest.approx(1e4 * (lam - 1) ** 2, rel=1e-9)
    # head circle scaled by lam about its centre: ring and diameter springs,
    # curvature 2/(lam R (1 + cos dth))
    xh, yh = x0.copy(), y0.copy()
    xh[NF:] = c[0] + lam * (x0[NF:] - c[0])
    yh[NF:] = lam * y0[NF:]
    ring = NH * 1e4 * (lam - 1) ** 2 * CH + (NH // 2) * 1e4 * (lam - 1) ** 2 * 2 * HR
    assert energy(only("KHT"), xh, yh) == pytest.approx(ring, rel=1e-9)
    assert energy(only("KHC"), xh, yh) == pytest.approx(0.8 * NH * (kap / lam - 1 / HR) ** 2 * CH, rel=1e-12)
    # flagellum on a circular arc of radius R (angle step phi between
    # points): discrete curvature 2/(R (1 + cos phi)) at interior nodes
    R, phi = 0.7, 0.02
    xa, ya = x0.copy(), y0.copy()
    th = phi * np.arange(NF)
    xa[:NF] = R * np.sin(th)
    ya[:NF] = R * (1 - np.cos(th))
    ka = 2.0 / (R * (1 + np.cos(phi)))
    zh = core.sperm_zhat(s, 0.1, 2 * np.pi, 4 * np.pi, 0.0, 0.1)
    assert energy(only("KC"), xa, ya, 0.0, 0.1) == pytest.approx(8.0 * np.sum((ka - zh) ** 2) * DS, rel=1e-11)
    # head shifted right by delta: neck springs in closed form
    delta = 2e-3
    xt = x0.copy()
    xt[NF:] += delta
    cd, sd = np.cos(DTH), np.sin(DTH)

    def neck(gap):
        # last point to pi -+ dth, pi, pi + dth; the one before to pi -+ dth
        return [np.hypot(gap + HR * (1 - cd), HR * sd), gap, np.hypot(gap + HR * (1 - cd), HR * sd),
                np.hypot(DS + gap + HR * (1 - cd), HR * sd), np.hypot(DS + gap + HR * (1 - cd), HR * sd)]
    L0, L1 = np.array(neck(DN)), np.array(neck(DN + delta))
    assert energy(only("KNT"), xt, y0) == pytest.approx(np.sum(500.0 * (L1 / L0 - 1) ** 2 * L0), rel=1e-9)
    # head rotated by beta about its centre: z1 . z2 = 2 R sin(dth) sin(beta) (dN + R)
    beta = 0.05
    xr, yr = x0.copy(), y0.copy()
    dx, dy = x0[NF:] - c[0], y0[NF:]
    xr[NF:] = c[0] + np.cos(beta) * dx - np.sin(beta) * dy
    yr[NF:] = np.sin(beta) * dx + np.cos(beta) * dy
    dot = 2 * HR * sd * np.sin(beta) * (DN + HR)
    assert energy(only("KNA"), xr, yr) == pytest.approx(1e4 * dot ** 2, rel=1e-9)


def perturbed(seed, scale=2e-3):
    x, y = core.sperm_initial(NF, NH, HR, DN, 0.1, 0.2)
    rng = np.random.Generator(np.random.PCG64(seed))
    return x + scale * rng.normal(size=x.size) * DS, y + scale * 20 * rng.normal(size=y.size) * DS


@pytest.mark.parametrize("term", ["KC", "KT", "KHT", "KHC", "KNT", "KNA", None])
def test_forces_are_minus_the_energy_gradient(term):
    r = row() if term is None else only(term)
    x, y = perturbed(3)
    ph, t = 0.7, 0.13
    fx, fy = core.sperm_forces(NF, NH, HR, DN, r, ph, t, x, y)
    h = 1e-7
    gx, gy = np.empty_like(x), np.empty_like(y)
    for i in range(x.size):
        for arr, g in ((x, gx), (y, gy)):
            keep = arr[i]
            arr[i] = keep + h
            ep = energy(r, x, y, ph, t)
            arr[i] = keep - h
            em = energy(r, x, y, ph, t)
            arr[i] = keep
            g[i] = (ep - em) / (2 * h)
    scale = max(np.max(np.abs(fx)), np.max(np.abs(fy)))
    assert scale > 0
    assert np.max(np.abs(fx + gx)) < 1e-5 * scale and np.max(np.abs(fy + gy)) < 1e-5 * scale


def test_internal_forces_have_no_net_force_or_torque():
    x, y = perturbed(4, 5e-3)
    fx, fy = core.sperm_forces(NF, NH, HR, DN, row(), 0.3, 0.7, x, y)
    mag = np.sum(np.hypot(fx, fy))
    assert abs(fx.sum()) < 1e-12 * mag and abs(fy.sum()) < 1e-12 * mag
    assert abs(np.sum(x * fy - y * fx)) < 1e-12 * mag * np.max(np.hypot(x, y))


def test_passive_swimmer_loses_energy():
    """No beat (a = 0): the dynamics dX/dt = M F with F = -dE/dX and a
    positive definite Brinkmanlet mobility only dissipate; the run starts
    from the closed-form head-bending energy of the regular polygon."""
    r = row(a=0.0)
    x0, y0 = core.sperm_initial(NF, NH, HR, DN)
    kap = 2.0 / (HR * (1 + np.cos(DTH)))
    E = [energy(r, x0, y0)]
    assert E[0] == pytest.approx(0.8 * NH * (kap - 1 / HR) ** 2 * CH, rel=1e-12)
    for steps in (5, 10, 20, 40):
        out = core.sperm_forward(r, [[0.0, 0.0, 0.0]], NF, NH, 0.045, HR, DN, steps, 1e-6, 0)
        assert out["status"] == 0
        E.append(energy(r, out["x"], out["y"]))
    assert np.all(np.diff(E) < 0), E


def test_two_mirrored_swimmers_stay_mirrored():
    d, steps = 0.3, 40
    sw = np.array([[0.0, d / 2, 0.0], [0.0, -d / 2, np.pi]])
    out = core.sperm_forward(row(), sw, NF, NH, 0.045, HR, DN, steps, 1e-5, 10)
    assert out["status"] == 0
    for k in ("head", "tail"):
        a, b = out[k][0], out[k][1]
        assert np.max(np.abs(a[:, 0] - b[:, 0])) < 1e-12
        assert np.max(np.abs(a[:, 1] + b[:, 1])) < 1e-12
    # they moved (the check is not vacuous)
    assert np.max(np.abs(out["tail"][0, -1] - out["tail"][0, 0])) > 1e-4


def test_forward_samples_and_one_step():
    """Sample 0 is the initial state; one step equals X + dt u(X) with u the
    velocity sum of the forces of both swimmers (the run's assembly of
    pinned parts: which forces, phases, fluid and blob)."""
    r = row(alpha=0.6)
    sw = np.array([[0.0, 0.0, 0.3], [0.2, 0.5, 1.4]])
    out = core.sperm_forward(r, sw, NF, NH, 0.045, HR, DN, 1, 1e-5, 1)
    xs, ys = [], []
    for m in range(2):
        x, y = core.sperm_initial(NF, NH, HR, DN, sw[m, 0], sw[m, 1])
        assert np.allclose(out["head"][m, 0], [x[NF:].mean(), y[NF:].mean()], atol=1e-15)
        assert np.array_equal(out["tail"][m, 0], [x[0], y[0]])
        xs.append(x)
        ys.append(y)
    F = [core.sperm_forces(NF, NH, HR, DN, r, sw[m, 2], 0.0, xs[m], ys[m]) for m in range(2)]
    X, Y = np.concatenate(xs), np.concatenate(ys)
    ux, uy = core.velocity(X, Y, np.concatenate([f[0] for f in F]), np.concatenate([f[1] for f in F]), 0.6, 0.045)
    np.testing.assert_allclose(out["x"], X + 1e-5 * ux, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out["y"], Y + 1e-5 * uy, rtol=0, atol=1e-15)


def test_observables():
    """Head-centre velocities of a run and the pair distances of two
    swimmers: at sample 0 the heads and tails sit exactly d apart; a run's
    velocities sum to the head's total displacement over the time."""
    d = 0.5
    sw = np.array([[0.0, d / 2, 0.0], [0.0, -d / 2, 0.0]])
    out = core.sperm_forward(row(), sw, NF, NH, 0.045, HR, DN, 60, 1e-5, 20)
    v = core.sperm_head_velocity(out["head"], 20 * 1e-5)
    assert v.shape == (3, 2)
    np.testing.assert_allclose(v.sum(0) * 20e-5, out["head"][0, -1] - out["head"][0, 0], rtol=1e-12, atol=1e-17)
    dist = core.sperm_pair_distances(out["head"], out["tail"])
    assert dist.shape == (3, 2)
    h, t = out["head"], out["tail"]
    assert np.hypot(*(t[0, 0] - t[1, 0])) == pytest.approx(d, abs=1e-15)
    assert np.hypot(*(h[0, 0] - h[1, 0])) == pytest.approx(d, abs=1e-15)
    np.testing.assert_allclose(dist[:, 0], np.hypot(*(t[0, 1:] - t[1, 1:]).T), rtol=1e-15)
    np.testing.assert_allclose(dist[:, 1], np.hypot(*(h[0, 1:] - h[1, 1:]).T), rtol=1e-15)
    # a uniformly moving head: constant velocity
    H = np.zeros((1, 5, 2))
    H[0, :, 0] = 0.3 + 0.01 * np.arange(5)
    H[0, :, 1] = -0.002 * np.arange(5)
    np.testing.assert_allclose(core.sperm_head_velocity(H, 0.5), np.tile([0.02, -0.004], (4, 1)), rtol=1e-12)
