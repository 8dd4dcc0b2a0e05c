"""Parity at the batched workload's full size as first stated: 4096 prior
draws (Philox seed 1), N = 128, 5000 steps of dt = 5e-5 with the closed-form
blob, FP32, default launch shapes, one swim_forward call.  (The benchmark
times the same batch over the same time in 10000 steps of 2.5e-5 with the
paper's blob, away from the stability edge: that configuration is held to
1e-4 in test_gpu_paper_blob.py::test_batched_workload_as_benchmarked.)

Sampled outputs the oracle recomputes one by one: two runs that complete
(the first in draw order and the one closest to the data) and the two
earliest blow-ups.  Over the whole batch, the tolerance and accept set
follow the oracle's definitions applied to the GPU distances.

The completed samples sit near forward Euler's stability edge (dt * rho
close to 2, like the data's true parameters).  There the initial snap of
the straight filament to its preferred shape excites stiff, slowly damped
oscillating modes that amplify the per-step rounding of the FP32 velocity
sums (~1e-6) by ~1e3 over the first few hundred steps, and what remains of
that transient depends on the order in which the partial sums round: runs
of the same system with 1 to 16 wavefronts per system differ from each
other by up to ~7e-4 in the mean speed and RMS distance.  So FP64 is held
to 1e-11 on the complete series; FP32 is checked as five rounding draws
(the batch run and re-runs with 1, 2, 4 and 8 wavefronts per system): each
within 2e-3 of the oracle on the trajectory summaries the ABC uses (the
mean speed, the RMS distance to the data) and on the displacement series
from step 1000 on, and their mean closer to the oracle than the draws are
to each other (no bias beyond the rounding spread).  Runs away from the
stability edge meet 1e-4 (test_gpu_parity.py).
"""
import os

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("reading_blob_module")]

torch = pytest.importorskip("torch")

from paper_1910_12007_amd import inputs, swim  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = swim.Context(0)
    swim.swim_set_option(c, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_READING)
    yield c
    c.close()


def fp32_rerun(ctx, prow, N, steps, dt, oe, data, wps):
    """One FP32 run of one system with wps wavefronts per system: its head
    series, mean speed and RMS distance to the data (oracle definition)."""
    from oracle import abc
    swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, wps)
    try:
        obs = torch.empty((1, steps // oe, 2), dtype=torch.float32, device="cuda")
        speed = torch.empty(1, dtype=torch.float32, device="cuda")
        status = torch.empty(1, dtype=torch.int32, device="cuda")
        swim.swim_forward(ctx, [N], None, torch.from_numpy(prow[None].copy()).cuda(), steps, dt, oe, 1.5, obs, speed,
                          status)
        torch.cuda.synchronize()
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_WPS, 0)
    assert status.item() == 0
    ob = obs.cpu().double().numpy()[0]
    return ob, speed.item(), abc.distance(ob[None], data[:steps // oe])[0]


def test_batched_workload_sampled_against_oracle(ctx, oracle_core):
    from oracle import abc
    n, N, steps, dt, oe = 4096, 128, 5000, 5e-5, 100
    theta = swim.abc_prior_draw(1, n, inputs.PRIOR_LO, inputs.PRIOR_HI)
    P = inputs.theta_rows(theta)
    obs = torch.empty((n, steps // oe, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    steps_done = torch.empty(n, dtype=torch.int32, device="cuda")
    swim.swim_forward(ctx, np.full(n, N, np.int32), None, torch.from_numpy(P).cuda(), steps, dt, oe, 1.5, obs,
                      speed, status, steps_done)
    data = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "abc_data_batch.txt"))[:, :2]
    dist = torch.empty(n, dtype=torch.float64, device="cuda")
    tol = torch.empty(1, dtype=torch.float64, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")
    swim.abc_distance(ctx, obs, torch.from_numpy(data).cuda(), status, dist)
    swim.abc_select(ctx, dist, 0.05, tol, acc)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    o = obs.cpu().double().numpy()
    d = dist.cpu().numpy()
    assert tol.item() == abc.tolerance(d, 0.05)
    assert np.array_equal(acc.cpu().numpy().astype(bool), abc.accept(d, tol.item()))
    ok = np.flatnonzero(st == 0)
    bad = np.flatnonzero(st != 0)
    assert 50 < ok.size < n
    x0 = np.array([1.0, 0.0])
    spd = speed.cpu().double().numpy()
    samples = [ok[0], ok[np.argmin(d[ok])]]
    # FP64 runs of the sampled systems at full length, same launch path
    P2 = torch.from_numpy(P[samples]).cuda()
    obs64 = torch.empty((2, steps // oe, 2), dtype=torch.float64, device="cuda")
    sp64 = torch.empty(2, dtype=torch.float64, device="cuda")
    st64 = torch.empty(2, dtype=torch.int32, device="cuda")
    swim.swim_forward(ctx, np.full(2, N, np.int32), None, P2, steps, dt, oe, 1.5, obs64, sp64, st64)
    torch.cuda.synchronize()
    o64 = obs64.cpu().numpy()
    for k, i in enumerate(samples):
        ref = oracle_core.forward(P[i:i + 1], N, steps, dt, oe)
        assert ref["status"] == 0 and st64[k].item() == 0, i
        r = ref["obs"][0]
        # FP64: complete series
        assert np.linalg.norm(o64[k] - r) <= 1e-11 * np.linalg.norm(r - x0), (i, "fp64")
        # FP32: five rounding draws of the same run
        d_ref = abc.distance(r[None], data[:steps // oe])[0]
        late = slice(1000 // oe - 1, None)
        scale = np.linalg.norm(r[late] - x0)
        floor = np.linalg.norm(np.spacing(np.abs(r[late]).astype(np.float32)))
        draws = [(o[i], spd[i], d[i])] + [fp32_rerun(ctx, P[i], N, steps, dt, oe, data, w) for w in (1, 2, 4, 8)]
        for w, (ob, sp, dd) in zip((0, 1, 2, 4, 8), draws):
            assert abs(sp / ref["speed"][0] - 1) < 2e-3, (i, w, sp, ref["speed"][0])
            assert abs(dd / d_ref - 1) < 2e-3, (i, w, dd, d_ref)
            err = np.linalg.norm(ob[late] - r[late])
            assert err <= 2e-3 * scale + floor, (i, w, theta[i], err / scale)
        mean = np.mean([ob for ob, _, _ in draws], axis=0)
        spread = max(np.linalg.norm(a[0][late] - b[0][late]) for a in draws for b in draws)
        assert np.linalg.norm(mean[late] - r[late]) <= spread, (i, np.linalg.norm(mean[late] - r[late]), spread)
    # the two earliest blow-ups blow up in the oracle too
    sd = steps_done.cpu().numpy()
    for i in bad[np.argsort(sd[bad], kind="stable")[:2]]:
        ref = oracle_core.forward(P[i:i + 1], N, steps, dt, oe)
        assert ref["status"] != 0, (i, theta[i], sd[i])
