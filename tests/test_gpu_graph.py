"""Captured forward runs (hipGraph) against eager launches.

A batch mixing persistent-kernel systems and a large system (per-step
kernel, one launch per step) runs eagerly, then with capture on a repeated
layout: first sight eager, the repeat captured and launched, later calls
replayed, with unrelated eager work and synchronizations between the
calls.  Every call's outputs must equal the eager run's bit for bit
(the kernels are deterministic), also after the parameter values change in
place between replays.
"""
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


def _layout():
    lay = inputs.dense_layout(n_samples=1, seed=7)[0]
    big = lay.copy()
    big[:, 0] = 1.3
    big[:, 7] -= 2.75
    big[:, 8] -= 0.75
    small = inputs.param_rows(3, Sb=0.05, Ss=500.0)
    small[:, 0] = [0.0, 2.0, 7.5]
    P = np.vstack([small, big])
    N = np.array([64, 96, 128, 80], np.int32)
    nsw = np.array([1, 1, 1, 8], np.int32)
    return P, N, nsw


@pytest.mark.parametrize("dtype", [swim.SWIM_F32, swim.SWIM_F64])
def test_graph_replays_match_eager(ctx, dtype):
    P, N, nsw = _layout()
    td = torch.float32 if dtype == swim.SWIM_F32 else torch.float64
    steps, dt, oe = 120, 2e-5, 40
    nfil = P.shape[0]
    Pd = torch.from_numpy(P).cuda()
    obs = torch.empty((nfil, steps // oe, 2), dtype=td, device="cuda")
    speed = torch.empty(nfil, dtype=td, device="cuda")
    status = torch.empty(len(N), dtype=torch.int32, device="cuda")
    done = torch.empty(len(N), dtype=torch.int32, device="cuda")

    def run():
        obs.fill_(-1.0)
        speed.fill_(-1.0)
        torch.cuda.synchronize()
        swim.swim_forward(ctx, N, nsw, Pd, steps, dt, oe, 1.5, obs, speed, status, done)
        torch.cuda.synchronize()
        return obs.cpu().numpy().copy(), speed.cpu().numpy().copy(), status.cpu().numpy().copy(), \
            done.cpu().numpy().copy()

    # unrelated eager work between calls
    x = torch.randn(512, dtype=td, device="cuda")
    u = torch.empty_like(x)
    v = torch.empty_like(x)

    def other():
        swim.swim_pair_velocity(ctx, np.array([0, 512]), [0.5], [0.01], x, x.flip(0).contiguous(), x, x, u, v)
        torch.cuda.synchronize()

    # FP64 takes the reading's blob: the paper blob's per-pair quadrature
    # would make the 640-point system's seven runs minutes long (its FP32
    # tables, the default, are replayed here; test_gpu_paper_blob replays a
    # graph that rebuilds them)
    blob = swim.SWIM_BLOB_READING if dtype == swim.SWIM_F64 else swim.SWIM_BLOB_PAPER
    try:
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, blob)
        swim.swim_set_option(ctx, swim.SWIM_OPT_GRAPH, 0)
        ref = run()
        assert np.all(ref[2] == 0) and np.all(ref[3] == steps)
        P2 = P.copy()
        P2[:, 0] = P2[:, 0] * 0.5 + 0.1
        Pd.copy_(torch.from_numpy(P2))
        torch.cuda.synchronize()
        ref2 = run()
        Pd.copy_(torch.from_numpy(P))
        torch.cuda.synchronize()
        swim.swim_set_option(ctx, swim.SWIM_OPT_GRAPH, 1)
        launches0 = swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_LAUNCHES)
        captures0 = swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_CAPTURES)
        outs = []
        for call in range(4):
            outs.append(run())
            other()
        assert swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_CAPTURES) - captures0 == 1
        assert swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_LAUNCHES) - launches0 == 3
        for o in outs:
            for a, b in zip(o, ref):
                assert np.array_equal(a, b)
        # new parameter values in the same buffer: the replay reads them
        Pd.copy_(torch.from_numpy(P2))
        torch.cuda.synchronize()
        for call in range(2):
            o = run()
            other()
            for a, b in zip(o, ref2):
                assert np.array_equal(a, b)
        assert swim.swim_get_option(ctx, swim.SWIM_OPT_GRAPH_LAUNCHES) - launches0 == 5
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_GRAPH, 1)
        swim.swim_set_option(ctx, swim.SWIM_OPT_BLOB, swim.SWIM_BLOB_PAPER)


def test_kernel_timing_option(ctx):
    """SWIM_OPT_TIME_KERNEL: timed calls (eager, events around the
    persistent launches) give the same outputs as untimed ones, and
    SWIM_OPT_KERNEL_US reports a positive interval no longer than the call;
    reading it before any timed call, or setting a bad value, is an error."""
    import time
    P, N, nsw = _layout()
    steps, dt, oe = 120, 2e-5, 40
    nfil = P.shape[0]
    Pd = torch.from_numpy(P).cuda()
    outs = []
    with pytest.raises(swim.SwimError):
        swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, 2)
    swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, 1)
    try:
        with pytest.raises(swim.SwimError):
            swim.swim_get_option(ctx, swim.SWIM_OPT_KERNEL_US)
        for timed in (1, 0):
            swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, timed)
            obs = torch.empty((nfil, steps // oe, 2), dtype=torch.float32, device="cuda")
            speed = torch.empty(nfil, dtype=torch.float32, device="cuda")
            status = torch.empty(len(N), dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            swim.swim_forward(ctx, N, nsw, Pd, steps, dt, oe, 1.5, obs, speed, status)
            if timed:
                us = swim.swim_get_option(ctx, swim.SWIM_OPT_KERNEL_US)
                wall_us = 1e6 * (time.perf_counter() - t0)
                assert 0 < us <= wall_us, (us, wall_us)
            torch.cuda.synchronize()
            outs.append((obs.cpu().numpy(), speed.cpu().numpy(), status.cpu().numpy()))
    finally:
        swim.swim_set_option(ctx, swim.SWIM_OPT_TIME_KERNEL, 0)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b, equal_nan=True)
