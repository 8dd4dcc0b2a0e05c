"""Population Monte Carlo over the batched forward model, end to end on the
GPU (abc_step): uneven filament sizes, two generations.  Against the
oracle's definitions: generation 0's proposals are the prior draws; the
tolerance is the ceil(q * completed)-th smallest finite distance and
exactly those particles are accepted; later proposals are the oracle's PMC
proposals from the previous accepted population, inside the prior box;
weights are the oracle's Beaumont weights; the tolerance decreases."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1910_12007_amd import inputs, swim, surrogate_abc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = swim.Context(0)
    yield c
    c.close()


def test_pmc_generations(ctx):
    from oracle import abc
    n, steps = 1024, 1000
    N = inputs.uneven_sizes(n, seed=12)
    model = surrogate_abc.batch_model(steps=steps, dt=5e-5, obs_every=100)
    data = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "abc_data_batch.txt"))[:steps // 100, :2]
    g0 = swim.abc_step(ctx, model, data, N, 3, 0, 0.5)
    assert np.array_equal(g0["theta"], abc.prior_draw(3, n, inputs.PRIOR_LO, inputs.PRIOR_HI))
    d = g0["dist"]
    assert g0["tol"] == abc.tolerance(d, 0.5)
    assert np.array_equal(g0["accept"], abc.accept(d, g0["tol"]))
    nf = int(np.isfinite(d).sum())
    assert 0 < nf < n and g0["accept"].sum() == int(np.ceil(0.5 * nf))
    acc0 = g0["accept"]
    assert abs(g0["w"][acc0].sum() - 1.0) < 1e-12 and np.all(g0["w"][~acc0] == 0)
    g1 = swim.abc_step(ctx, model, data, N, 3, 1, 0.25, g0["theta"][acc0], g0["w"][acc0])
    prop = abc.pmc_propose(3, 1, n, g0["theta"][acc0], g0["w"][acc0], inputs.PRIOR_LO, inputs.PRIOR_HI)
    np.testing.assert_allclose(g1["theta"], prop, rtol=1e-12, atol=0)
    assert np.all(g1["theta"] >= inputs.PRIOR_LO) and np.all(g1["theta"] <= inputs.PRIOR_HI)
    assert g1["tol"] == abc.tolerance(g1["dist"], 0.25)
    acc1 = g1["accept"]
    assert np.array_equal(acc1, abc.accept(g1["dist"], g1["tol"]))
    w_ref = abc.pmc_weights(g1["theta"], acc1, g0["theta"][acc0], g0["w"][acc0])
    np.testing.assert_allclose(g1["w"][acc1], w_ref, rtol=1e-9)
    assert g1["tol"] < g0["tol"]
    # the second generation concentrates on runs that complete
    assert np.isfinite(g1["dist"]).mean() > np.isfinite(d).mean()
