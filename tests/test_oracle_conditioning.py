"""Conditioning of the batched workload's forward run near forward Euler's
stability edge, in the oracle (FP64, the reading's closed-form blob for
speed; the step is the same forward Euler update, eq. BrV then the
Appendix's numerical algorithm).  A relative perturbation of the velocity
of 1e-7 per component and step (random, about two FP32 unit roundoffs)
moves the head series of a run near the edge (the batch's first completed
draw, dt rho close to 2) by more than 1e-4 of its displacement within 600
steps: an FP32 forward run there cannot be held to 1e-4 on the whole
series, whatever its arithmetic, because its velocity carries relative
errors of that size from FP32 inputs alone.  The same perturbation of a
well-damped run (S_b = 0.03) decays: there FP32 meets 1e-4."""
import numpy as np
import pytest

from oracle import core
from paper_1910_12007_amd import inputs

pytestmark = pytest.mark.usefixtures("reading_blob_module")

N, DT, OE, STEPS, ETA = 128, 5e-5, 100, 600, 1e-7


def _run(P, eta, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ds = 1.0 / (N - 1)
    x, y = P[7] + np.arange(N) * ds, np.full(N, P[8])
    obs = []
    for s in range(STEPS):
        fx, fy = core.forces(x, y, P[1], P[2], core.kappa0(N, P[3], P[5], P[4], P[6], s * DT))
        ux, uy = core.velocity(x, y, fx, fy, P[0], 1.5 * ds)
        if eta:
            ux = ux * (1 + eta * rng.normal(size=N))
            uy = uy * (1 + eta * rng.normal(size=N))
        x, y = x + DT * ux, y + DT * uy
        if (s + 1) % OE == 0:
            obs.append([x[-1], y[-1]])
    return np.array(obs)


@pytest.mark.parametrize("theta,lo,hi", [((1.60278217, 0.112909086, 1433.92411), 1e-4, 1e-1),
                                         ((4.0, 0.03, 2000.0), 0.0, 1e-6)])
def test_perturbation_growth(theta, lo, hi):
    P = inputs.theta_rows(np.array(theta))[0]
    ref = _run(P, 0.0, 0)
    r = core.forward(P[None], N, STEPS, DT, OE)
    assert r["status"] == 0 and np.array_equal(r["obs"][0], ref)  # the loop is the oracle's forward run
    x0 = np.array([1.0, 0.0])
    err = np.linalg.norm(_run(P, ETA, 1) - ref) / np.linalg.norm(ref - x0)
    print({"theta": theta, "series_error": err, "amplification": err / ETA})
    assert lo < err < hi
