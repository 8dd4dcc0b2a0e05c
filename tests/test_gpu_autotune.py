"""The launch-shape autotuner: on an uneven batch (persistent-kernel buckets
and a large system) it returns valid shapes, keeps them in the context,
round-trips them through the tune file, and runs under them stay within
the parity bar of the oracle."""
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


def test_autotune_choices_and_tune_file(ctx, oracle_core, tmp_path):
    lay = inputs.dense_layout(n_samples=1, seed=9)[0]
    lay[:, 0] = 0.9
    lay[:, 7] -= 2.75
    lay[:, 8] -= 0.75
    small = inputs.param_rows(4, Sb=0.02, Ss=300.0, x0=-1.0)
    small[:, 0] = [0.0, 1.0, 3.0, 6.0]
    P = np.vstack([small, lay])
    N = np.array([64, 200, 320, 500, 80], np.int32)
    nsw = np.array([1, 1, 1, 1, 8], np.int32)
    Pd = torch.from_numpy(P).cuda()
    ch = swim.swim_autotune(ctx, swim.SWIM_F32, N, nsw, Pd, 20, 2e-6)
    # buckets present: tpl 1 (64 points), 4 (200), 6 (320), 8 (500); 640 is
    # large.  Five parts on four streams: the closest pair in size (6 and 8)
    # merges, so the 320-point system runs in the tpl-8 launch and tpl 6 is
    # never launched nor tuned
    for t in (1, 4, 8):
        assert ch["wps"][t] in (2, 4, 8, 16), (t, ch)
    assert ch["wps"][2] == 0 and ch["wps"][3] == 0 and ch["wps"][6] == 0, ch
    assert ch["big_tpl"] in (0, 1, 2, 4)
    assert swim.swim_get_option(ctx, swim.SWIM_OPT_BIG_TPL) == ch["big_tpl"]
    f = tmp_path / "tune.txt"
    swim.swim_tune_save(ctx, f)
    c2 = swim.Context(0)
    try:
        swim.swim_tune_load(c2, f)
        assert swim.swim_get_option(c2, swim.SWIM_OPT_BIG_TPL) == ch["big_tpl"]
        bad = tmp_path / "bad.txt"
        bad.write_text("not a tune file\n")
        with pytest.raises(swim.SwimError):
            swim.swim_tune_load(c2, bad)
    finally:
        c2.close()
    # a run under the tuned shapes against the oracle
    steps, dt, oe = 60, 2e-6, 20
    nfil = P.shape[0]
    obs = torch.empty((nfil, steps // oe, 2), dtype=torch.float32, device="cuda")
    speed = torch.empty(nfil, dtype=torch.float32, device="cuda")
    status = torch.empty(len(N), dtype=torch.int32, device="cuda")
    swim.swim_forward(ctx, N, nsw, Pd, steps, dt, oe, 1.5, obs, speed, status)
    torch.cuda.synchronize()
    o = obs.cpu().double().numpy()
    assert np.all(status.cpu().numpy() == 0)
    for i in range(4):
        ref = oracle_core.forward(P[i:i + 1], int(N[i]), steps, dt, oe)["obs"][0]
        x0 = np.array([0.0, 0.0])
        err = np.linalg.norm(o[i] - ref)
        allow = 1e-4 * np.linalg.norm(ref - x0) + np.linalg.norm(np.spacing(np.abs(ref).astype(np.float32)))
        assert err <= allow + 4 * np.finfo(np.float32).eps * np.sqrt(steps * ref.size), (i, err, allow)
