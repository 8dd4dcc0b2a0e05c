"""Seeded synthetic inputs for the workloads (numpy PCG64).

This module holds none of the method's arithmetic: it only draws parameter
sets, filament sizes, phases and test geometries.  Random numbers that the
ABC method itself draws (prior draws, PMC resampling and perturbation) are
not made here; they come from the Philox4x32-10 generator that the library
and the test oracle each implement.

Workloads (the forward model runs on a filament of length 1 with N points,
ds = 1/(N-1), blob width eps = 1.5 ds, initially straight along x):
  single   N=64, FP64, alpha in {1, 0}, S_b=0.1, S_s=1e3, b=0.1, k=omega=2 pi,
           dt=1e-4, 2000 steps.
  batch    4096 parameter sets, alpha~U[0,10], S_b~U[0.01,1], S_s~U[1e2,1e4],
           N=128, 5000 steps at dt=5e-5, head observed every 100 steps.
  uneven   16384 particles, N~U{64,96,...,512}, same priors, 3 PMC generations.
  dense    64 samples x 8 swimmers x N=512 on a 2x4 grid (spacing 1.5),
           phases~U[0,2pi), alpha~U[0,10].
  surrogate 65536 training runs (N=128) and 1M prescreened proposals.
  sperm    full sperm model (Appendix, Table Tab:param): N_F = 50, N_H = 24,
           eps = 0.045, K_tens = K_H,tens = K_N,ang = 1e4, K_N,tens = 500,
           K_H,C = 0.8, a = 0.1, eta = 2 pi, omega = 4 pi; (alpha, K_C) ~
           U[0,2] x U[0,16] (the paper's prior box); one swimmer, or two
           swimmers with head centres d apart vertically, same beat phase.
"""
import numpy as np

TWO_PI = 2.0 * np.pi

# default swimmer constants of the single-filament workload
DEFAULTS = dict(alpha=1.0, Sb=0.1, Ss=1e3, b=0.1, omega=TWO_PI, k=TWO_PI, phase=0.0, x0=0.0, y0=0.0)
PARAM_FIELDS = ("alpha", "Sb", "Ss", "b", "omega", "k", "phase", "x0", "y0")

# uniform prior box on (alpha, S_b, S_s)
PRIOR_LO = np.array([0.0, 0.01, 1e2])
PRIOR_HI = np.array([10.0, 1.0, 1e4])
TRUE_THETA = np.array([2.0, 0.1, 1e3])
# the batched workload's time grid: T = 0.25 in 10000 forward-Euler steps of
# 2.5e-5, the head every 200 steps (the synthetic data's 50 times).  Half the
# step of the workload as first stated (5000 of 5e-5): with the paper's blob
# the true parameters are beyond forward Euler's stability bound at 5e-5.
BATCH_STEPS, BATCH_DT, BATCH_OBS_EVERY = 10000, 2.5e-5, 200

UNEVEN_N_CHOICES = np.arange(64, 513, 32)


def param_rows(n, **overrides):
    """(n, 9) array of swimmer parameter rows (columns PARAM_FIELDS)."""
    P = np.empty((n, len(PARAM_FIELDS)))
    for i, f in enumerate(PARAM_FIELDS):
        P[:, i] = overrides.get(f, DEFAULTS[f])
    return P


def theta_rows(theta, **overrides):
    """Parameter rows from an (n, 3) array of (alpha, S_b, S_s)."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    P = param_rows(theta.shape[0], **overrides)
    P[:, 0:3] = theta
    return P


def uneven_sizes(n, seed=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(UNEVEN_N_CHOICES, size=n).astype(np.int32)


def dense_layout(n_samples=64, seed=3, n_cols=4, n_rows=2, spacing=1.5):
    """Swimmer rows for the multi-swimmer workload: (n_samples, 8, 9)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    alpha = rng.uniform(0.0, 10.0, size=n_samples)
    phase = rng.uniform(0.0, TWO_PI, size=(n_samples, n_cols * n_rows))
    P = np.empty((n_samples, n_cols * n_rows, len(PARAM_FIELDS)))
    for s in range(n_samples):
        rows = param_rows(n_cols * n_rows, alpha=alpha[s])
        m = 0
        for r in range(n_rows):
            for c in range(n_cols):
                rows[m, 6] = phase[s, m]
                rows[m, 7] = spacing * c
                rows[m, 8] = spacing * r
                m += 1
        P[s] = rows
    return P


def filament_geometry(N, seed, n_swim=1, amp=0.08, spacing=1.5, jitter=1e-3):
    """Bent filaments of length ~1 (a travelling-wave shape plus jitter) for
    single-evaluation tests.  Returns x, y of shape (n_swim*N,)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.linspace(0.0, 1.0, N)
    xs, ys = [], []
    for m in range(n_swim):
        ph = rng.uniform(0.0, TWO_PI)
        x = s + jitter * rng.standard_normal(N) / N
        y = amp * np.sin(TWO_PI * s + ph) + jitter * rng.standard_normal(N) / N
        xs.append(x + spacing * (m % 4))
        ys.append(y + spacing * (m // 4))
    return np.concatenate(xs), np.concatenate(ys)


def force_pattern(N, seed, n_swim=1, tension=50.0, smooth=5.0):
    """Point forces shaped like a filament's: a large alternating tension part
    T_k - T_{k-1} along x plus a smooth part, with zero sum per filament."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fxs, fys = [], []
    for _ in range(n_swim):
        T = tension * rng.standard_normal(N + 1)
        T[0] = T[-1] = 0.0
        fx = T[1:] - T[:-1] + smooth * rng.standard_normal(N)
        fy = smooth * np.sin(np.linspace(0, 3 * np.pi, N)) * rng.uniform(0.5, 1.5) + \
            0.2 * smooth * rng.standard_normal(N)
        fx -= fx.mean()
        fy -= fy.mean()
        fxs.append(fx)
        fys.append(fy)
    return np.concatenate(fxs), np.concatenate(fys)


def surrogate_inputs(n, seed):
    """(alpha, log S_b, log S_s, b, omega) rows drawn from the prior box with b
    and omega at their defaults."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(PRIOR_LO[0], PRIOR_HI[0], n)
    sb = rng.uniform(PRIOR_LO[1], PRIOR_HI[1], n)
    ss = rng.uniform(PRIOR_LO[2], PRIOR_HI[2], n)
    return np.stack([a, sb, ss], axis=1)


def observation_noise(n_obs, sigma=1e-3, seed=20191027):
    rng = np.random.Generator(np.random.PCG64(seed))
    return sigma * rng.standard_normal((n_obs, 2))


MLP_LAYERS = (5, 256, 256, 256, 256, 33)


def mlp_init(seed=0, layers=MLP_LAYERS):
    """He-uniform initial weights (U(+-sqrt(6/fan_in))) and zero biases, as a
    list of (W, b) and as the flat FP32 vector of the library's layout
    (per layer: W row-major fan_in x fan_out, then b)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for a, b in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / a)
        params.append((rng.uniform(-lim, lim, (a, b)).astype(np.float32).astype(np.float64), np.zeros(b)))
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)
    return params, flat


def unflatten(flat, layers=MLP_LAYERS):
    out, o = [], 0
    for a, b in zip(layers[:-1], layers[1:]):
        W = np.asarray(flat[o:o + a * b], dtype=np.float64).reshape(a, b)
        o += a * b
        bb = np.asarray(flat[o:o + b], dtype=np.float64)
        o += b
        out.append((W, bb))
    return out


def epoch_permutations(n, epochs, seed=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


# full sperm model: Table Tab:param constants (system row order SPERM_FIELDS)
SPERM_FIELDS = ("alpha", "KC", "KT", "KHT", "KHC", "KNT", "KNA", "a", "eta", "omega")
SPERM_TABLE = dict(alpha=1.0, KC=8.0, KT=1e4, KHT=1e4, KHC=0.8, KNT=500.0, KNA=1e4, a=0.1, eta=TWO_PI,
                   omega=2.0 * TWO_PI)
SPERM_PRIOR_LO = np.array([0.0, 0.0])   # (alpha, K_C)
SPERM_PRIOR_HI = np.array([2.0, 16.0])


def sperm_rows(n, seed=None, **overrides):
    """(n, 10) system rows: Table values, (alpha, K_C) drawn from the prior box
    when seed is given, then the overrides."""
    P = np.empty((n, len(SPERM_FIELDS)))
    for i, f in enumerate(SPERM_FIELDS):
        P[:, i] = SPERM_TABLE[f]
    if seed is not None:
        rng = np.random.Generator(np.random.PCG64(seed))
        P[:, 0] = rng.uniform(SPERM_PRIOR_LO[0], SPERM_PRIOR_HI[0], n)
        P[:, 1] = rng.uniform(SPERM_PRIOR_LO[1], SPERM_PRIOR_HI[1], n)
    for f, v in overrides.items():
        P[:, SPERM_FIELDS.index(f)] = v
    return P


def sperm_swimmers(n_sys, n_swim=1, d=0.5, phases=None):
    """(n_sys * n_swim, 3) swimmer rows (x0, y0, phase): swimmers of one
    system stacked vertically d apart (centred on y = 0), all starting at
    x0 = 0; phases per swimmer (default 0)."""
    W = np.zeros((n_sys, n_swim, 3))
    W[:, :, 1] = (np.arange(n_swim) - 0.5 * (n_swim - 1)) * d
    if phases is not None:
        W[:, :, 2] = np.asarray(phases)
    return W.reshape(-1, 3)
