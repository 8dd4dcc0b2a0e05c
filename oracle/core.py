"""ctypes wrappers around the oracle's C library (test infrastructure only).

Every function takes and returns numpy float64 arrays.  The C sources cite the
paper passages each step follows (Sec. 2.1 eq. BrV; Appendix eqs. EFB, curva,
EFT; forward Euler).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


class _blob:
    """Context manager selecting the blob of the oracle's kernel functions
    inside it, restoring the previous choice on exit."""

    value = None

    def __enter__(self):
        self._prev = lib().oracle_get_blob()
        lib().oracle_set_blob(self.value)
        return self

    def __exit__(self, *exc):
        lib().oracle_set_blob(self._prev)
        return False


class paper_blob(_blob):
    """The paper's blob 3 eps^3 / (2 pi R^5) (eq. eqnblob), the oracle's
    default: closed forms in the Stokes limit, quadrature for alpha > 0."""

    value = 1


class reading_blob(_blob):
    """The blob of the kernel reading (closed forms for every alpha; see
    swim_oracle.c)."""

    value = 0


def lib():
    """Load liboracle.so, building it with gcc if it is missing."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build
            build.build()
        L = ctypes.CDLL(path)
        L.oracle_bessel.argtypes = [ctypes.c_int64, _D, _D, _D, _D]
        L.oracle_kernel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D, _D, _D]
        L.oracle_velocity.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double,
                                      ctypes.c_double, _D, _D]
        L.oracle_velocity_at.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int64, _I64, _D, _D]
        L.oracle_energy.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_double,
                                    ctypes.c_double, _D]
        L.oracle_energy.restype = ctypes.c_double
        L.oracle_forces.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, ctypes.c_double,
                                    ctypes.c_double, _D, _D, _D]
        L.oracle_kappa0.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _D]
        L.oracle_forward.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _I32]
        L.oracle_forward.restype = ctypes.c_int
        L.oracle_sperm_zhat.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, _D]
        L.oracle_sperm_initial.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_sperm_energy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D,
                                          ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_sperm_energy.restype = ctypes.c_double
        L.oracle_sperm_forces.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D,
                                          ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.oracle_sperm_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, _D, _D, _D, _D, _I32]
        L.oracle_sperm_forward.restype = ctypes.c_int
        L.oracle_set_blob.argtypes = [ctypes.c_int]
        L.oracle_get_blob.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_blob.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D, _D, _D]
        L.oracle_field.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int64, _D, _D, _D, _D, _D]
        _LIB = L
    return _LIB


def num_threads():
    """Threads the oracle's parallel velocity sums use."""
    return int(lib().oracle_num_threads())


def set_threads(n):
    """Sets the threads of the oracle's parallel velocity sums."""
    lib().oracle_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def bessel(z):
    """K0(z), K1(z) and q(z) = z K1(z) - 1 (integral representation, A&S 9.6.24;
    ascending series A&S 9.6.11 for q at z <= 2)."""
    z = _f64(z).ravel()
    k0, k1, q = (np.empty_like(z) for _ in range(3))
    lib().oracle_bessel(z.size, _p(z), _p(k0), _p(k1), _p(q))
    return k0, k1, q


def kernel(alpha, eps, t):
    """H1(r), H2(r) of eq. (BrV) at squared distances t = r^2 (blob reading in
    swim_oracle.c)."""
    t = _f64(t)
    shape = t.shape
    t = t.ravel()
    H1, H2 = np.empty_like(t), np.empty_like(t)
    lib().oracle_kernel(float(alpha), float(eps), t.size, _p(t), _p(H1), _p(H2))
    return H1.reshape(shape), H2.reshape(shape)


def velocity(x, y, fx, fy, alpha, eps):
    """Dense sum of eq. (BrV) over all points of one system: u_i = sum_j
    [H1 F_j + H2 (F_j . x_ij) x_ij], x_ij = X_i - X_j, j ascending."""
    x, y, fx, fy = map(_f64, (x, y, fx, fy))
    ux, uy = np.empty_like(x), np.empty_like(x)
    lib().oracle_velocity(x.size, _p(x), _p(y), _p(fx), _p(fy), float(alpha), float(eps),
                          _p(ux), _p(uy))
    return ux, uy


def velocity_at(x, y, fx, fy, alpha, eps, idx):
    """Same sum as velocity(), at the targets idx only."""
    x, y, fx, fy = map(_f64, (x, y, fx, fy))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ux, uy = np.empty(idx.size), np.empty(idx.size)
    lib().oracle_velocity_at(x.size, _p(x), _p(y), _p(fx), _p(fy), float(alpha), float(eps),
                             idx.size, idx.ctypes.data_as(_I64), _p(ux), _p(uy))
    return ux, uy


def kappa0(N, b, k, omega, phase, t):
    """Preferred curvature -k^2 b sin(k s - omega t + phase) at s_i = i/(N-1)."""
    out = np.empty(N)
    lib().oracle_kappa0(N, 1.0 / (N - 1), float(b), float(k), float(omega), float(phase),
                        float(t), _p(out))
    return out


def energy(x, y, Sb, Ss, kap0):
    """Discrete E_tens + E_bend of one filament (Appendix EFT, EFB, curva)."""
    x, y, kap0 = map(_f64, (x, y, kap0))
    N = x.size
    return lib().oracle_energy(N, 1.0 / (N - 1), _p(x), _p(y), float(Sb), float(Ss), _p(kap0))


def forces(x, y, Sb, Ss, kap0):
    """F = -dE/dX of energy() (eq. Fenergy)."""
    x, y, kap0 = map(_f64, (x, y, kap0))
    N = x.size
    fx, fy = np.empty(N), np.empty(N)
    lib().oracle_forces(N, 1.0 / (N - 1), _p(x), _p(y), float(Sb), float(Ss), _p(kap0),
                        _p(fx), _p(fy))
    return fx, fy


PARAM_FIELDS = ("alpha", "Sb", "Ss", "b", "omega", "k", "phase", "x0", "y0")


def forward(params, N, steps, dt, obs_every, eps_over_ds=1.5):
    """Forward-Euler run of one system.

    params: array (n_swim, 9) with columns PARAM_FIELDS (alpha from row 0).
    Returns dict(obs=(n_swim, steps//obs_every, 2), speed=(n_swim,),
    x=(n_swim*N,), y=(n_swim*N,), status=int).
    """
    P = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n_swim = P.shape[0]
    n_obs = steps // obs_every if obs_every > 0 else 0
    obs = np.full((n_swim, max(n_obs, 1), 2), np.nan)
    speed = np.empty(n_swim)
    xo, yo = np.empty(n_swim * N), np.empty(n_swim * N)
    st = ctypes.c_int32(0)
    lib().oracle_forward(n_swim, N, _p(P), float(eps_over_ds), int(steps), float(dt),
                         int(obs_every), _p(obs), _p(speed), _p(xo), _p(yo), ctypes.byref(st))
    return dict(obs=obs[:, :n_obs], speed=speed, x=xo, y=yo, status=int(st.value))


# ---------------------------------------------------------------------------
# full sperm model (Appendix): system row SPERM_FIELDS, swimmer rows
# (x0, y0, phase); geometry (nf, nh, H_r, dN) shared by all swimmers
# ---------------------------------------------------------------------------
SPERM_FIELDS = ("alpha", "KC", "KT", "KHT", "KHC", "KNT", "KNA", "a", "eta", "omega")


def sperm_zhat(s, a, eta, omega, phase, t):
    """Preferred flagellum curvature: second s-derivative of the tapered beat
    a (1 - s) sin(eta s - omega t + phase)."""
    s = _f64(s).ravel()
    out = np.empty_like(s)
    lib().oracle_sperm_zhat(s.size, _p(s), float(a), float(eta), float(omega), float(phase), float(t), _p(out))
    return out


def sperm_initial(nf, nh, hr, dn, x0=0.0, y0=0.0):
    """Initial positions of one swimmer: flagellum points 0..nf-1, then the
    head points 0..nh-1 (angle m 2 pi / nh about the head centre)."""
    x, y = np.empty(nf + nh), np.empty(nf + nh)
    lib().oracle_sperm_initial(int(nf), int(nh), float(hr), float(dn), float(x0), float(y0), _p(x), _p(y))
    return x, y


def sperm_energy(nf, nh, hr, dn, sys_row, phase, t, x, y):
    """Discrete energy of one swimmer (swim_oracle.c lists its terms)."""
    sp = _f64(sys_row)
    x, y = _f64(x), _f64(y)
    return lib().oracle_sperm_energy(int(nf), int(nh), float(hr), float(dn), _p(sp), float(phase), float(t),
                                     _p(x), _p(y))


def sperm_forces(nf, nh, hr, dn, sys_row, phase, t, x, y):
    """F = -dE/dX of sperm_energy (eq. Fenergy)."""
    sp = _f64(sys_row)
    x, y = _f64(x), _f64(y)
    fx, fy = np.empty_like(x), np.empty_like(x)
    lib().oracle_sperm_forces(int(nf), int(nh), float(hr), float(dn), _p(sp), float(phase), float(t), _p(x),
                              _p(y), _p(fx), _p(fy))
    return fx, fy


def sperm_forward(sys_row, swimmers, nf, nh, eps, hr, dn, steps, dt, obs_every):
    """Forward-Euler run of one system of sperm swimmers.

    swimmers: (n_swim, 3) rows (x0, y0, phase).  Returns dict(head, tail)
    of shape (n_swim, n_obs + 1, 2) (sample 0: the initial state; NaN for
    samples a stopped run does not reach), x, y (final positions) and
    status."""
    sp = _f64(sys_row)
    sw = _f64(np.atleast_2d(swimmers))
    n_swim = sw.shape[0]
    n_obs = steps // obs_every if obs_every > 0 else 0
    head = np.full((n_swim, n_obs + 1, 2), np.nan)
    tail = np.full((n_swim, n_obs + 1, 2), np.nan)
    x, y = np.empty(n_swim * (nf + nh)), np.empty(n_swim * (nf + nh))
    st = ctypes.c_int32(0)
    lib().oracle_sperm_forward(n_swim, int(nf), int(nh), float(eps), float(hr), float(dn), _p(sp), _p(sw),
                               int(steps), float(dt), int(obs_every), _p(head), _p(tail), _p(x), _p(y),
                               ctypes.byref(st))
    return dict(head=head, tail=tail, x=x, y=y, status=int(st.value))


def sperm_head_velocity(head, dt_obs):
    """Sec. 4.1 observables: velocity of swimmer 0's head centre over each
    sampling interval, (h_k - h_{k-1}) / dt_obs for k = 1..n_obs; head as
    returned by sperm_forward.  (n_obs, 2)."""
    h = np.asarray(head, dtype=np.float64)[0]
    return (h[1:] - h[:-1]) / dt_obs


def sperm_pair_distances(head, tail):
    """Secs. 4.2-4.3 observables: at samples k = 1..n_obs, the distance
    between the tail ends and between the head centres of swimmers 0 and 1,
    in the order (tail, head).  (n_obs, 2)."""
    h = np.asarray(head, dtype=np.float64)
    t = np.asarray(tail, dtype=np.float64)
    dt_ = np.linalg.norm(t[0, 1:] - t[1, 1:], axis=-1)
    dh = np.linalg.norm(h[0, 1:] - h[1, 1:], axis=-1)
    return np.stack([dt_, dh], axis=-1)


def blob(alpha, eps, t):
    """The blob of the kernel reading, phi(r), and its mass inside r over r^2,
    m(r)/r^2 (m = 2 pi int_0^r s phi ds), at squared distances t."""
    t = _f64(t).ravel()
    phi, m = np.empty_like(t), np.empty_like(t)
    lib().oracle_blob(float(alpha), float(eps), t.size, _p(t), _p(phi), _p(m))
    return phi, m


def field(x, y, fx, fy, alpha, eps, tx, ty):
    """Velocity (eq. BrV) and pressure (eq. BrP, p = sum F . grad G_eps) at
    the target points (tx, ty) from the point forces of one system."""
    x, y, fx, fy, tx, ty = map(_f64, (x, y, fx, fy, tx, ty))
    u, v, p = np.empty(tx.size), np.empty(tx.size), np.empty(tx.size)
    lib().oracle_field(x.size, _p(x), _p(y), _p(fx), _p(fy), float(alpha), float(eps), tx.size, _p(tx), _p(ty),
                       _p(u), _p(v), _p(p))
    return u, v, p
