"""Thin ctypes binding of libswim (include/swim.h).

Functions carry the C names and only marshal arguments: device arrays are
torch tensors on the HIP device (their data pointers are passed), host arrays
are numpy arrays.  Every computation happens inside libswim.so; there is no
Python or CPU fallback -- if the library is missing, loading raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswim.so")

SWIM_OK, SWIM_EINVAL, SWIM_EHIP, SWIM_ENOMEM, SWIM_ESTATE = 0, -1, -2, -3, -4
SWIM_F32, SWIM_F64 = 0, 1
SWIM_ST_OK, SWIM_ST_NONFINITE, SWIM_ST_BOUND, SWIM_ST_BADPARAM, SWIM_ST_REJECTED = 0, 1, 2, 3, 4
SWIM_NPARAM = 9
SWIM_OPT_WPS, SWIM_OPT_BIG_TPL, SWIM_OPT_GRAPH, SWIM_OPT_GRAPH_LAUNCHES, SWIM_OPT_GRAPH_CAPTURES = 1, 2, 3, 4, 5
SWIM_OPT_BLOB, SWIM_BLOB_READING, SWIM_BLOB_PAPER = 6, 0, 1
SWIM_OPT_EARLY_STOP, SWIM_OPT_TIME_KERNEL, SWIM_OPT_KERNEL_US = 7, 8, 9
SWIM_MLP_NPARAM, SWIM_MLP_IN, SWIM_MLP_OUT = 207393, 5, 33
# full sperm model: system row fields (SWIM_SP_*) and swimmer row width
SPERM_FIELDS = ("alpha", "KC", "KT", "KHT", "KHC", "KNT", "KNA", "a", "eta", "omega")
SWIM_SP_NPARAM, SWIM_SW_NPARAM = 10, 3
SWIM_OBS_HEAD_VELOCITY, SWIM_OBS_PAIR_DISTANCES = 0, 1

_c = ctypes
_P = _c.c_void_p
_I64P = _c.POINTER(_c.c_int64)
_I32P = _c.POINTER(_c.c_int32)
_DP = _c.POINTER(_c.c_double)
_U8P = _c.POINTER(_c.c_uint8)

# name -> (restype, argtypes); mirrors include/swim.h
SIGNATURES = {
    "swim_create": (_c.c_int, [_c.POINTER(_P), _c.c_int]),
    "swim_destroy": (None, [_P]),
    "swim_last_error": (_c.c_char_p, []),
    "swim_version": (_c.c_int, []),
    "swim_set_option": (_c.c_int, [_P, _c.c_int32, _c.c_int32]),
    "swim_get_option": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int32)]),
    "swim_autotune": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _I32P, _I32P, _P, _c.c_int32, _c.c_double, _c.c_double,
                                 _I32P]),
    "swim_tune_save": (_c.c_int, [_P, _c.c_char_p]),
    "swim_tune_load": (_c.c_int, [_P, _c.c_char_p]),
    "swim_pair_velocity": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _I64P, _DP, _DP, _P, _P, _P, _P, _P, _P, _P]),
    "swim_pair_velocity_noalloc": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _I64P, _DP, _DP, _P, _P, _P, _P, _P, _P,
                                              _P]),
    "swim_elastic_forces": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _I32P, _DP, _c.c_double, _P, _P, _P, _P, _P]),
    "swim_forward": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _I32P, _I32P, _P, _c.c_int32, _c.c_double,
                                _c.c_int32, _c.c_double, _P, _P, _P, _P, _P]),
    "swim_sperm_forward": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _P, _P, _P, _c.c_int32, _c.c_double, _c.c_int32,
                                      _P, _P, _P, _P]),
    "swim_sperm_observables": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_int64, _c.c_int32, _c.c_int32,
                                          _c.c_double, _P, _P, _P, _P, _P]),
    "tmcmc_loglik2": (_c.c_int, [_P, _c.c_int64, _c.c_int32, _P, _P, _P, _P, _P, _P]),
    "tmcmc_sperm_run": (_c.c_int, [_P, _P, _DP, _P, _DP, _c.c_int32, _c.c_int64, _c.c_uint64, _DP, _DP, _DP, _I32P,
                                   _DP, _I64P, _I64P, _DP]),
    "swim_flow_field": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _P, _P, _P, _P, _c.c_double, _c.c_double, _c.c_int64,
                                   _P, _P, _P, _P, _P, _P]),
    "abc_distance": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _c.c_int32, _P, _P, _P, _P, _P]),
    "abc_select": (_c.c_int, [_P, _c.c_int64, _P, _c.c_double, _P, _P, _P]),
    "abc_prior_draw": (_c.c_int, [_c.c_uint64, _c.c_int64, _c.c_int32, _DP, _DP, _DP]),
    "abc_pmc_propose": (_c.c_int, [_c.c_uint64, _c.c_int32, _c.c_int64, _DP, _DP, _c.c_int64, _DP, _DP, _DP]),
    "abc_pmc_weights": (_c.c_int, [_c.c_int64, _DP, _U8P, _DP, _DP, _c.c_int64, _DP]),
    "abc_step": (_c.c_int, [_P, _P, _DP, _c.c_int32, _c.c_int64, _I32P, _c.c_uint64, _c.c_int32, _DP, _DP,
                            _c.c_int64, _c.c_double, _DP, _DP, _U8P, _DP, _DP, _I32P]),
    "swim_kernel_eval_host": (_c.c_int, [_c.c_int32, _c.c_double, _c.c_double, _c.c_int32, _c.c_int64, _DP, _DP, _DP,
                                         _DP]),
    "swim_forward_plan": (_c.c_int, [_c.c_int32, _c.c_int64, _I32P, _I32P, _c.c_double, _I32P]),
    "tmcmc_loglik": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _c.c_int32, _P, _P, _P, _P, _P, _P]),
    "tmcmc_run": (_c.c_int, [_P, _P, _P, _DP, _c.c_int32, _c.c_int32, _c.c_int64, _c.c_uint64, _DP, _DP, _DP, _I32P,
                             _DP, _I64P, _I64P, _DP]),
    "surrogate_forward": (_c.c_int, [_P, _c.c_int64, _P, _P, _P, _P]),
    "surrogate_grad": (_c.c_int, [_P, _c.c_int64, _P, _P, _P, _P, _P, _P]),
    "surrogate_train": (_c.c_int, [_P, _c.c_int64, _P, _P, _P, _c.c_int32, _c.c_int32, _c.c_float, _P, _P, _P, _P,
                                   _P]),
    "surrogate_prescreen": (_c.c_int, [_P, _c.c_int64, _P, _P, _P, _P, _P, _c.c_int32, _c.c_float, _P, _P, _P, _P,
                                       _P]),
    "surrogate_features": (_c.c_int, [_P, _c.c_int64, _P, _c.c_double, _c.c_double, _P, _P, _P, _P]),
    "surrogate_targets": (_c.c_int, [_P, _c.c_int32, _c.c_int64, _c.c_int32, _P, _P, _c.c_double, _c.c_double, _I32P,
                                     _c.c_int32, _P, _P]),
    "surrogate_colstats": (_c.c_int, [_P, _c.c_int64, _c.c_int32, _P, _P, _P, _P]),
    "surrogate_standardize": (_c.c_int, [_P, _c.c_int64, _c.c_int32, _P, _P, _P, _P]),
    "abc_prior_draw_device": (_c.c_int, [_P, _c.c_uint64, _c.c_int64, _DP, _DP, _P, _P]),
    "swim_param_rows": (_c.c_int, [_P, _c.c_int64, _P, _P, _c.c_int64, _P, _c.c_double, _c.c_double, _c.c_double, _P,
                                   _P]),
    "swim_select": (_c.c_int, [_P, _c.c_int64, _P, _c.c_int32, _P, _P, _P, _P]),
    "swim_gather_rows": (_c.c_int, [_P, _c.c_int64, _P, _P, _c.c_int64, _P, _c.c_int32, _P, _P]),
    "surrogate_dataset": (_c.c_int, [_P, _P, _c.c_int32, _c.c_int64, _c.c_uint64, _I32P, _c.c_int32, _c.c_double,
                                     _c.c_int64, _P, _P, _P, _P, _P, _P, _I64P, _P]),
    "abc_prescreened": (_c.c_int, [_P, _P, _c.c_int32, _P, _P, _P, _P, _P, _I32P, _c.c_int32, _DP, _c.c_int32,
                                   _c.c_double, _c.c_double, _c.c_int64, _c.c_uint64, _c.c_int64, _DP, _DP, _U8P,
                                   _I64P, _c.POINTER(_c.c_float)]),
}

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libswim.so not built ({LIB_PATH}); run `python -m paper_1910_12007_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


class SwimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libswim error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != SWIM_OK:
        raise SwimError(rc, lib().swim_last_error().decode())
    return rc


class abc_model(ctypes.Structure):
    _fields_ = [("lo", _c.c_double * 3), ("hi", _c.c_double * 3), ("b", _c.c_double), ("omega", _c.c_double),
                ("k", _c.c_double), ("steps", _c.c_int32), ("obs_every", _c.c_int32), ("dt", _c.c_double),
                ("eps_over_ds", _c.c_double), ("dtype", _c.c_int32), ("use_graph", _c.c_int32)]


class tmcmc_opts(ctypes.Structure):
    _fields_ = [("lo", _c.c_double * 4), ("hi", _c.c_double * 4), ("cv_target", _c.c_double),
                ("cov_scale", _c.c_double), ("max_stages", _c.c_int32)]


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return _P(t.data_ptr())


def _stream(s):
    if s is None:
        return None
    return _P(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))


def _h(a, dtype, ptr):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ptr)


def dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return SWIM_F32
    if t.dtype == torch.float64:
        return SWIM_F64
    raise ValueError("dtype must be float32 or float64")


class Context:
    """Owns one swim_ctx."""

    def __init__(self, device=0):
        h = _P()
        _check(lib().swim_create(ctypes.byref(h), int(device)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().swim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def swim_set_option(ctx, key, value):
    return _check(lib().swim_set_option(ctx.handle, int(key), int(value)))


def swim_get_option(ctx, key):
    v = ctypes.c_int32()
    _check(lib().swim_get_option(ctx.handle, int(key), ctypes.byref(v)))
    return v.value


def swim_autotune(ctx, dtype, N, n_swim, params, probe_steps, dt, eps_over_ds=1.5):
    """Returns the chosen shapes: waves per system for tpl 1..8 (0: not
    tuned) and the large-system targets per lane."""
    n, n_p = _h(N, np.int32, _I32P)
    ns, ns_p = (None, None) if n_swim is None else _h(n_swim, np.int32, _I32P)
    out = np.zeros(9, dtype=np.int32)
    _check(lib().swim_autotune(ctx.handle, int(dtype), len(n), n_p, ns_p, _dptr(params), int(probe_steps), float(dt),
                               float(eps_over_ds), out.ctypes.data_as(_I32P)))
    return dict(wps={t: int(out[t - 1]) for t in (1, 2, 3, 4, 6, 8)}, big_tpl=int(out[8]))


def swim_tune_save(ctx, path):
    return _check(lib().swim_tune_save(ctx.handle, str(path).encode()))


def swim_tune_load(ctx, path):
    return _check(lib().swim_tune_load(ctx.handle, str(path).encode()))


def swim_pair_velocity(ctx, sys_off, alpha, eps, x, y, fx, fy, ux, uy, stream=None):
    so, so_p = _h(sys_off, np.int64, _I64P)
    a, a_p = _h(alpha, np.float64, _DP)
    e, e_p = _h(eps, np.float64, _DP)
    return _check(lib().swim_pair_velocity(ctx.handle, dtype_code(x), len(a), so_p, a_p, e_p, _dptr(x), _dptr(y),
                                           _dptr(fx), _dptr(fy), _dptr(ux), _dptr(uy), _stream(stream)))


def swim_pair_velocity_noalloc(ctx, sys_off, alpha, eps, x, y, fx, fy, ux, uy, stream=None):
    so, so_p = _h(sys_off, np.int64, _I64P)
    a, a_p = _h(alpha, np.float64, _DP)
    e, e_p = _h(eps, np.float64, _DP)
    return _check(lib().swim_pair_velocity_noalloc(ctx.handle, dtype_code(x), len(a), so_p, a_p, e_p, _dptr(x),
                                                   _dptr(y), _dptr(fx), _dptr(fy), _dptr(ux), _dptr(uy),
                                                   _stream(stream)))


def swim_elastic_forces(ctx, N, params, t, x, y, fx, fy, stream=None):
    n, n_p = _h(N, np.int32, _I32P)
    P, P_p = _h(params, np.float64, _DP)
    return _check(lib().swim_elastic_forces(ctx.handle, dtype_code(x), len(n), n_p, P_p, float(t), _dptr(x),
                                            _dptr(y), _dptr(fx), _dptr(fy), _stream(stream)))


def swim_forward(ctx, N, n_swim, params, steps, dt, obs_every, eps_over_ds, obs, speed, status, steps_done=None,
                 stream=None):
    n, n_p = _h(N, np.int32, _I32P)
    if n_swim is None:
        ns_p = None
    else:
        ns, ns_p = _h(n_swim, np.int32, _I32P)
    return _check(lib().swim_forward(ctx.handle, dtype_code(speed), len(n), n_p, ns_p, _dptr(params), int(steps),
                                     float(dt), int(obs_every), float(eps_over_ds), _dptr(obs), _dptr(speed),
                                     _dptr(status), _dptr(steps_done), _stream(stream)))


def abc_distance(ctx, obs, data, status, dist, stream=None):
    n, n_obs = obs.shape[0], obs.shape[1]
    return _check(lib().abc_distance(ctx.handle, dtype_code(obs), n, n_obs, _dptr(obs), _dptr(data),
                                     _dptr(status), _dptr(dist), _stream(stream)))


def abc_select(ctx, dist, q, tol, accept=None, stream=None):
    return _check(lib().abc_select(ctx.handle, dist.numel(), _dptr(dist), float(q), _dptr(tol), _dptr(accept),
                                   _stream(stream)))


def abc_prior_draw(seed, n, lo, hi):
    lo_, lo_p = _h(lo, np.float64, _DP)
    hi_, hi_p = _h(hi, np.float64, _DP)
    out = np.empty((n, len(lo_)))
    _check(lib().abc_prior_draw(int(seed), int(n), len(lo_), lo_p, hi_p, out.ctypes.data_as(_DP)))
    return out


def abc_pmc_propose(seed, generation, n, prev_theta, prev_w, lo, hi):
    pt, pt_p = _h(prev_theta, np.float64, _DP)
    pw, pw_p = _h(prev_w, np.float64, _DP)
    lo_, lo_p = _h(lo, np.float64, _DP)
    hi_, hi_p = _h(hi, np.float64, _DP)
    out = np.empty((n, 3))
    _check(lib().abc_pmc_propose(int(seed), int(generation), int(n), pt_p, pw_p, pt.shape[0], lo_p, hi_p,
                                 out.ctypes.data_as(_DP)))
    return out


def abc_pmc_weights(theta, accept, prev_theta, prev_w):
    th, th_p = _h(theta, np.float64, _DP)
    ac, ac_p = _h(accept, np.uint8, _U8P)
    pt, pt_p = _h(prev_theta, np.float64, _DP)
    pw, pw_p = _h(prev_w, np.float64, _DP)
    w = np.empty(th.shape[0])
    _check(lib().abc_pmc_weights(th.shape[0], th_p, ac_p, pt_p, pw_p, pt.shape[0], w.ctypes.data_as(_DP)))
    return w


def abc_step(ctx, model, data, N, seed, generation, q, prev_theta=None, prev_w=None):
    d, d_p = _h(data, np.float64, _DP)
    n_, n_p = _h(N, np.int32, _I32P)
    n = len(n_)
    if prev_theta is None:
        pt_p = pw_p = None
        n_prev = 0
    else:
        pt, pt_p = _h(prev_theta, np.float64, _DP)
        pw, pw_p = _h(prev_w, np.float64, _DP)
        n_prev = pt.shape[0]
    theta = np.empty((n, 3))
    dist = np.empty(n)
    acc = np.empty(n, dtype=np.uint8)
    w = np.empty(n)
    tol = np.empty(1)
    steps = np.empty(n, dtype=np.int32)
    _check(lib().abc_step(ctx.handle, ctypes.byref(model), d_p, d.shape[0], n, n_p, int(seed), int(generation),
                          pt_p, pw_p, n_prev, float(q), theta.ctypes.data_as(_DP), dist.ctypes.data_as(_DP),
                          acc.ctypes.data_as(_U8P), w.ctypes.data_as(_DP), tol.ctypes.data_as(_DP),
                          steps.ctypes.data_as(_I32P)))
    return dict(theta=theta, dist=dist, accept=acc.astype(bool), w=w, tol=float(tol[0]), steps=steps)


def tmcmc_loglik(ctx, dtype, obs, data, sigma, status, logl, stream=None):
    """Device tensors: obs [n][n_obs][2] (run dtype), data [n_obs][2] FP64,
    sigma [n] FP64, status [n] int32 -> logl [n] FP64."""
    n, n_obs = obs.shape[0], obs.shape[1]
    _check(lib().tmcmc_loglik(ctx.handle, int(dtype), n, n_obs, _dptr(obs), _dptr(data), _dptr(sigma), _dptr(status),
                              _dptr(logl), _stream(stream)))


def tmcmc_run(ctx, model, lo, hi, data, N, n, seed, cv_target=1.0, cov_scale=0.2, max_stages=40):
    """One TMCMC run over the forward model; host arrays in and out."""
    d, d_p = _h(data, np.float64, _DP)
    o = tmcmc_opts()
    for i in range(4):
        o.lo[i] = float(lo[i])
        o.hi[i] = float(hi[i])
    o.cv_target, o.cov_scale, o.max_stages = float(cv_target), float(cov_scale), int(max_stages)
    theta = np.empty((n, 4))
    logl = np.empty(n)
    q = np.full(max_stages + 1, np.nan)
    ns = np.zeros(1, dtype=np.int32)
    lev = np.empty(1)
    acc = np.zeros(max_stages, dtype=np.int64)
    runs = np.zeros(1, dtype=np.int64)
    secs = np.zeros(1)
    _check(lib().tmcmc_run(ctx.handle, ctypes.byref(model), ctypes.byref(o), d_p, d.shape[0], int(N), int(n), int(seed),
                           theta.ctypes.data_as(_DP), logl.ctypes.data_as(_DP), q.ctypes.data_as(_DP),
                           ns.ctypes.data_as(_I32P), lev.ctypes.data_as(_DP), acc.ctypes.data_as(_I64P),
                           runs.ctypes.data_as(_I64P), secs.ctypes.data_as(_DP)))
    k = int(ns[0])
    return dict(theta=theta, logl=logl, q=q[:k + 1], n_stages=k, log_evidence=float(lev[0]), accepted=acc[:k],
                runs=int(runs[0]), seconds=float(secs[0]))


def swim_forward_plan(dtype, N, n_swim=None, eps_over_ds=1.5):
    """Targets per lane of the launch each system runs in (-1: the
    large-system step); host only."""
    n_, n_p = _h(N, np.int32, _I32P)
    s_p = None
    if n_swim is not None:
        s_, s_p = _h(n_swim, np.int32, _I32P)
    out = np.empty(n_.size, dtype=np.int32)
    _check(lib().swim_forward_plan(int(dtype), n_.size, n_p, s_p, float(eps_over_ds), out.ctypes.data_as(_I32P)))
    return out


def swim_kernel_eval_host(dtype, alpha, eps, t, blob=SWIM_BLOB_PAPER):
    t_, t_p = _h(t, np.float64, _DP)
    h1t, h2 = np.empty_like(t_), np.empty_like(t_)
    h1c = ctypes.c_double()
    _check(lib().swim_kernel_eval_host(int(dtype), float(alpha), float(eps), int(blob), t_.size, t_p,
                                       h1t.ctypes.data_as(_DP), h2.ctypes.data_as(_DP), ctypes.byref(h1c)))
    return h1t, h2, h1c.value


# --------------------------------------------------------------------------
# surrogate (device tensors unless noted)
# --------------------------------------------------------------------------
def surrogate_forward(ctx, X, params, Y, stream=None):
    return _check(lib().surrogate_forward(ctx.handle, X.shape[0], _dptr(X), _dptr(params), _dptr(Y), _stream(stream)))


def surrogate_grad(ctx, X, T, params, grads, loss=None, stream=None):
    return _check(lib().surrogate_grad(ctx.handle, X.shape[0], _dptr(X), _dptr(T), _dptr(params), _dptr(grads),
                                       _dptr(loss), _stream(stream)))


def surrogate_train(ctx, X, T, perm, epochs, batch, lr, params, adam_m, adam_v, loss_out=None, stream=None):
    return _check(lib().surrogate_train(ctx.handle, X.shape[0], _dptr(X), _dptr(T), _dptr(perm), int(epochs),
                                        int(batch), float(lr), _dptr(params), _dptr(adam_m), _dptr(adam_v),
                                        _dptr(loss_out), _stream(stream)))


def surrogate_prescreen(ctx, X, params, out_mu, out_sd, obs_sum, n_sum, tol, keep, idx, n_keep, dist=None,
                        stream=None):
    return _check(lib().surrogate_prescreen(ctx.handle, X.shape[0], _dptr(X), _dptr(params), _dptr(out_mu),
                                            _dptr(out_sd), _dptr(obs_sum), int(n_sum), float(tol), _dptr(dist),
                                            _dptr(keep), _dptr(idx), _dptr(n_keep), _stream(stream)))


def surrogate_features(ctx, theta, b, omega, X, mu=None, sd=None, stream=None):
    return _check(lib().surrogate_features(ctx.handle, theta.shape[0], _dptr(theta), float(b), float(omega),
                                           _dptr(mu), _dptr(sd), _dptr(X), _stream(stream)))


def surrogate_targets(ctx, obs, speed, x0, y0, sum_idx, T, stream=None):
    si, si_p = _h(sum_idx, np.int32, _I32P)
    return _check(lib().surrogate_targets(ctx.handle, dtype_code(obs), obs.shape[0], obs.shape[1], _dptr(obs),
                                          _dptr(speed), float(x0), float(y0), si_p, len(si), _dptr(T),
                                          _stream(stream)))


def surrogate_colstats(ctx, A, mu, sd, stream=None):
    return _check(lib().surrogate_colstats(ctx.handle, A.shape[0], A.shape[1], _dptr(A), _dptr(mu), _dptr(sd),
                                           _stream(stream)))


def surrogate_standardize(ctx, A, mu, sd, stream=None):
    return _check(lib().surrogate_standardize(ctx.handle, A.shape[0], A.shape[1], _dptr(A), _dptr(mu), _dptr(sd),
                                              _stream(stream)))


def abc_prior_draw_device(ctx, seed, lo, hi, theta, stream=None):
    lo_, lo_p = _h(lo, np.float64, _DP)
    hi_, hi_p = _h(hi, np.float64, _DP)
    return _check(lib().abc_prior_draw_device(ctx.handle, int(seed), theta.shape[0], lo_p, hi_p, _dptr(theta),
                                              _stream(stream)))


def swim_param_rows(ctx, theta, b, omega, k, rows, idx=None, n_dev=None, cap=None, stream=None):
    cap = rows.shape[0] if cap is None else cap
    return _check(lib().swim_param_rows(ctx.handle, int(cap), _dptr(n_dev), _dptr(idx), theta.shape[0], _dptr(theta),
                                        float(b), float(omega), float(k), _dptr(rows), _stream(stream)))


def swim_select(ctx, keep, idx, n_keep, values=None, want=0, stream=None):
    return _check(lib().swim_select(ctx.handle, keep.numel(), _dptr(values), int(want), _dptr(keep), _dptr(idx),
                                    _dptr(n_keep), _stream(stream)))


def swim_gather_rows(ctx, idx, n_dev, src, dst, cap=None, stream=None):
    cap = dst.shape[0] if cap is None else cap
    return _check(lib().swim_gather_rows(ctx.handle, int(cap), _dptr(n_dev), _dptr(idx), src.shape[0], _dptr(src),
                                         src.shape[1], _dptr(dst), _stream(stream)))


def surrogate_dataset(ctx, model, N, n_runs, seed, sum_idx, max_disp, X, T, in_mu, in_sd, out_mu, out_sd,
                      stream=None):
    """Returns the number of rows written (kept runs, at most X.shape[0])."""
    si, si_p = _h(sum_idx, np.int32, _I32P)
    n_out = ctypes.c_int64()
    _check(lib().surrogate_dataset(ctx.handle, ctypes.byref(model), int(N), int(n_runs), int(seed), si_p, len(si),
                                   float(max_disp), X.shape[0], _dptr(X), _dptr(T), _dptr(in_mu), _dptr(in_sd), _dptr(out_mu),
                                   _dptr(out_sd), ctypes.byref(n_out), _stream(stream)))
    return n_out.value


def abc_prescreened(ctx, model, N, params, in_mu, in_sd, out_mu, out_sd, sum_idx, data, tol, factor, n_prop,
                    seed, cap):
    si, si_p = _h(sum_idx, np.int32, _I32P)
    d, d_p = _h(data, np.float64, _DP)
    theta = np.empty((cap, 3))
    dist = np.empty(cap)
    acc = np.empty(cap, dtype=np.uint8)
    n_surv = ctypes.c_int64()
    ms = (ctypes.c_float * 2)()
    _check(lib().abc_prescreened(ctx.handle, ctypes.byref(model), int(N), _dptr(params), _dptr(in_mu), _dptr(in_sd),
                                 _dptr(out_mu), _dptr(out_sd), si_p, len(si), d_p, d.shape[0], float(tol),
                                 float(factor), int(n_prop), int(seed), int(cap), theta.ctypes.data_as(_DP),
                                 dist.ctypes.data_as(_DP), acc.ctypes.data_as(_U8P), ctypes.byref(n_surv), ms))
    n = min(n_surv.value, cap)
    return dict(n_surv=n_surv.value, theta=theta[:n], dist=dist[:n], accept=acc[:n].astype(bool),
                ms_prescreen=float(ms[0]), ms_rerun=float(ms[1]))


class swim_sperm_shape(ctypes.Structure):
    _fields_ = [("n_flag", ctypes.c_int32), ("n_head", ctypes.c_int32), ("n_swim", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eps", ctypes.c_double), ("head_radius", ctypes.c_double),
                ("neck_gap", ctypes.c_double)]


def sperm_shape(n_flag=50, n_head=24, n_swim=1, eps=0.045, head_radius=0.05, neck_gap=None):
    """Shape of the full sperm model (defaults: Table Tab:param sizes and
    blob; head radius 0.05 and neck gap ds, which the paper does not state)."""
    return swim_sperm_shape(int(n_flag), int(n_head), int(n_swim), 0, float(eps), float(head_radius),
                            float(1.0 / (n_flag - 1) if neck_gap is None else neck_gap))


def swim_sperm_forward(ctx, dtype, shape, sys_params, swim_params, steps, dt, obs_every, head, tail, status,
                       stream=None):
    """sys_params device float64 (n_sys, 10); swim_params device float64
    (n_sys * n_swim, 3); head, tail device tensors (n_sys * n_swim,
    n_obs + 1, 2) of the run's dtype; status device int32 (n_sys,)."""
    n_sys = status.numel()
    return _check(lib().swim_sperm_forward(ctx.handle, int(dtype), n_sys, ctypes.byref(shape), _dptr(sys_params),
                                           _dptr(swim_params), int(steps), float(dt), int(obs_every), _dptr(head),
                                           _dptr(tail), _dptr(status), _stream(stream)))


def swim_sperm_observables(ctx, dtype, kind, n_swim, dt_obs, head, tail, status, g, stream=None):
    """g device float64 (n_sys, n_obs, 2) from head/tail (n_sys * n_swim,
    n_obs + 1, 2)."""
    n_sys, n_obs = g.shape[0], g.shape[1]
    return _check(lib().swim_sperm_observables(ctx.handle, int(dtype), int(kind), n_sys, int(n_swim), n_obs,
                                               float(dt_obs), _dptr(head), _dptr(tail), _dptr(status), _dptr(g),
                                               _stream(stream)))


def tmcmc_loglik2(ctx, g, data, sigma2, status, logl, stream=None):
    """g device float64 (n, n_obs, 2); data (n_obs, 2); sigma2 (n, 2);
    status int32 (n,) or None; logl float64 (n,)."""
    return _check(lib().tmcmc_loglik2(ctx.handle, g.shape[0], g.shape[1], _dptr(g), _dptr(data), _dptr(sigma2),
                                      _dptr(status), _dptr(logl), _stream(stream)))


class sperm_tmcmc_model(ctypes.Structure):
    _fields_ = [("shape", swim_sperm_shape), ("sys_row", ctypes.c_double * 10), ("n_theta", ctypes.c_int32),
                ("n_sigma", ctypes.c_int32), ("field", ctypes.c_int32 * 3), ("kind", ctypes.c_int32),
                ("beta", ctypes.c_double * 2), ("steps", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("dt", ctypes.c_double), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def sperm_model(shape, sys_row, fields, n_sigma, kind, beta, steps, obs_every, dt, dtype=SWIM_F64):
    """fields: names from SPERM_FIELDS set by the leading theta entries."""
    m = sperm_tmcmc_model()
    m.shape = shape
    for i, v in enumerate(sys_row):
        m.sys_row[i] = float(v)
    m.n_theta = len(fields) + int(n_sigma)
    m.n_sigma = int(n_sigma)
    for i, f in enumerate(fields[:3]):
        m.field[i] = SPERM_FIELDS.index(f)
    m.kind = int(kind)
    m.beta[0], m.beta[1] = float(beta[0]), float(beta[1])
    m.steps, m.obs_every, m.dt, m.dtype = int(steps), int(obs_every), float(dt), int(dtype)
    return m


def tmcmc_sperm_run(ctx, model, swim_rows, lo, hi, data, n, seed, cv_target=1.0, cov_scale=0.2, max_stages=40):
    """One TMCMC run over the sperm model; host arrays in and out."""
    sw, sw_p = _h(swim_rows, np.float64, _DP)
    d_, d_p = _h(data, np.float64, _DP)
    dth = model.n_theta
    o = tmcmc_opts()
    for i in range(min(4, len(lo), len(hi))):
        o.lo[i] = float(lo[i])
        o.hi[i] = float(hi[i])
    o.cv_target, o.cov_scale, o.max_stages = float(cv_target), float(cov_scale), int(max_stages)
    theta = np.empty((max(n, 1), max(dth, 1)))
    logl = np.empty(max(n, 1))
    q = np.full(max_stages + 1, np.nan)
    ns = np.zeros(1, dtype=np.int32)
    lev = np.empty(1)
    acc = np.zeros(max_stages, dtype=np.int64)
    runs = np.zeros(1, dtype=np.int64)
    secs = np.zeros(1)
    _check(lib().tmcmc_sperm_run(ctx.handle, ctypes.byref(model), sw_p, ctypes.byref(o), d_p, d_.shape[0], int(n),
                                 int(seed), theta.ctypes.data_as(_DP), logl.ctypes.data_as(_DP),
                                 q.ctypes.data_as(_DP), ns.ctypes.data_as(_I32P), lev.ctypes.data_as(_DP),
                                 acc.ctypes.data_as(_I64P), runs.ctypes.data_as(_I64P), secs.ctypes.data_as(_DP)))
    k = int(ns[0])
    return dict(theta=theta, logl=logl, q=q[:k + 1], n_stages=k, log_evidence=float(lev[0]), accepted=acc[:k],
                runs=int(runs[0]), seconds=float(secs[0]))


def swim_flow_field(ctx, x, y, fx, fy, alpha, eps, tx, ty, u, v, p, stream=None):
    """Velocity and pressure at target points (device tensors of one dtype)."""
    return _check(lib().swim_flow_field(ctx.handle, dtype_code(x), x.numel(), _dptr(x), _dptr(y), _dptr(fx),
                                        _dptr(fy), float(alpha), float(eps), tx.numel(), _dptr(tx), _dptr(ty),
                                        _dptr(u), _dptr(v), _dptr(p), _stream(stream)))
