"""Thin ctypes binding of libsbv.so (argument marshalling only).

Every function here carries the name of the C entry point it calls
(include/sbv.h) and only converts arguments; all computation happens in the
HIP library.  If libsbv.so is missing the first call raises -- there is no
fallback path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsbv.so")
_LIB = None

SBV_OK, SBV_E_INVAL, SBV_E_NOMEM, SBV_E_DEVICE, SBV_E_NOTPD, SBV_E_NOCONV = range(6)
SBV_FP64, SBV_FP32 = 0, 1
SBV_KMEANS, SBV_RAC = 0, 1
SBV_NELDER_MEAD, SBV_LBFGS = 0, 1

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_i32 = C.POINTER(C.c_int32)
_h = C.c_void_p
_f32 = C.POINTER(C.c_float)


class SBVError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sbv status {status}: {msg}")
        self.status = status


class sbv_build_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("lloyd_iters", C.c_int32), ("min_bs", C.c_int32),
                ("max_bs", C.c_int32), ("n_slabs", C.c_int32), ("seed", C.c_uint64), ("nns_alpha", C.c_double)]


class sbv_fit_opts(C.Structure):
    _fields_ = [("optimizer", C.c_int32), ("prec", C.c_int32), ("fp64_polish", C.c_int32),
                ("max_evals", C.c_int32), ("ftol", C.c_double), ("gtol", C.c_double),
                ("rebuild_rounds", C.c_int32), ("lbfgs_m", C.c_int32), ("init_step", C.c_double),
                ("checkpoint_path", C.c_char_p)]


def lib():
    """Load libsbv.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_2504_12004_amd/build.py")
    # PyTorch (when installed) carries its own copy of the HIP runtime under a
    # different file name; importing it first makes the process use that one
    # runtime for both torch and this library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(_LIB_PATH)
    sig = {
        "sbv_last_error": (C.c_char_p, []),
        "sbv_max_joint_size": (C.c_int32, []),
        "sbv_build_blocks": (C.c_int, [_d, _d, C.c_int64, C.c_int32, _d, C.c_int64, C.c_int32,
                                       C.POINTER(sbv_build_opts), C.POINTER(_h)]),
        "sbv_blocks_import": (C.c_int, [_d, _d, C.c_int64, C.c_int32, C.c_int64, _i64, _i64, _i64, _i64,
                                        C.POINTER(_h)]),
        "sbv_blocks_info": (C.c_int, [_h, _i64, _i32, _i64, _i64]),
        "sbv_blocks_export": (C.c_int, [_h, _i64, _i64, _i64, _i64]),
        "sbv_blocks_set_y": (C.c_int, [_h, _d]),
        "sbv_blocks_set_y_dev": (C.c_int, [_h, C.c_void_p, C.c_void_p]),
        "sbv_blocks_free": (None, [_h]),
        "sbv_loglik": (C.c_int, [C.POINTER(_h), C.c_int32, _d, _i32, C.c_int32, _d]),
        "sbv_loglik_dev": (C.c_int, [C.POINTER(_h), C.c_int32, C.c_void_p, _i32, C.c_int32, C.c_void_p,
                                     C.c_void_p]),
        "sbv_loglik_noalloc_dev": (C.c_int, [_h, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
        "sbv_loglik_grad": (C.c_int, [C.POINTER(_h), C.c_int32, _d, _i32, C.c_int32, _d, _d]),
        "sbv_loglik_grad_dev": (C.c_int, [C.POINTER(_h), C.c_int32, C.c_void_p, _i32, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_void_p]),
        "sbv_blocks_fallback_count": (C.c_int, [_h, _i64]),
        "sbv_blocks_terms": (C.c_int, [_h, _d]),
        "sbv_sample": (C.c_int, [_h, _d, C.c_int32, _d, _d]),
        "sbv_sample_dev": (C.c_int, [_h, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
        "sbv_fit": (C.c_int, [_h, _d, C.c_int32, C.POINTER(sbv_fit_opts), _d, _d, _i32, _d]),
        "sbv_minimize": (C.c_int, [C.c_int32, C.c_int32, _d, C.c_void_p, C.c_void_p, C.POINTER(sbv_fit_opts), _d,
                                   _i32]),
        "sbv_mlp_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_h)]),
        "sbv_mlp_free": (None, [_h]),
        "sbv_mlp_num_params": (C.c_int64, [_h]),
        "sbv_mlp_get_params": (C.c_int, [_h, _f32]),
        "sbv_mlp_set_params": (C.c_int, [_h, _f32]),
        "sbv_mlp_loss_grad": (C.c_int, [_h, _f32, _f32, C.c_int32, _f32, _f32]),
        "sbv_mlp_train": (C.c_int, [_h, _f32, _f32, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64, _f32]),
        "sbv_mlp_predict": (C.c_int, [_h, _f32, C.c_int64, _f32]),
        "sbv_mlp_save": (C.c_int, [_h, C.c_char_p]),
        "sbv_mlp_load": (C.c_int, [C.c_char_p, C.POINTER(_h)]),
        "sbv_features": (C.c_int, [_d, _d, C.c_int64, C.c_int32, C.c_int64, C.c_uint64, _d]),
        "sbv_pred_build": (C.c_int, [_h, _d, C.c_int64, _d, C.c_int64, C.c_int32, C.POINTER(sbv_build_opts),
                                     C.POINTER(_h)]),
        "sbv_pred_import": (C.c_int, [_h, _d, C.c_int64, C.c_int64, _i64, _i64, _i64, _i64, C.POINTER(_h)]),
        "sbv_pred_info": (C.c_int, [_h, _i64, _i64, _i64]),
        "sbv_pred_export": (C.c_int, [_h, _i64, _i64, _i64, _i64]),
        "sbv_pred_free": (None, [_h]),
        "sbv_predict": (C.c_int, [_h, _d, C.c_int32, _d, _d]),
        "sbv_predict_draws_dev": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                            C.c_void_p]),
        "sbv_cov_matrix_dev": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                         C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
        "sbv_eval_graph_dev": (C.c_int, [C.POINTER(_h), C.c_int32, C.c_void_p, _i32, C.c_int32, C.c_int32,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
        "sbv_autotune": (C.c_int, [C.POINTER(_h), C.c_int32, _i32, _d, C.c_int32, C.c_int32, _i32, _i32, _i32,
                                   _i32]),
        "sbv_timing_enable": (C.c_int, [C.c_int32]),
        "sbv_timing_read": (C.c_int, [C.c_int32, _i32, _d, _i64]),
        "sbv_plan_flops": (C.c_int, [C.POINTER(_h), C.c_int32, _i32, _d, _i32, _i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(st):
    if st != SBV_OK:
        raise SBVError(st, lib().sbv_last_error().decode())


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ci64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a, t=_d):
    return a.ctypes.data_as(t)


class Blocks:
    """Owning wrapper of an sbv_blocks handle.  Its sizes are read from the
    library on every access (sbv_fit with rebuild rounds changes them)."""

    def __init__(self, handle):
        self.handle = C.c_void_p(handle)
        self._info()

    def _info(self):
        n, d, K, nnz = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(lib().sbv_blocks_info(self.handle, C.byref(n), C.byref(d), C.byref(K), C.byref(nnz)))
        return n.value, d.value, K.value, nnz.value

    n = property(lambda self: self._info()[0])
    d = property(lambda self: self._info()[1])
    K = property(lambda self: self._info()[2])
    nnz = property(lambda self: self._info()[3])

    def free(self):
        if self.handle is not None and self.handle.value:
            lib().sbv_blocks_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sbv_blocks_import(X, y, block_ptr, block_pts, nn_ptr, nn_idx):
    X = _c64(X)
    n, d = X.shape
    y = None if y is None else _c64(y)
    bp, pts, npt, nid = _ci64(block_ptr), _ci64(block_pts), _ci64(nn_ptr), _ci64(nn_idx)
    if len(nid) == 0:
        nid = np.zeros(1, np.int64)
    h = C.c_void_p()
    _check(lib().sbv_blocks_import(_p(X), _p(y) if y is not None else None, n, d, len(bp) - 1, _p(bp, _i64),
                                   _p(pts, _i64), _p(npt, _i64), _p(nid, _i64), C.byref(h)))
    return Blocks(h.value)


def sbv_build_blocks(X, y, beta_build, n_blocks, m, method=SBV_KMEANS, lloyd_iters=10, min_bs=0, max_bs=0,
                     seed=0, n_slabs=1, nns_alpha=0.0):
    X = _c64(X)
    n, d = X.shape
    y = None if y is None else _c64(y)
    bb = _c64(beta_build)
    o = sbv_build_opts(int(method), int(lloyd_iters), int(min_bs), int(max_bs), int(n_slabs), int(seed),
                       float(nns_alpha))
    h = C.c_void_p()
    _check(lib().sbv_build_blocks(_p(X), _p(y) if y is not None else None, n, d, _p(bb), int(n_blocks), int(m),
                                  C.byref(o), C.byref(h)))
    return Blocks(h.value)


def sbv_blocks_export(b):
    n, _, K, nnz = b._info()
    bp = np.empty(K + 1, np.int64)
    pts = np.empty(n, np.int64)
    npt = np.empty(K + 1, np.int64)
    nid = np.empty(max(nnz, 1), np.int64)
    _check(lib().sbv_blocks_export(b.handle, _p(bp, _i64), _p(pts, _i64), _p(npt, _i64), _p(nid, _i64)))
    return bp, pts, npt, nid[:nnz]


def sbv_blocks_set_y(b, y):
    y = _c64(y)
    _check(lib().sbv_blocks_set_y(b.handle, _p(y)))


def sbv_blocks_set_y_dev(b, y_dev, stream=None):
    """y_dev: a device tensor/pointer (torch tensor accepted), original order."""
    _check(lib().sbv_blocks_set_y_dev(b.handle, C.c_void_p(_ptr(y_dev)), C.c_void_p(_stream(stream))))


def _handles(sets):
    if isinstance(sets, Blocks):
        sets = [sets]
    arr = (C.c_void_p * len(sets))(*[s.handle.value for s in sets])
    return arr, len(sets)


def _ptr(t):
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return int(t)


def _stream(s):
    if s is None:
        return 0
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def sbv_loglik(sets, theta, two_nu, prec=SBV_FP64):
    hs, ns = _handles(sets)
    th = _c64(np.concatenate([np.ravel(t) for t in theta]) if isinstance(theta, (list, tuple)) else theta)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    out = np.empty(ns)
    _check(lib().sbv_loglik(hs, ns, _p(th), _p(tn, _i32), int(prec), _p(out)))
    return out


def sbv_loglik_dev(sets, theta_dev, two_nu, out_dev, prec=SBV_FP64, stream=None):
    hs, ns = _handles(sets)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    _check(lib().sbv_loglik_dev(hs, ns, C.c_void_p(_ptr(theta_dev)), _p(tn, _i32), int(prec),
                                C.c_void_p(_ptr(out_dev)), C.c_void_p(_stream(stream))))


def sbv_loglik_noalloc_dev(b, theta_dev, two_nu, out_dev, prec=SBV_FP64, stream=None):
    _check(lib().sbv_loglik_noalloc_dev(b.handle, C.c_void_p(_ptr(theta_dev)), int(two_nu), int(prec),
                                        C.c_void_p(_ptr(out_dev)), C.c_void_p(_stream(stream))))


def sbv_loglik_grad(sets, theta, two_nu, prec=SBV_FP64):
    hs, ns = _handles(sets)
    th = _c64(np.concatenate([np.ravel(t) for t in theta]) if isinstance(theta, (list, tuple)) else theta)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    out = np.empty(ns)
    g = np.empty(len(th))
    _check(lib().sbv_loglik_grad(hs, ns, _p(th), _p(tn, _i32), int(prec), _p(out), _p(g)))
    return out, g


def sbv_loglik_grad_dev(sets, theta_dev, two_nu, out_dev, grad_dev, prec=SBV_FP64, stream=None):
    hs, ns = _handles(sets)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    _check(lib().sbv_loglik_grad_dev(hs, ns, C.c_void_p(_ptr(theta_dev)), _p(tn, _i32), int(prec),
                                     C.c_void_p(_ptr(out_dev)), C.c_void_p(_ptr(grad_dev)),
                                     C.c_void_p(_stream(stream))))


def sbv_blocks_fallback_count(b):
    c = C.c_int64()
    _check(lib().sbv_blocks_fallback_count(b.handle, C.byref(c)))
    return c.value


def sbv_blocks_terms(b):
    out = np.empty(b.K)
    _check(lib().sbv_blocks_terms(b.handle, _p(out)))
    return out


def sbv_max_joint_size():
    return lib().sbv_max_joint_size()


def sbv_blocks_free(b):
    b.free()


def sbv_blocks_info(b):
    return b._info()


def sbv_last_error():
    return lib().sbv_last_error().decode()


def sbv_timing_enable(on):
    _check(lib().sbv_timing_enable(int(bool(on))))


def sbv_timing_read(prec):
    """Per-variant (ms_total, launches) of timed launches of one precision."""
    nv = C.c_int32()
    ms = np.zeros(16)
    la = np.zeros(16, np.int64)
    _check(lib().sbv_timing_read(int(prec), C.byref(nv), _p(ms), _p(la, _i64)))
    return ms[:nv.value], la[:nv.value]


def sbv_plan_flops(sets, two_nu):
    """Per-variant algorithmic FLOP of one evaluation and the variants' tile capacities."""
    hs, ns = _handles(sets)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    fl = np.zeros(16)
    tiles = np.zeros(16, np.int32)
    nv = C.c_int32()
    _check(lib().sbv_plan_flops(hs, ns, _p(tn, _i32), _p(fl), _p(tiles, _i32), C.byref(nv)))
    return fl[:nv.value], tiles[:nv.value]


def sbv_sample(b, theta, two_nu, xi):
    """Vecchia conditional simulation on b's structure; returns y (original order)."""
    th, x = _c64(theta), _c64(xi)
    y = np.empty(b.n)
    _check(lib().sbv_sample(b.handle, _p(th), int(two_nu), _p(x), _p(y)))
    return y


def sbv_sample_dev(b, theta_dev, two_nu, xi_dev, y_dev=None, stream=None):
    _check(lib().sbv_sample_dev(b.handle, C.c_void_p(_ptr(theta_dev)), int(two_nu), C.c_void_p(_ptr(xi_dev)),
                                C.c_void_p(_ptr(y_dev) if y_dev is not None else 0), C.c_void_p(_stream(stream))))


OBJECTIVE = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


def make_fit_opts(optimizer=SBV_LBFGS, prec=SBV_FP64, fp64_polish=False, max_evals=500, ftol=1e-12, gtol=1e-6,
                  lbfgs_m=10, init_step=0.5, checkpoint_path=None, rebuild_rounds=0):
    return sbv_fit_opts(int(optimizer), int(prec), int(bool(fp64_polish)), int(max_evals), float(ftol), float(gtol),
                        int(rebuild_rounds), int(lbfgs_m), float(init_step),
                        checkpoint_path.encode() if checkpoint_path else None)


def sbv_minimize(method, x0, fn, opts):
    """Minimise fn(x) -> f or fn(x, want_grad) -> (f, g) with the library's optimisers."""
    x = _c64(x0).copy()
    n = len(x)

    def cb(xp, gp, _ctx):
        xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        if gp:
            f, g = fn(xv, True)
            gv = np.ctypeslib.as_array(gp, shape=(n,))
            gv[:] = g
            return float(f)
        return float(fn(xv, False))

    cfun = OBJECTIVE(cb)
    fb = C.c_double()
    ne = C.c_int32()
    st = lib().sbv_minimize(int(method), n, _p(x), C.cast(cfun, C.c_void_p), None, C.byref(opts), C.byref(fb),
                            C.byref(ne))
    if st not in (SBV_OK, SBV_E_NOCONV):
        _check(st)
    return x, fb.value, ne.value, st == SBV_OK


def sbv_fit(b, theta0, two_nu, opts):
    """MLE on one handle; returns (theta_hat, loglik_fp64, n_evals, seconds, converged)."""
    th = _c64(theta0)
    out = np.empty_like(th)
    l64 = C.c_double()
    ne = C.c_int32()
    sec = C.c_double()
    st = lib().sbv_fit(b.handle, _p(th), int(two_nu), C.byref(opts), _p(out), C.byref(l64), C.byref(ne),
                       C.byref(sec))
    if st not in (SBV_OK, SBV_E_NOCONV):
        _check(st)
    return out, l64.value, ne.value, sec.value, st == SBV_OK


def _cf32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class MLP:
    """Owning wrapper of an sbv_mlp handle."""

    def __init__(self, handle, n_out=None):
        self.handle = C.c_void_p(handle)
        self.num_params = lib().sbv_mlp_num_params(self.handle)
        self.n_out = n_out

    def free(self):
        if self.handle is not None and self.handle.value:
            lib().sbv_mlp_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sbv_mlp_create(n_in, hidden, layers, n_out, seed=0):
    h = C.c_void_p()
    _check(lib().sbv_mlp_create(int(n_in), int(hidden), int(layers), int(n_out), int(seed), C.byref(h)))
    return MLP(h.value, int(n_out))


def sbv_mlp_free(m):
    m.free()


def sbv_mlp_num_params(m):
    return m.num_params


def sbv_mlp_get_params(m):
    out = np.empty(m.num_params, np.float32)
    _check(lib().sbv_mlp_get_params(m.handle, _p(out, _f32)))
    return out


def sbv_mlp_set_params(m, params):
    p = _cf32(params)
    _check(lib().sbv_mlp_set_params(m.handle, _p(p, _f32)))


def sbv_mlp_loss_grad(m, X, Y):
    X, Y = _cf32(X), _cf32(Y)
    loss = C.c_float()
    g = np.empty(m.num_params, np.float32)
    _check(lib().sbv_mlp_loss_grad(m.handle, _p(X, _f32), _p(Y, _f32), X.shape[0], C.byref(loss), _p(g, _f32)))
    return loss.value, g


def sbv_mlp_train(m, X, Y, epochs, batch=256, lr=1e-3, seed=0):
    X, Y = _cf32(X), _cf32(Y)
    fl = C.c_float()
    _check(lib().sbv_mlp_train(m.handle, _p(X, _f32), _p(Y, _f32), X.shape[0], int(epochs), int(batch), float(lr),
                               int(seed), C.byref(fl)))
    return fl.value


def sbv_mlp_predict(m, X):
    X = _cf32(X)
    out = np.empty((X.shape[0], _mlp_out(m)), np.float32)
    _check(lib().sbv_mlp_predict(m.handle, _p(X, _f32), X.shape[0], _p(out, _f32)))
    return out


def _mlp_out(m):
    return m.n_out


def sbv_mlp_save(m, path):
    _check(lib().sbv_mlp_save(m.handle, str(path).encode()))


def sbv_mlp_load(path, n_out):
    h = C.c_void_p()
    _check(lib().sbv_mlp_load(str(path).encode(), C.byref(h)))
    return MLP(h.value, int(n_out))


def sbv_features(X, y, sub_n=20000, seed=0):
    X, y = _c64(X), _c64(y)
    n, d = X.shape
    f = np.empty(4 + 5 * (d + 2))
    _check(lib().sbv_features(_p(X), _p(y), n, d, int(sub_n), int(seed), _p(f)))
    return f


def sbv_eval_graph_dev(sets, theta_dev, two_nu, out_dev, prec=SBV_FP64, grad_dev=None, stream=None):
    hs, ns = _handles(sets)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    _check(lib().sbv_eval_graph_dev(hs, ns, C.c_void_p(_ptr(theta_dev)), _p(tn, _i32), int(prec),
                                    int(grad_dev is not None), C.c_void_p(_ptr(out_dev)),
                                    C.c_void_p(_ptr(grad_dev) if grad_dev is not None else 0),
                                    C.c_void_p(_stream(stream))))


def sbv_autotune(sets, theta, two_nu, prec=SBV_FP64, reps=2, with_schedule=False):
    """Chosen tile capacity per size bucket; with_schedule=True also returns
    the per-bucket lookahead choice (1 = lookahead schedule), the waves per
    workgroup of the chosen kernel, and whether the single persistent launch
    won over per-bucket launches."""
    hs, ns = _handles(sets)
    th = _c64(np.concatenate([np.ravel(t) for t in theta]) if isinstance(theta, (list, tuple)) else theta)
    tn = np.ascontiguousarray(np.broadcast_to(np.asarray(two_nu, np.int32), (ns,)), dtype=np.int32)
    ch = np.zeros(16, np.int32)
    la = np.zeros(16, np.int32)
    wv = np.zeros(16, np.int32)
    pers = C.c_int32()
    _check(lib().sbv_autotune(hs, ns, _p(tn, _i32), _p(th), int(prec), int(reps), _p(ch, _i32), _p(la, _i32),
                              _p(wv, _i32), C.byref(pers)))
    if with_schedule:
        return ch[ch > 0], la[ch > 0], wv[ch > 0], bool(pers.value)
    return ch[ch > 0]


class Pred:
    """Owning wrapper of an sbv_pred prediction structure (keeps its observed
    handle alive)."""

    def __init__(self, handle, blocks):
        self.handle = C.c_void_p(handle)
        self.blocks = blocks
        n, K, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().sbv_pred_info(self.handle, C.byref(n), C.byref(K), C.byref(nnz)))
        self.n_pred, self.K, self.nnz = n.value, K.value, nnz.value

    def free(self):
        if self.handle is not None and self.handle.value:
            lib().sbv_pred_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sbv_pred_build(b, Xp, beta_build, n_blocks, m_pred, method=SBV_KMEANS, lloyd_iters=10, min_bs=0, max_bs=0,
                   seed=0):
    Xp = _c64(Xp)
    bb = _c64(beta_build)
    o = sbv_build_opts(int(method), int(lloyd_iters), int(min_bs), int(max_bs), 1, int(seed), -1.0)
    h = C.c_void_p()
    _check(lib().sbv_pred_build(b.handle, _p(Xp), Xp.shape[0], _p(bb), int(n_blocks), int(m_pred), C.byref(o),
                                C.byref(h)))
    return Pred(h.value, b)


def sbv_pred_import(b, Xp, block_ptr, block_pts, nn_ptr, nn_idx):
    Xp = _c64(Xp)
    bp, pts, npt, nid = _ci64(block_ptr), _ci64(block_pts), _ci64(nn_ptr), _ci64(nn_idx)
    if len(nid) == 0:
        nid = np.zeros(1, np.int64)
    h = C.c_void_p()
    _check(lib().sbv_pred_import(b.handle, _p(Xp), Xp.shape[0], len(bp) - 1, _p(bp, _i64), _p(pts, _i64),
                                 _p(npt, _i64), _p(nid, _i64), C.byref(h)))
    return Pred(h.value, b)


def sbv_pred_export(p):
    bp = np.empty(p.K + 1, np.int64)
    pts = np.empty(p.n_pred, np.int64)
    npt = np.empty(p.K + 1, np.int64)
    nid = np.empty(max(p.nnz, 1), np.int64)
    _check(lib().sbv_pred_export(p.handle, _p(bp, _i64), _p(pts, _i64), _p(npt, _i64), _p(nid, _i64)))
    return bp, pts, npt, nid[:p.nnz]


def sbv_pred_info(p):
    return p.n_pred, p.K, p.nnz


def sbv_pred_free(p):
    p.free()


def sbv_predict(p, theta, two_nu):
    """Predictive means and variances (host arrays in the order of X*)."""
    th = _c64(theta)
    mean = np.empty(p.n_pred)
    var = np.empty(p.n_pred)
    _check(lib().sbv_predict(p.handle, _p(th), int(two_nu), _p(mean), _p(var)))
    return mean, var


def sbv_predict_draws_dev(mean_dev, var_dev, xi_dev, n_draws, stats_dev, stream=None):
    """Draw summaries on the device: stats_dev gets (mean, var, lo, hi) x n_pred."""
    n = int(mean_dev.numel()) if hasattr(mean_dev, "numel") else None
    _check(lib().sbv_predict_draws_dev(C.c_void_p(_ptr(mean_dev)), C.c_void_p(_ptr(var_dev)), n,
                                       C.c_void_p(_ptr(xi_dev)), int(n_draws), C.c_void_p(_ptr(stats_dev)),
                                       C.c_void_p(_stream(stream))))


def sbv_cov_matrix_dev(Xa_dev, Xb_dev, theta_dev, two_nu, out_dev, same=False, stream=None):
    """Dense covariance matrix on the device (torch tensors: Xa na x d, Xb nb x d, out na x nb)."""
    na, d = Xa_dev.shape
    nb = Xb_dev.shape[0]
    _check(lib().sbv_cov_matrix_dev(C.c_void_p(_ptr(Xa_dev)), int(na), C.c_void_p(_ptr(Xb_dev)), int(nb), int(d),
                                    C.c_void_p(_ptr(theta_dev)), int(two_nu), int(bool(same)),
                                    C.c_void_p(_ptr(out_dev)), C.c_void_p(_stream(stream))))
