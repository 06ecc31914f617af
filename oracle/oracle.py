"""ctypes wrapper of the plain FP64 C oracle (test infrastructure only).

Every function mirrors one C entry point of sbv_oracle.c / mlp_oracle.c and only
marshals numpy arrays; all arithmetic is in the C code.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ENOTPD = 0, 1, 2, 4

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_f = C.POINTER(C.c_float)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.sbv_oracle_rho.restype = C.c_double
        L.sbv_oracle_rho.argtypes = [C.c_double, C.c_int]
        L.sbv_oracle_mdrho_over_r.restype = C.c_double
        L.sbv_oracle_mdrho_over_r.argtypes = [C.c_double, C.c_int]
        L.sbv_oracle_cov_matrix.argtypes = [_d, C.c_int64, _d, C.c_int64, C.c_int, _d, C.c_int, C.c_int, _d]
        L.sbv_oracle_exact_loglik.argtypes = [_d, _d, C.c_int64, C.c_int, _d, C.c_int, _d, _d]
        L.sbv_oracle_build.restype = C.c_void_p
        L.sbv_oracle_build.argtypes = [_d, C.c_int64, C.c_int, _d, C.c_int64, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_uint64]
        L.sbv_oracle_structure_info.argtypes = [C.c_void_p, _i64, _i64, _i64, C.POINTER(C.c_int)]
        L.sbv_oracle_structure_get.argtypes = [C.c_void_p, _i64, _i64, _i64, _i64, _d]
        L.sbv_oracle_structure_free.argtypes = [C.c_void_p]
        L.sbv_oracle_sbv_loglik.argtypes = [_d, _d, C.c_int64, C.c_int, C.c_int64, _i64, _i64, _i64, _i64,
                                            _d, C.c_int, _d, _d, _d, C.c_int, _d]
        L.sbv_oracle_sample.argtypes = [_d, C.c_int64, C.c_int, C.c_int64, _i64, _i64, _i64, _i64, _d,
                                        C.c_int, _d, _d]
        L.sbv_oracle_predict.argtypes = [_d, _d, C.c_int64, C.c_int, _d, C.c_int64, C.c_int64, _i64, _i64, _i64,
                                         _i64, _d, C.c_int, _d, _d]
        L.sbv_oracle_pred_neighbours.argtypes = [_d, C.c_int64, C.c_int, _d, C.c_int64, _i64, _i64, _d, C.c_int,
                                                 _i64]
        if hasattr(L, "mlp_oracle_forward"):
            L.mlp_oracle_forward.argtypes = [_d, C.c_int, _d, C.c_int, C.c_int, C.c_int, C.c_int, _d, _d]
            L.mlp_oracle_loss_grad.restype = C.c_double
            L.mlp_oracle_loss_grad.argtypes = [_d, C.c_int, _d, _d, C.c_int, C.c_int, C.c_int, C.c_int, _d]
            L.mlp_oracle_adam.argtypes = [_d, _d, _d, _d, C.c_int64, C.c_int, C.c_double, C.c_double,
                                          C.c_double, C.c_double]
            L.sbv_oracle_features.argtypes = [_d, _d, C.c_int64, C.c_int, _i64, C.c_int64, _d]
        _LIB = L
    return _LIB


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ci64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def rho(r, two_nu):
    """Matern correlation of Eq. (maternkernel) in the literal parameterisation."""
    return lib().sbv_oracle_rho(float(r), int(two_nu))


def mdrho_over_r(r, two_nu):
    return lib().sbv_oracle_mdrho_over_r(float(r), int(two_nu))


def cov_matrix(Xa, Xb, theta, two_nu, same):
    Xa, Xb, th = _c64(Xa), _c64(Xb), _c64(theta)
    out = np.empty((Xa.shape[0], Xb.shape[0]))
    st = lib().sbv_oracle_cov_matrix(_p(Xa), Xa.shape[0], _p(Xb), Xb.shape[0], Xa.shape[1], _p(th),
                                     int(two_nu), int(bool(same)), _p(out))
    assert st == 0, st
    return out


def exact_loglik(X, y, theta, two_nu, grad=False):
    """Exact GP log-likelihood, Eq. (1); optionally its gradient in log theta."""
    X, y, th = _c64(X), _c64(y), _c64(theta)
    ll = np.zeros(1)
    g = np.zeros(X.shape[1] + 2) if grad else None
    st = lib().sbv_oracle_exact_loglik(_p(X), _p(y), X.shape[0], X.shape[1], _p(th), int(two_nu), _p(ll),
                                       _p(g) if grad else None)
    if st not in (OR_OK, OR_ENOTPD):
        raise ValueError(f"oracle exact_loglik status {st}")
    return (ll[0], g) if grad else ll[0]


class Structure:
    """Block structure in the exchange format (original point ids)."""

    def __init__(self, n, d, m, block_ptr, block_pts, nn_ptr, nn_idx, kmeans_obj=None):
        self.n, self.d, self.m = int(n), int(d), int(m)
        self.block_ptr = _ci64(block_ptr)
        self.block_pts = _ci64(block_pts)
        self.nn_ptr = _ci64(nn_ptr)
        self.nn_idx = _ci64(nn_idx)
        self.kmeans_obj = kmeans_obj

    @property
    def K(self):
        return len(self.block_ptr) - 1

    def block(self, r):
        return (self.block_pts[self.block_ptr[r]:self.block_ptr[r + 1]],
                self.nn_idx[self.nn_ptr[r]:self.nn_ptr[r + 1]])


def subset(S, blocks):
    """Sub-structure holding only the listed blocks (ids still index the full X)."""
    bp, pts, npt, nid = [0], [], [0], []
    for r in blocks:
        B, J = S.block(int(r))
        pts.extend(B.tolist())
        nid.extend(J.tolist())
        bp.append(len(pts))
        npt.append(len(nid))
    return Structure(S.n, S.d, S.m, bp, pts, npt, nid)


def build(X, beta_build, K, m, lloyd_iters=10, min_bs=0, max_bs=0, seed=0):
    """Oracle block builder: scaling, anchors/k-means, size bounds, random order,
    centres and exact m nearest earlier neighbours."""
    X, bb = _c64(X), _c64(beta_build)
    n, d = X.shape
    L = lib()
    h = L.sbv_oracle_build(_p(X), n, d, _p(bb), int(K), int(m), int(lloyd_iters), int(min_bs), int(max_bs),
                           C.c_uint64(int(seed)))
    if not h:
        raise ValueError("oracle build rejected its arguments")
    try:
        nn_, K_, nnz, nobj = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int()
        L.sbv_oracle_structure_info(h, C.byref(nn_), C.byref(K_), C.byref(nnz), C.byref(nobj))
        bp = np.empty(K_.value + 1, np.int64)
        pts = np.empty(n, np.int64)
        npt = np.empty(K_.value + 1, np.int64)
        nidx = np.empty(max(nnz.value, 1), np.int64)
        obj = np.empty(max(nobj.value, 1))
        L.sbv_oracle_structure_get(h, _p(bp, _i64), _p(pts, _i64), _p(npt, _i64), _p(nidx, _i64), _p(obj))
    finally:
        L.sbv_oracle_structure_free(h)
    return Structure(n, d, m, bp, pts, npt, nidx[:nnz.value], obj[:nobj.value])


def sbv_loglik(X, y, S, theta, two_nu, grad=False, blocks=False, nthreads=0, parts=False):
    """SBV log-likelihood (sum of Alg. 5 block terms); optionally the per-block
    terms, the gradient in log theta, and (parts=True, not with grad) each
    block's u_i = v^T v and d_i = 2 log det L' as a K x 2 array."""
    X, y, th = _c64(X), _c64(y), _c64(theta)
    n, d = X.shape
    ll = np.zeros(1)
    lb = np.empty(S.K)
    g = np.zeros(d + 2)
    ud = np.full((S.K, 2), np.nan) if parts else None
    st = lib().sbv_oracle_sbv_loglik(_p(X), _p(y), n, d, S.K, _p(S.block_ptr, _i64), _p(S.block_pts, _i64),
                                     _p(S.nn_ptr, _i64), _p(S.nn_idx if len(S.nn_idx) else np.zeros(1, np.int64), _i64),
                                     _p(th), int(two_nu), _p(lb), _p(ll), _p(g) if grad else None, int(nthreads),
                                     _p(ud) if parts else None)
    if st == OR_EINVAL:
        raise ValueError("oracle sbv_loglik rejected its arguments")
    out = [ll[0]]
    if grad:
        out.append(g)
    if blocks:
        out.append(lb)
    if parts:
        out.append(ud)
    return out[0] if len(out) == 1 else tuple(out)


def sample(X, S, theta, two_nu, xi):
    """Vecchia conditional simulator over the structure's rank order."""
    X, th, xi = _c64(X), _c64(theta), _c64(xi)
    n, d = X.shape
    y = np.zeros(n)
    st = lib().sbv_oracle_sample(_p(X), n, d, S.K, _p(S.block_ptr, _i64), _p(S.block_pts, _i64),
                                 _p(S.nn_ptr, _i64), _p(S.nn_idx if len(S.nn_idx) else np.zeros(1, np.int64), _i64),
                                 _p(th), int(two_nu), _p(xi), _p(y))
    if st != OR_OK:
        raise ValueError(f"oracle sample status {st}")
    return y


def mlp_shapes(n_in, hidden, layers, n_out):
    """Offsets of each layer's (W, b) in the packed parameter vector."""
    offs, o, din = [], 0, n_in
    for l in range(layers + 1):
        dout = hidden if l < layers else n_out
        offs.append((o, dout, din))
        o += dout * din + dout
        din = hidden
    return offs, o


def mlp_forward(params, X, n_in, hidden, layers, n_out):
    p, X = _c64(params), _c64(X)
    out = np.empty((X.shape[0], n_out))
    lib().mlp_oracle_forward(_p(p), n_in, _p(X), X.shape[0], hidden, layers, n_out, _p(out), None)
    return out


def mlp_loss_grad(params, X, Y, n_in, hidden, layers, n_out):
    p, X, Y = _c64(params), _c64(X), _c64(Y)
    g = np.empty(len(p))
    loss = lib().mlp_oracle_loss_grad(_p(p), n_in, _p(X), _p(Y), X.shape[0], hidden, layers, n_out, _p(g))
    return loss, g


def mlp_adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays p, m, v."""
    gg = _c64(g)
    lib().mlp_oracle_adam(_p(p), _p(gg), _p(m), _p(v), len(p), int(t), float(lr), float(b1), float(b2), float(eps))


def features(X, y, sub):
    X, y, sub = _c64(X), _c64(y), _ci64(sub)
    d = X.shape[1]
    f = np.empty(4 + 5 * (d + 2))
    st = lib().sbv_oracle_features(_p(X), _p(y), X.shape[0], d, _p(sub, _i64), len(sub), _p(f))
    if st:
        raise ValueError("oracle features rejected its arguments")
    return f


def pred_structure(X, Xp, beta_build, K, m, lloyd_iters=10, min_bs=0, max_bs=0, seed=0):
    """Prediction structure: blocks of the new points Xp (the oracle builder's
    clustering with no conditioning) and, per block, the m observed points of X
    nearest its centroid.  Returned as a Structure over Xp's ids whose nn_idx
    are observed ids."""
    B = build(Xp, beta_build, K, 0, lloyd_iters=lloyd_iters, min_bs=min_bs, max_bs=max_bs, seed=seed)
    X, Xp, bb = _c64(X), _c64(Xp), _c64(beta_build)
    mm = min(int(m), X.shape[0])
    nid = np.empty(max(B.K * mm, 1), np.int64)
    st = lib().sbv_oracle_pred_neighbours(_p(X), X.shape[0], X.shape[1], _p(Xp), B.K, _p(B.block_ptr, _i64),
                                          _p(B.block_pts, _i64), _p(bb), int(m), _p(nid, _i64))
    if st:
        raise ValueError("oracle pred_neighbours rejected its arguments")
    return Structure(Xp.shape[0], X.shape[1], mm, B.block_ptr, B.block_pts, np.arange(B.K + 1) * mm,
                     nid[:B.K * mm])


def predict(X, y, Xp, P, theta, two_nu):
    """Predictive means and variances diag(Sigma_new) of the new points (Alg. 5
    Step 1 per prediction block), in the order of Xp."""
    X, y, Xp, th = _c64(X), _c64(y), _c64(Xp), _c64(theta)
    mean = np.empty(Xp.shape[0])
    var = np.empty(Xp.shape[0])
    st = lib().sbv_oracle_predict(_p(X), _p(y), X.shape[0], X.shape[1], _p(Xp), Xp.shape[0], P.K,
                                  _p(P.block_ptr, _i64), _p(P.block_pts, _i64), _p(P.nn_ptr, _i64),
                                  _p(P.nn_idx if len(P.nn_idx) else np.zeros(1, np.int64), _i64), _p(th),
                                  int(two_nu), _p(mean), _p(var))
    if st == OR_EINVAL:
        raise ValueError("oracle predict rejected its arguments")
    return mean, var


def pred_draws(mean, var, xi):
    """Conditional simulation of predictions (Sec. 5.5): draws mean + sqrt(var) xi
    (xi: n_draws x n_pred), their sample mean and variance (divisor n_draws - 1)
    and the 95 % interval sample mean -/+ z_{0.025} sample sd."""
    from scipy.stats import norm
    draws = np.asarray(mean)[None, :] + np.sqrt(np.asarray(var))[None, :] * np.asarray(xi)
    m = draws.mean(axis=0)
    v = draws.var(axis=0, ddof=1)
    z = norm.ppf(0.975)
    return m, v, m - z * np.sqrt(v), m + z * np.sqrt(v)
