"""Python handle on the oracle (``rfo.c``): a plain scalar FP64 CPU evaluator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It never imports the GPU package and
the GPU package never imports it.

The oracle follows the paper's account of RooFit's per-event evaluation
(Section 4): one event at a time, top node evaluated in FP64, parameter-only
branches (normalisations) computed once per parameter point, and
NLL = -sum_i log p_i with compensated summation.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rfo.c")
_LIB = os.path.join(_HERE, "librfo.so")

# node kinds: the oracle's own numbering (rfo.h)
KIND = {
    "obs": 1, "param": 2, "const": 3, "linear": 4, "product": 5, "ratio": 6, "extended": 32,
    "gauss": 10, "cheb": 11, "exp": 12, "decay_gauss": 13, "argus": 14,
    "bw": 15, "numconv_bw_cb": 16, "mlp": 17, "poisson": 18, "add": 30, "prod": 31,
}


def build(force=False):
    """Compile the oracle with gcc -O2 (no fast-math), single threaded."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        DP = ctypes.POINTER(ctypes.c_double)
        L.rfo_last_error.restype = ctypes.c_char_p
        L.rfo_model_new.restype = P
        L.rfo_model_free.argtypes = [P]
        L.rfo_node.argtypes = [P, I, ctypes.POINTER(ctypes.c_int), I, DP, I]
        L.rfo_n_params.argtypes = [P]
        L.rfo_n_obs.argtypes = [P]
        L.rfo_set_mlp_weights.argtypes = [P, I, DP]
        L.rfo_nll.argtypes = [P, I, DP, ctypes.POINTER(DP), I64, DP, DP, ctypes.POINTER(I64)]
        L.rfo_nll_ex.argtypes = [P, I, DP, ctypes.POINTER(DP), I64, DP, DP, DP, ctypes.POINTER(I64)]
        L.rfo_nll_w.argtypes = [P, I, DP, ctypes.POINTER(DP), DP, I64, DP, DP, DP, ctypes.POINTER(I64)]
        L.rfo_values.argtypes = [P, I, DP, ctypes.POINTER(DP), I64, DP]
        L.rfo_nll_hess.argtypes = [P, I, DP, ctypes.POINTER(DP), DP, I64, DP, DP, DP, ctypes.POINTER(I64)]
        L.rfo_norm.argtypes = [P, I, DP, DP, DP]
        L.rfo_gauss_legendre.argtypes = [I, D, D, DP, DP]
        L.rfo_mlp_forward.argtypes = [DP, DP, I64, DP]
        L.rfo_mlp_backward.argtypes = [DP, DP, I64, DP, DP, DP]
        L.rfo_binned_nll.argtypes = [I, I, I, I, DP, DP, DP, DP, DP, DP, DP]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc < 0:
        raise RuntimeError("oracle: %s (rc=%d)" % (lib().rfo_last_error().decode(), rc))
    return rc


class Model:
    """A model graph in the oracle.  Nodes are added in dependency order."""

    def __init__(self):
        self.h = lib().rfo_model_new()
        self._keep = []

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rfo_model_free(self.h)
            self.h = None

    def node(self, kind, inputs=(), attrs=()):
        ins = (ctypes.c_int * max(1, len(inputs)))(*inputs)
        at = _f64(list(attrs) if len(attrs) else [0.0])
        return _check(lib().rfo_node(self.h, KIND[kind], ins, len(inputs), _dp(at), len(attrs)))

    @property
    def n_params(self):
        return lib().rfo_n_params(self.h)

    @property
    def n_obs(self):
        return lib().rfo_n_obs(self.h)

    def set_mlp_weights(self, node, w):
        w = _f64(w)
        assert w.size == 8833
        _check(lib().rfo_set_mlp_weights(self.h, node, _dp(w)))

    def _cols(self, cols):
        cs = [_f64(c) for c in cols]
        assert len(cs) == self.n_obs
        n = len(cs[0]) if cs else 0
        arr = (ctypes.POINTER(ctypes.c_double) * max(1, len(cs)))(*[_dp(c) for c in cs])
        return cs, arr, n

    def nll(self, top, theta, cols, grad=True):
        th = _f64(theta)
        assert th.size == self.n_params
        cs, arr, n = self._cols(cols)
        out = ctypes.c_double()
        g = np.zeros(max(1, self.n_params))
        nb = ctypes.c_int64()
        _check(lib().rfo_nll(self.h, top, _dp(th), arr, n, ctypes.byref(out),
                             _dp(g) if grad else None, ctypes.byref(nb)))
        return out.value, (g[: self.n_params] if grad else None), nb.value

    def nll_ex(self, top, theta, cols, weights=None):
        """(nll, grad, gabs, n_bad); gabs[k] = sum_i |d(-log p_i)/d theta_k|.
        weights: per-event w_i (NLL = -sum_i w_i log p_i), or None."""
        th = _f64(theta)
        cs, arr, n = self._cols(cols)
        out = ctypes.c_double()
        g = np.zeros(max(1, self.n_params))
        ga = np.zeros(max(1, self.n_params))
        nb = ctypes.c_int64()
        if weights is None:
            _check(lib().rfo_nll_ex(self.h, top, _dp(th), arr, n, ctypes.byref(out), _dp(g), _dp(ga),
                                    ctypes.byref(nb)))
        else:
            w = _f64(weights)
            assert w.size == n
            _check(lib().rfo_nll_w(self.h, top, _dp(th), arr, _dp(w), n, ctypes.byref(out), _dp(g), _dp(ga),
                                   ctypes.byref(nb)))
        return out.value, g[: self.n_params], ga[: self.n_params], nb.value

    def nll_hess(self, top, theta, cols, weights=None):
        """(nll, grad, hess[P, P], n_bad): the NLL with its gradient and Hessian."""
        th = _f64(theta)
        cs, arr, n = self._cols(cols)
        out = ctypes.c_double()
        P = self.n_params
        g = np.zeros(max(1, P))
        h = np.zeros(max(1, P * P))
        nb = ctypes.c_int64()
        w = None if weights is None else _f64(weights)
        _check(lib().rfo_nll_hess(self.h, top, _dp(th), arr, None if w is None else _dp(w), n, ctypes.byref(out),
                                  _dp(g), _dp(h), ctypes.byref(nb)))
        return out.value, g[:P], h[: P * P].reshape(P, P), nb.value

    def values(self, top, theta, cols):
        th = _f64(theta)
        cs, arr, n = self._cols(cols)
        out = np.empty(n)
        _check(lib().rfo_values(self.h, top, _dp(th), arr, n, _dp(out)))
        return out

    def norm(self, node, theta):
        th = _f64(theta)
        N = ctypes.c_double()
        dN = np.zeros(max(1, self.n_params))
        _check(lib().rfo_norm(self.h, node, _dp(th), ctypes.byref(N), _dp(dN)))
        return N.value, dN[: self.n_params]


def gauss_legendre(K, lo, hi):
    x = np.empty(K)
    w = np.empty(K)
    _check(lib().rfo_gauss_legendre(K, lo, hi, _dp(x), _dp(w)))
    return x, w


def mlp_forward(w, inp):
    w, inp = _f64(w), _f64(inp)
    n = inp.shape[0]
    out = np.empty(n)
    lib().rfo_mlp_forward(_dp(w), _dp(inp), n, _dp(out))
    return out


def mlp_backward(w, inp, dout):
    """Returns (dL/dw summed over rows, dL/dinput per row) for cotangents dout."""
    w, inp, dout = _f64(w), _f64(inp), _f64(dout)
    n = inp.shape[0]
    dw = np.zeros(8833)
    din = np.empty((n, 6))
    lib().rfo_mlp_backward(_dp(w), _dp(inp), n, _dp(dout), _dp(dw), _dp(din))
    return dw, din


def binned_nll(T, Lp, Lm, nobs, theta, grad=True):
    """T[C,S,B], Lp/Lm[C,S,J,B], nobs[C,B], theta=(mu, alpha_1..alpha_J)."""
    T, Lp, Lm, nobs, th = _f64(T), _f64(Lp), _f64(Lm), _f64(nobs), _f64(theta)
    C, S, B = T.shape
    J = Lp.shape[2]
    assert th.size == J + 1
    out = ctypes.c_double()
    g = np.zeros(J + 1)
    lib().rfo_binned_nll(C, S, B, J, _dp(T), _dp(Lp), _dp(Lm), _dp(nobs), _dp(th),
                         ctypes.byref(out), _dp(g) if grad else None)
    return out.value, (g if grad else None)


def combined_nll(terms, constraints, theta):
    """Combined likelihood of independent terms that share parameters, times
    Gaussian constraint factors (the combined measurements of Section 3):

        NLL(theta) = sum_t NLL_t(theta[map_t]) + sum_c (theta[k_c] - m_c)^2 / (2 w_c^2).

    terms: (f, index_map) pairs; f(theta_t) returns (nll_t, grad_t, scale_t)
    for the term's own parameter vector theta_t = theta[index_map] (scale_t:
    per parameter, the sum of the magnitudes of its gradient terms, for scaled
    error metrics; zeros where a term has none).  constraints: (k, m, w)
    triples.  Returns (nll, grad, scale): each term's gradient entry j is
    added to global parameter index_map[j]."""
    theta = np.asarray(theta, dtype=np.float64)
    nll = 0.0
    grad = np.zeros(theta.size)
    scale = np.zeros(theta.size)
    for f, index_map in terms:
        th_t = np.array([theta[k] for k in index_map])
        n_t, g_t, s_t = f(th_t)
        nll += n_t
        for j, k in enumerate(index_map):
            grad[k] += g_t[j]
            scale[k] += s_t[j]
    for k, m, w in constraints:
        z = (theta[k] - m) / w
        nll += 0.5 * z * z
        grad[k] += z / w
        scale[k] += abs(z / w)
    return nll, grad, scale


def from_spec(spec):
    """Build an oracle Model from a declarative node list.

    spec: sequence of (kind, name, inputs, attrs) with inputs given by name;
    OBS attrs = (lo, hi), PARAM attrs = (lo, hi) (bounds; unused here),
    CONST attrs = (value,).  The last entry is the top PDF.
    Returns (model, top_id, ids_by_name)."""
    m = Model()
    ids = {}
    top = None
    for kind, name, inputs, attrs in spec:
        ins = [ids[i] for i in inputs]
        at = list(attrs)
        if kind == "param":
            at = []
        top = ids[name] = m.node(kind, ins, at)
    return m, top, ids
