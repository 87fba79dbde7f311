"""Thin Python binding of librfgpu (argument marshalling only).

Every computation runs in the C library and its GPU kernels; this module
converts arguments, keeps bound tensors alive and maps status codes to
exceptions.  torch is imported first so that the library shares torch's HIP
runtime, devices and streams.  If the library is missing, importing this
module fails: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfgpu.so")

FP64, FP32 = 0, 1
RF_COMPILE_NO_LOAD, RF_VALIDATE, RF_COMPILE_WEIGHTED = 1, 2, 4
OPS = {
    "gauss": 1, "cheb": 2, "exp": 3, "decay_gauss": 4, "argus": 5, "bw": 6,
    "numconv_bw_cb": 7, "mlp": 8, "poisson": 9, "add": 20, "prod": 21, "extended": 22, "linear": 40, "product": 41, "ratio": 42,
}
STATUS = {0: "RF_OK", -1: "RF_E_INVALID", -2: "RF_E_DOMAIN", -3: "RF_E_NONFINITE",
          -4: "RF_E_DEVICE", -5: "RF_E_OOM", -6: "RF_E_STATE"}

if not os.path.exists(LIB_PATH):
    raise ImportError("librfgpu.so is not built: run `python -m paper_2003_12861_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

_P, _I32, _I64, _D, _U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
_DP = ctypes.POINTER(ctypes.c_double)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PP = ctypes.POINTER(ctypes.c_void_p)
_F = ctypes.c_float

_SIGS = {
    "rf_last_error": ([], ctypes.c_char_p),
    "rf_version": ([], ctypes.c_char_p),
    "rf_graph_new": ([_PP], _I32),
    "rf_graph_free": ([_P], None),
    "rf_graph_observable": ([_P, ctypes.c_char_p, _D, _D, _PI32], _I32),
    "rf_graph_parameter": ([_P, ctypes.c_char_p, _D, _D, _PI32], _I32),
    "rf_graph_constant": ([_P, _D, _PI32], _I32),
    "rf_graph_node": ([_P, _I32, _PI32, _I32, _DP, _I32, _PI32], _I32),
    "rf_compile": ([_P, _I32, _I32, _U32, _PP], _I32),
    "rf_program_free": ([_P], None),
    "rf_program_info": ([_P, _PI32, _PI32, _PI32], _I32),
    "rf_program_source": ([_P], ctypes.c_char_p),
    "rf_program_stats": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I32),
    "rf_bind_columns": ([_P, _PP, _I32, _I64, _P], _I32),
    "rf_bind_columns_strided": ([_P, _PP, _PI64, _PI32, _I32, _I64, _P], _I32),
    "rf_bind_weights": ([_P, _I32, _P, _P], _I32),
    "rf_set_launch": ([_P, _I32, _I32], _I32),
    "rf_eval_values": ([_P, _DP, _P, _P], _I32),
    "rf_nll": ([_P, _DP, _DP, _PI64, _P], _I32),
    "rf_nll_grad": ([_P, _DP, _DP, _DP, _PI64, _P], _I32),
    "rf_nll_grad_async": ([_P, _DP, _P], _I32),
    "rf_program_result": ([_P], _P),
    "rf_fit_bfgs": ([_P, _DP, _D, _I32, _DP, _DP, _DP, _P], _I32),
    "rf_fit_bfgs_ex": ([_P, _DP, _DP, _D, _I32, _DP, _DP, _DP, _DP, _P], _I32),
    "rf_gauss_legendre": ([_I32, _D, _D, _DP, _DP], _I32),
    "rf_sum_new": ([_I32, _DP, _DP, _PP], _I32),
    "rf_sum_free": ([_P], None),
    "rf_sum_add_program": ([_P, _P, _PI32], _I32),
    "rf_sum_add_binned": ([_P, _P, _PI32], _I32),
    "rf_sum_add_constraint": ([_P, _I32, _D, _D], _I32),
    "rf_sum_nll_grad": ([_P, _DP, _DP, _DP, _PI64, _P], _I32),
    "rf_sum_fit_bfgs": ([_P, _DP, _D, _I32, _DP, _DP, _DP, _DP, _P], _I32),
}
_OPTIONAL = {
    "rf_binned_new": ([_I32, _I32, _I32, _I32, _DP, _DP, _DP, _DP, _P, _PP], _I32),
    "rf_binned_free": ([_P], None),
    "rf_binned_nll_grad": ([_P, _DP, _DP, _DP, _P], _I32),
    "rf_binned_nll_grad_async": ([_P, _DP, _P], _I32),
    "rf_binned_result": ([_P], _P),
    "rf_mlp_forward": ([_P, _P, _I64, _P, _P, _P], _I32),
    "rf_mlp_backward": ([_P, _P, _P, _P, _I64, _P, _P, _P], _I32),
    "rf_adam_step": ([_P, _P, _P, _P, _P, _I64, _F, _F, _F, _F, _I32, _P], _I32),
    "rf_mse_grad": ([_P, _P, _I64, _F, _P, _P], _I32),
    "rf_mlp_train_step": ([_P, _P, _P, _P, _P, _P, _P, _I64, _I64, _U32, _F, _F, _F, _F, _I32, _P, _P], _I32),
    "rf_nll_unfused": ([_P, _P, _P, _P, _P], _I32),
    "rf_unfused_build": ([_P], _I32),
    "rf_bwcb_logpdf": ([_P, _I64, _I32, _D, _D, _D, _D, _P, _P], _I32),
    "rf_mlp_targets": ([_P, _I64, _I32, _D, _D, _D, _D, _P, _P], _I32),
    "rf_peak": ([_I32, _I32, _I64, _DP, _DP], _I32),
    "rf_eval_math": ([_I32, _P, _I64, _P, _P], _I32),
    "rf_nll_grad_noalloc": ([_P, _DP, _P, _P], _I32),
    "rf_nll_grad_hess": ([_P, _DP, _DP, _DP, _DP, _PI64, _P], _I32),
    "rf_hess_build": ([_P], _I32),
}


def _bind(table, required):
    for name, (args, res) in table.items():
        fn = getattr(_lib, name, None)
        if fn is None:
            if required:
                raise ImportError("librfgpu.so lacks " + name)
            continue
        fn.argtypes = args
        fn.restype = res
        globals()[name] = fn


_bind(_SIGS, True)
_bind(_OPTIONAL, False)

# the synchronous calls through the CPython module (same library instance:
# it calls the addresses ctypes resolved above)
try:
    from . import _rfcall
except ImportError as e:
    raise ImportError("the _rfcall module is not built: run `python -m paper_2003_12861_amd.build`") from e
_rfcall.init(*[ctypes.cast(f, ctypes.c_void_p).value for f in (rf_nll_grad, rf_binned_nll_grad, rf_sum_nll_grad)])


class RfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


def check(rc):
    if rc < 0:
        raise RfError(rc, rf_last_error().decode(errors="replace"))
    return rc


def _dptr(a):
    return a.ctypes.data_as(_DP)


_last_stream = [None, 0]  # the last torch stream object resolved, and its handle


def _stream(stream=None):
    """hipStream_t as an integer: torch's current stream, a torch stream, or a raw handle."""
    if type(stream) is int:
        return stream
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if stream is _last_stream[0]:  # held here, so the object (and its handle) is still alive
        return _last_stream[1]
    if isinstance(stream, torch.cuda.Stream):
        _last_stream[0], _last_stream[1] = stream, stream.cuda_stream
        return _last_stream[1]
    return int(stream) if stream else 0


def gauss_legendre(K, lo, hi):
    x, w = np.empty(K), np.empty(K)
    check(rf_gauss_legendre(K, lo, hi, _dptr(x), _dptr(w)))
    return x, w


# --------------------------------------------------------------------- graph
class Graph:
    """A model graph: observables, parameters, constants, functions and PDFs."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(rf_graph_new(ctypes.byref(h)))
        self.h = h
        self.ids = {}
        self.top = None
        self.param_names = []
        self.obs_names = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            try:
                rf_graph_free(h)
            except Exception:  # interpreter shutdown: the library may be gone
                pass

    def _id(self, name, rc, out):
        check(rc)
        self.ids[name] = out.value
        self.top = out.value
        return out.value

    def observable(self, name, lo, hi):
        out = ctypes.c_int32()
        self.obs_names.append(name)
        return self._id(name, rf_graph_observable(self.h, name.encode(), lo, hi, ctypes.byref(out)), out)

    def parameter(self, name, lo, hi):
        out = ctypes.c_int32()
        self.param_names.append(name)
        return self._id(name, rf_graph_parameter(self.h, name.encode(), lo, hi, ctypes.byref(out)), out)

    def constant(self, value, name=None):
        out = ctypes.c_int32()
        return self._id(name or "const%d" % len(self.ids), rf_graph_constant(self.h, value, ctypes.byref(out)), out)

    def node(self, op, inputs, attrs=(), name=None):
        ins = [self.ids[i] if isinstance(i, str) else int(i) for i in inputs]
        iarr = (ctypes.c_int32 * max(1, len(ins)))(*ins)
        at = np.ascontiguousarray(list(attrs) if len(attrs) else [0.0], dtype=np.float64)
        out = ctypes.c_int32()
        opc = OPS[op] if isinstance(op, str) else int(op)
        return self._id(name or "n%d" % len(self.ids),
                        rf_graph_node(self.h, opc, iarr, len(ins), _dptr(at), len(attrs), ctypes.byref(out)), out)

    @classmethod
    def from_spec(cls, spec):
        """spec: sequence of (kind, name, inputs, attrs); the last entry is the top PDF."""
        g = cls()
        for kind, name, inputs, attrs in spec:
            if kind == "obs":
                g.observable(name, attrs[0], attrs[1])
            elif kind == "param":
                g.parameter(name, attrs[0], attrs[1])
            elif kind == "const":
                g.constant(attrs[0], name)
            else:
                g.node(kind, inputs, attrs, name)
        return g


# -------------------------------------------------------------------- program
class Program:
    """A compiled graph: one fused kernel per precision form."""

    def __init__(self, graph, top=None, precision=FP64, load=True, flags=0, weighted=False, validate=False):
        """weighted: bind() takes one more column, the per-event weights
        (NLL = -sum w_i log p_i); validate: bind() checks the columns."""
        h = ctypes.c_void_p()
        top = graph.top if top is None else (graph.ids[top] if isinstance(top, str) else top)
        fl = flags | (0 if load else RF_COMPILE_NO_LOAD) | (RF_COMPILE_WEIGHTED if weighted else 0)
        fl |= RF_VALIDATE if validate else 0
        check(rf_compile(graph.h, top, precision, fl, ctypes.byref(h)))
        self.h = h
        self.precision = precision
        self.param_names = list(graph.param_names)
        self.ids = dict(graph.ids)
        npar, ncol, nsum = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(rf_program_info(h, ctypes.byref(npar), ctypes.byref(ncol), ctypes.byref(nsum)))
        self.n_params, self.n_columns, self.n_sums = npar.value, ncol.value, nsum.value
        self._cols = []
        self._weights = None
        self.n_events = None
        # argument and result buffers reused by every call (no allocation or
        # pointer conversion per evaluation)
        self._v, self._nb = ctypes.c_double(), ctypes.c_int64()
        self._vref, self._nbref = ctypes.byref(self._v), ctypes.byref(self._nb)
        self._g = np.zeros(max(1, self.n_params))
        self._gptr = _dptr(self._g)
        self._gview = self._g[: self.n_params]
        self._th = np.zeros(max(1, self.n_params))
        self._thptr = _dptr(self._th)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            try:
                rf_program_free(h)
            except Exception:  # interpreter shutdown: the library may be gone
                pass

    @property
    def source(self):
        return rf_program_source(self.h).decode()

    @property
    def dtype(self):
        return torch.float32 if self.precision == FP32 else torch.float64

    def bind(self, cols, stream=None):
        """cols: device tensors (one per observable, then the event weights for a
        weighted program), float32 or float64.  Columns in the program's dtype
        with unit stride are bound in place; 1-D columns with another stride or
        dtype are copied by the library into contiguous arrays of the
        program's dtype (rf_bind_columns_strided)."""
        cols = [c if c.dim() == 1 and c.stride(0) >= 1 else c.contiguous().reshape(-1) for c in cols]
        for c in cols:
            if c.dtype not in (torch.float32, torch.float64) or not c.is_cuda:
                raise RfError(-1, "columns must be float32 or float64 tensors on the GPU")
        n = int(cols[0].numel()) if cols else 0
        if any(int(c.numel()) != n for c in cols):
            raise RfError(-1, "columns differ in length")
        arr = (ctypes.c_void_p * max(1, len(cols)))(*[c.data_ptr() for c in cols])
        if all(c.dtype == self.dtype and (c.stride(0) == 1 or n <= 1) for c in cols):
            check(rf_bind_columns(self.h, arr, len(cols), n, _stream(stream)))
        else:
            strides = (ctypes.c_int64 * max(1, len(cols)))(*[c.stride(0) for c in cols])
            dts = (ctypes.c_int32 * max(1, len(cols)))(*[0 if c.dtype == torch.float32 else 1 for c in cols])
            check(rf_bind_columns_strided(self.h, arr, strides, dts, len(cols), n, _stream(stream)))
        self._cols = cols
        self.n_events = n
        return self

    def bind_weights(self, node, w_bf16, stream=None):
        nid = self.ids[node] if isinstance(node, str) else int(node)
        if w_bf16.dtype != torch.bfloat16 or w_bf16.numel() != 8833 or not w_bf16.is_cuda:
            raise RfError(-1, "weights must be 8833 bf16 values on the GPU")
        w = w_bf16.contiguous()
        check(rf_bind_weights(self.h, nid, ctypes.c_void_p(w.data_ptr()), _stream(stream)))
        self._weights = w

    def set_launch(self, blocks=0, threads=0):
        check(rf_set_launch(self.h, blocks, threads))

    def _theta(self, theta):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        if th.size != self.n_params:
            raise RfError(-1, "theta has %d values, the program %d parameters" % (th.size, self.n_params))
        return th

    def _theta_ptr(self, theta):
        """theta copied into the program's argument buffer; returns its pointer"""
        if len(theta) != self.n_params:
            raise RfError(-1, "theta has %d values, the program %d parameters" % (len(theta), self.n_params))
        self._th[: self.n_params] = theta
        return self._thptr

    def values(self, theta, out=None, stream=None):
        th = self._theta(theta)
        if out is None:
            out = torch.empty(self.n_events, dtype=self.dtype, device=self._cols[0].device if self._cols else "cuda")
        check(rf_eval_values(self.h, _dptr(th), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def nll(self, theta, stream=None):
        rc = rf_nll(self.h, self._theta_ptr(theta), self._vref, self._nbref, _stream(stream))
        if rc != -3:
            check(rc)
        return self._v.value, self._nb.value

    def build_unfused(self):
        """Build the unfused mode's code object (no GPU needed)."""
        check(rf_unfused_build(self.h))

    def nll_unfused(self, theta, stream=None):
        """The NLL by the unfused per-node batch mode (an ablation of the fused
        kernel): (nll, n_bad)."""
        rc = rf_nll_unfused(self.h, self._theta_ptr(theta), self._vref, self._nbref, _stream(stream))
        if rc != -3:
            check(rc)
        return self._v.value, self._nb.value

    def nll_grad(self, theta, stream=None):
        """Returns (nll, grad, n_bad); nll = inf and grad = nan when n_bad > 0."""
        r = _rfcall.nll_grad(self.h.value, theta, self.n_params, stream if type(stream) is int else _stream(stream))
        if r is not None:
            if r[0] != 0 and r[0] != -3:
                check(r[0])
            return r[1], r[2], r[3]
        # theta is not n_params numbers: the checked path raises the error
        rc = rf_nll_grad(self.h, self._theta_ptr(theta), self._vref, self._gptr, self._nbref, _stream(stream))
        if rc != -3:
            check(rc)
        return self._v.value, self._gview.copy(), self._nb.value

    def nll_grad_async(self, theta, stream=None):
        check(rf_nll_grad_async(self.h, self._theta_ptr(theta), _stream(stream)))

    def nll_grad_hess(self, theta, stream=None):
        """Returns (nll, grad, hess[P, P], n_bad) from the Hessian kernel."""
        P = self.n_params
        h = np.zeros(max(1, P * P))
        g = np.zeros(max(1, P))
        rc = rf_nll_grad_hess(self.h, self._theta_ptr(theta), self._vref, _dptr(g), _dptr(h), self._nbref,
                              _stream(stream))
        if rc != -3:
            check(rc)
        return self._v.value, g[:P].copy(), h[: P * P].reshape(P, P).copy(), self._nb.value

    def build_hess(self):
        """Build the Hessian kernel's code object (no GPU needed)."""
        check(rf_hess_build(self.h))

    def nll_grad_noalloc(self, theta, out, stream=None):
        """Enqueue one NLL+gradient evaluation that allocates nothing: the
        result block [nll, grad, n_bad, sums] goes to out (float64 device
        tensor of n_params + 2 + n_sums values); asynchronous."""
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < self.n_params + 2 + self.n_sums:
            raise RfError(-1, "out must be a float64 device tensor of n_params + 2 + n_sums values")
        check(rf_nll_grad_noalloc(self.h, self._theta_ptr(theta), ctypes.c_void_p(out.data_ptr()), _stream(stream)))

    def stats(self):
        """(synchronous calls, calls whose wait fell back to a stream sync)"""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(rf_program_stats(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def result_ptr(self):
        return rf_program_result(self.h)

    def fit(self, theta0, edm_tol=1e-6, max_iter=1000, stream=None):
        th = self._theta(theta0)
        out = np.zeros(self.n_params)
        sig = np.zeros(self.n_params)
        info = np.zeros(4)
        check(rf_fit_bfgs(self.h, _dptr(th), edm_tol, max_iter, _dptr(out), _dptr(sig), _dptr(info), _stream(stream)))
        return out, sig, dict(iterations=int(info[0]), evaluations=int(info[1]), edm=float(info[2]),
                              converged=bool(info[3]))

    def fit_ex(self, theta0, hinv0=None, edm_tol=1e-6, max_iter=1000, uncertainties=True, stream=None):
        """fit() with an optional initial inverse Hessian (P x P).  Returns
        (theta, sigma, cov, info); with uncertainties=False no Hessian is
        formed at the minimum and sigma and cov are None."""
        th = self._theta(theta0)
        P = self.n_params
        h0 = None if hinv0 is None else np.ascontiguousarray(np.asarray(hinv0, dtype=np.float64).reshape(P, P))
        out, info = np.zeros(P), np.zeros(4)
        sig, cov = (np.zeros(P), np.zeros((P, P))) if uncertainties else (None, None)
        check(rf_fit_bfgs_ex(self.h, _dptr(th), None if h0 is None else _dptr(h0), edm_tol, max_iter, _dptr(out),
                             None if sig is None else _dptr(sig), None if cov is None else _dptr(cov), _dptr(info),
                             _stream(stream)))
        return out, sig, cov, dict(iterations=int(info[0]), evaluations=int(info[1]), edm=float(info[2]),
                                   converged=bool(info[3]))


def compile_program(graph, top=None, precision=FP64, load=True, flags=0, weighted=False, validate=False):
    return Program(graph, top, precision, load, flags, weighted, validate)


class NLLFunction(torch.autograd.Function):
    """NLL(theta) with the hand-written GPU adjoint as its backward.

    forward(theta: float64 tensor [P], program) -> scalar float64 tensor; the
    kernel computes NLL and dNLL/dtheta in one pass, backward scales the
    stored gradient.  Double backward is not supported."""

    @staticmethod
    def forward(ctx, theta, program):
        nll, g, nbad = program.nll_grad(theta.detach().to("cpu", torch.float64).numpy())
        ctx.save_for_backward(torch.from_numpy(g).to(theta.device, theta.dtype))
        return torch.tensor(nll, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout * g, None


class Binned:
    """Binned template likelihood (channels x samples x bins, J nuisances + signal strength)."""

    def __init__(self, T, Tp, Tm, nobs, stream=None):
        T = np.ascontiguousarray(T, dtype=np.float64)
        C, S, B = T.shape
        J = 0 if Tp is None else int(np.asarray(Tp).shape[2])
        Tp = np.ascontiguousarray(Tp if J else np.ones((C, S, 0, B)), dtype=np.float64)
        Tm = np.ascontiguousarray(Tm if J else np.ones((C, S, 0, B)), dtype=np.float64)
        nobs = np.ascontiguousarray(nobs, dtype=np.float64)
        h = ctypes.c_void_p()
        check(rf_binned_new(C, S, B, J, _dptr(T), _dptr(Tp), _dptr(Tm), _dptr(nobs), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.shape = (C, S, B, J)
        self.n_params = J + 1

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            try:
                rf_binned_free(h)
            except Exception:  # interpreter shutdown: the library may be gone
                pass

    def nll_grad(self, theta, stream=None):
        r = _rfcall.binned_nll_grad(self.h.value, theta, self.n_params, stream if type(stream) is int else _stream(stream))
        if r is not None:
            check(r[0])
            return r[1], r[2]
        # theta is not n_params numbers: the checked path raises the error
        if type(theta) is np.ndarray and theta.dtype == np.float64 and theta.ndim == 1 and theta.flags.c_contiguous:
            th = theta
        else:
            th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        if th.size != self.n_params:
            raise RfError(-1, "theta needs %d values" % self.n_params)
        if not hasattr(self, "_g"):  # result buffers reused by every call
            self._v, self._g = ctypes.c_double(), np.zeros(self.n_params)
            self._vref, self._gptr = ctypes.byref(self._v), _dptr(self._g)
        check(rf_binned_nll_grad(self.h, _dptr(th), self._vref, self._gptr, _stream(stream)))
        return self._v.value, self._g.copy()

    def nll_grad_async(self, theta, stream=None):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        check(rf_binned_nll_grad_async(self.h, _dptr(th), _stream(stream)))


# ------------------------------------------------------ combined likelihoods --
class Sum:
    """A combined likelihood: terms (Programs with bound columns, Binned models)
    sharing global parameters through index maps, plus Gaussian constraints
    on global parameters.  The terms must outlive the Sum."""

    def __init__(self, n_params, lo=None, hi=None):
        h = ctypes.c_void_p()
        lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        for b in (lo_a, hi_a):
            if b is not None and b.size != n_params:
                raise RfError(-1, "bounds need n_params values")
        check(rf_sum_new(n_params, None if lo_a is None else _dptr(lo_a), None if hi_a is None else _dptr(hi_a),
                         ctypes.byref(h)))
        self.h = h
        self.n_params = n_params
        self._terms = []  # keeps the terms alive as long as the sum
        self._g = np.zeros(n_params)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            try:
                rf_sum_free(h)
            except Exception:  # interpreter shutdown: the library may be gone
                pass

    def add(self, term, index_map):
        """term: a Program or a Binned model; index_map: the global index of each
        of its parameters (Binned: mu, then alpha_1..alpha_J)."""
        m = np.ascontiguousarray(index_map, dtype=np.int32)
        if m.size != term.n_params:
            raise RfError(-1, "the map needs one index per parameter of the term (%d)" % term.n_params)
        mp = m.ctypes.data_as(_PI32)
        if isinstance(term, Binned):
            check(rf_sum_add_binned(self.h, term.h, mp))
        else:
            check(rf_sum_add_program(self.h, term.h, mp))
        self._terms.append(term)
        return self

    def constrain(self, k, mean, width):
        """Gaussian constraint factor on global parameter k."""
        check(rf_sum_add_constraint(self.h, int(k), float(mean), float(width)))
        return self

    def nll_grad(self, theta, stream=None):
        """Returns (nll, grad, n_bad); nll = inf and grad = nan when n_bad > 0."""
        r = _rfcall.sum_nll_grad(self.h.value, theta, self.n_params, stream if type(stream) is int else _stream(stream))
        if r is not None:
            if r[0] != 0 and r[0] != -3:
                check(r[0])
            return r[1], r[2], r[3]
        # theta is not n_params numbers: the checked path raises the error
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        if th.size != self.n_params:
            raise RfError(-1, "theta needs %d values" % self.n_params)
        v, nb = ctypes.c_double(), ctypes.c_int64()
        rc = rf_sum_nll_grad(self.h, _dptr(th), ctypes.byref(v), _dptr(self._g), ctypes.byref(nb), _stream(stream))
        if rc != -3:
            check(rc)
        return v.value, self._g.copy(), nb.value

    def fit(self, theta0, edm_tol=1e-6, max_iter=500, uncertainties=True, stream=None):
        """BFGS on the combined NLL: (theta, sigma, cov, info dict)."""
        P = self.n_params
        t0 = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64).reshape(-1))
        if t0.size != P:
            raise RfError(-1, "theta0 needs %d values" % P)
        th, info = np.zeros(P), np.zeros(4)
        sig, cov = (np.zeros(P), np.zeros((P, P))) if uncertainties else (None, None)
        check(rf_sum_fit_bfgs(self.h, _dptr(t0), edm_tol, max_iter, _dptr(th), None if sig is None else _dptr(sig),
                              None if cov is None else _dptr(cov), _dptr(info), _stream(stream)))
        return th, sig, cov, dict(iterations=int(info[0]), evaluations=int(info[1]), edm=float(info[2]),
                                  converged=bool(info[3]))


# ----------------------------------------------------------- MLP kernels --
def _vp(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def mlp_forward(w_bf16, u, out=None, act=None, stream=None):
    """s = MLP(u) for u (n x 6, FP32 in [-1, 1]) with BF16 weights (8833)."""
    n = u.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=u.device)
    check(rf_mlp_forward(_vp(w_bf16), _vp(u), n, _vp(out), _vp(act), _stream(stream)))
    return out


def mlp_backward(w_bf16, u, dout, dw=None, din=None, stream=None):
    """dw (8833, FP32) = sum over rows of dout * ds/dw; din (n x 6) = dout * ds/du."""
    n = u.shape[0]
    if dw is None:
        dw = torch.empty(8833, dtype=torch.float32, device=u.device)
    check(rf_mlp_backward(_vp(w_bf16), _vp(u), ctypes.c_void_p(0), _vp(dout), n, _vp(dw), _vp(din), _stream(stream)))
    return dw, din


def adam_step(w32, w_bf16, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(rf_adam_step(_vp(w32), _vp(w_bf16), _vp(m), _vp(v), _vp(g), w32.numel(), lr, beta1, beta2, eps, step,
                       _stream(stream)))


def mse_grad(out, target, scale, dout, stream=None):
    check(rf_mse_grad(_vp(out), _vp(target), out.numel(), scale, _vp(dout), _stream(stream)))


def mlp_train_step(w_bf16, w32, m, v, u, target, idx, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, dw=None,
                   stream=None, validate=False):
    """One Adam step on the mean-squared error of MLP(u[idx]) against target[idx]
    (idx: int64 indices of the batch rows, or None for all rows of u);
    validate: check on the host that every index names a row of u."""
    batch = idx.numel() if idx is not None else u.shape[0]
    n_rows = min(u.shape[0], target.shape[0])
    check(rf_mlp_train_step(_vp(w_bf16), _vp(w32), _vp(m), _vp(v), _vp(u), _vp(target), _vp(idx), batch, n_rows,
                            RF_VALIDATE if validate else 0, lr, beta1, beta2, eps, step, _vp(dw), _stream(stream)))


def bwcb_logpdf(xq, K, window, x_range, out=None, stream=None):
    """Exact log p_sig at per-row parameters; xq: (n x 6) FP64 (x, M, Gamma, sigma, alpha, n)."""
    n = xq.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=xq.device)
    check(rf_bwcb_logpdf(_vp(xq), n, K, window[0], window[1], x_range[0], x_range[1], _vp(out), _stream(stream)))
    return out


def mlp_targets(xq, K, window, x_range, out=None, stream=None):
    """Training targets log p_sig - log b (FP32) at rows (x, M, Gamma, sigma, alpha, n) of xq (FP64)."""
    n = xq.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xq.device)
    check(rf_mlp_targets(_vp(xq), n, K, window[0], window[1], x_range[0], x_range[1], _vp(out), _stream(stream)))
    return out


PEAK_KINDS = {0: "fp32_fma", 1: "fp64_fma", 2: "fp32_exp2", 3: "fp32_mix_14fma_1trans", 4: "fp32_mix_12fma_1rcp",
              5: "fp64_exp_call", 6: "fp64_log_call", 7: "fp64_rcp_newton", 8: "stream_read_bytes",
              9: "fp64_log_own_call"}


def peak(kind, iters, stream_bytes=0):
    """(rate, seconds) of microbenchmark kind (see PEAK_KINDS) on the current device."""
    r, t = ctypes.c_double(), ctypes.c_double()
    check(rf_peak(kind, iters, stream_bytes, ctypes.byref(r), ctypes.byref(t)))
    return r.value, t.value


def eval_math(fn, x, out=None, stream=None):
    """The library's device math function fn (0: FP64 log, 1: 2^t for t <= 0) on a float64 device tensor."""
    if out is None:
        out = torch.empty_like(x)
    check(rf_eval_math(fn, _vp(x), x.numel(), _vp(out), _stream(stream)))
    return out
