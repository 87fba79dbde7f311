"""C-ABI checks that need no GPU: the library loads, exports every function
the public header declares, and the host-side paths (graph validation,
lowering, code generation and the code-object build) behave as documented.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfgpu.h")
LIB = os.path.join(ROOT, "paper_2003_12861_amd", "librfgpu.so")

RF_OK, RF_E_INVALID, RF_E_DOMAIN, RF_E_STATE = 0, -1, -2, -6
RF_FP64, RF_FP32 = 0, 1
RF_COMPILE_NO_LOAD = 1


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)  # drop comments
    names = re.findall(r"\b(rf_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def _consts():
    text = open(HEADER).read()
    return {k: int(v) for k, v in re.findall(r"\b(RF_OP_[A-Z0-9_]+)\s*=\s*(\d+)", text)}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librfgpu.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    PI = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "rf_last_error": ([], ctypes.c_char_p),
        "rf_version": ([], ctypes.c_char_p),
        "rf_graph_new": ([ctypes.POINTER(P)], I32),
        "rf_graph_free": ([P], None),
        "rf_graph_observable": ([P, ctypes.c_char_p, D, D, PI], I32),
        "rf_graph_parameter": ([P, ctypes.c_char_p, D, D, PI], I32),
        "rf_graph_constant": ([P, D, PI], I32),
        "rf_graph_node": ([P, I32, PI, I32, ctypes.POINTER(D), I32, PI], I32),
        "rf_compile": ([P, I32, I32, ctypes.c_uint32, ctypes.POINTER(P)], I32),
        "rf_program_free": ([P], None),
        "rf_program_info": ([P, PI, PI, PI], I32),
        "rf_program_source": ([P], ctypes.c_char_p),
        "rf_nll_grad": ([P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64), P], I32),
        "rf_gauss_legendre": ([I32, D, D, ctypes.POINTER(D), ctypes.POINTER(D)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


def test_every_declared_function_is_exported(lib):
    names = _declared()
    assert len(names) >= 30, names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version(lib):
    assert lib.rf_version().decode().startswith("rfgpu-")


class G:
    """Tiny graph builder over the raw C calls."""

    def __init__(self, lib):
        self.lib = lib
        self.h = ctypes.c_void_p()
        assert lib.rf_graph_new(ctypes.byref(self.h)) == RF_OK

    def obs(self, name, lo, hi):
        i = ctypes.c_int32()
        assert self.lib.rf_graph_observable(self.h, name.encode(), lo, hi, ctypes.byref(i)) == RF_OK
        return i.value

    def par(self, name, lo, hi):
        i = ctypes.c_int32()
        assert self.lib.rf_graph_parameter(self.h, name.encode(), lo, hi, ctypes.byref(i)) == RF_OK
        return i.value

    def const(self, v):
        i = ctypes.c_int32()
        assert self.lib.rf_graph_constant(self.h, v, ctypes.byref(i)) == RF_OK
        return i.value

    def node(self, op, name, inputs, attrs=()):
        i = ctypes.c_int32()
        ins = (ctypes.c_int32 * max(1, len(inputs)))(*inputs)
        at = (ctypes.c_double * max(1, len(attrs)))(*attrs)
        rc = self.lib.rf_graph_node(self.h, op, ins, len(inputs), at, len(attrs), ctypes.byref(i))
        return rc, i.value

    def free(self):
        self.lib.rf_graph_free(self.h)


def test_graph_validation_errors(lib):
    op = _consts()
    g = G(lib)
    x = g.obs("x", -10.0, 10.0)
    mu, s = g.par("mu", -5.0, 5.0), g.par("sigma", 0.1, 5.0)
    rc, _ = g.node(op["RF_OP_GAUSS"], "g", [x, mu])  # missing sigma
    assert rc == RF_E_INVALID
    assert b"wrong number of inputs" in lib.rf_last_error()
    rc, _ = g.node(op["RF_OP_GAUSS"], "g", [mu, x, s])  # observable must come first
    assert rc == RF_E_INVALID
    rc, _ = g.node(9999, "bad", [x])
    assert rc == RF_E_INVALID
    rc, gid = g.node(op["RF_OP_GAUSS"], "g", [x, mu, s])
    assert rc == RF_OK
    c1 = g.par("c1", -1.0, 1.0)
    rc, cid = g.node(op["RF_OP_CHEB"], "c", [x, c1])
    assert rc == RF_OK
    g.par("f", 0.0, 1.0)
    rc, add = g.node(op["RF_OP_ADD_PDF"], "m", [gid, cid])  # fraction missing: found when lowering
    assert rc == RF_OK
    rc, p = _compile(lib, g, add, RF_FP64)
    assert rc == RF_E_INVALID
    assert b"sum: inputs" in lib.rf_last_error()
    g.free()


def _compile(lib, g, top, prec, flags=RF_COMPILE_NO_LOAD):
    p = ctypes.c_void_p()
    rc = lib.rf_compile(g.h, top, prec, flags, ctypes.byref(p))
    return rc, p


def test_shared_pdf_node_is_expanded(lib):
    """A PDF node feeding two sums (here also nested: one use sits inside the
    other sum's first component) compiles to the program of the tree in
    which the node is written once per use."""
    op = _consts()
    info = []
    for shared in (True, False):
        g = G(lib)
        x = g.obs("x", -10.0, 10.0)
        mu, s, f1, f2 = g.par("mu", -5, 5), g.par("s", 0.1, 5), g.par("f1", 0, 1), g.par("f2", 0, 1)
        c1 = g.par("c1", -1, 1)
        _, gs = g.node(op["RF_OP_GAUSS"], "g", [x, mu, s])
        _, cb = g.node(op["RF_OP_CHEB"], "c", [x, c1])
        _, m1 = g.node(op["RF_OP_ADD_PDF"], "m1", [gs, cb, f1])
        g2 = gs if shared else g.node(op["RF_OP_GAUSS"], "g2", [x, mu, s])[1]
        _, m2 = g.node(op["RF_OP_ADD_PDF"], "m2", [m1, g2, f2])  # g feeds two sums
        for prec in (RF_FP64, RF_FP32):
            rc, p = _compile(lib, g, m2, prec)
            assert rc == RF_OK, lib.rf_last_error()
            npar, ncol, nsum = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            assert lib.rf_program_info(p, ctypes.byref(npar), ctypes.byref(ncol), ctypes.byref(nsum)) == RF_OK
            info.append((prec, npar.value, ncol.value, nsum.value))
            lib.rf_program_free(p)
        g.free()
    assert info[:2] == info[2:], info


@pytest.mark.parametrize("prec", [RF_FP64, RF_FP32])
def test_codegen_and_build_without_gpu(lib, prec):
    """Lowering, code generation and the gfx950 code-object build run on the
    host; the generated program has the documented entry points and sums."""
    op = _consts()
    g = G(lib)
    x = g.obs("x", -10.0, 10.0)
    mu, s, f = g.par("mu", -5, 5), g.par("sigma", 0.05, 10), g.par("f", 0, 1)
    c1, c2 = g.par("c1", -1, 1), g.par("c2", -1, 1)
    _, gs = g.node(op["RF_OP_GAUSS"], "sig", [x, mu, s])
    _, cb = g.node(op["RF_OP_CHEB"], "bkg", [x, c1, c2])
    _, m = g.node(op["RF_OP_ADD_PDF"], "model", [gs, cb, f])
    rc, p = _compile(lib, g, m, prec)
    assert rc == RF_OK, lib.rf_last_error()
    npar, ncol, nsum = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.rf_program_info(p, ctypes.byref(npar), ctypes.byref(ncol), ctypes.byref(nsum)) == RF_OK
    # theta = (mu, sigma, f, c1, c2); sums: log p, D(mu), D(sigma), D(c1), D(c2), Y(sig), Y(bkg)
    assert (npar.value, ncol.value, nsum.value) == (5, 1, 7)
    src = lib.rf_program_source(p).decode()
    for k in ("rf_k_values_", "rf_k_nll_", "rf_k_grad_", "rf_epilogue", "RF_PREC"):
        assert k in src
    assert ("#define RF_T float" in src) == (prec == RF_FP32)
    # a program compiled without loading cannot evaluate
    th = (ctypes.c_double * 5)(0, 1, 0.3, 0.2, -0.1)
    nll, g5, nb = ctypes.c_double(), (ctypes.c_double * 5)(), ctypes.c_int64()
    assert lib.rf_nll_grad(p, th, ctypes.byref(nll), g5, ctypes.byref(nb), None) == RF_E_STATE
    # the fit's initial inverse Hessian is checked before anything runs: a
    # non-positive or NaN diagonal entry or an infinite entry is refused; a
    # good one gets as far as the first evaluation (not loaded: RF_E_STATE)
    fit = lib.rf_fit_bfgs_ex
    DP = ctypes.POINTER(ctypes.c_double)
    fit.argtypes = [ctypes.c_void_p, DP, DP, ctypes.c_double, ctypes.c_int32, DP, DP, DP, DP, ctypes.c_void_p]
    fit.restype = ctypes.c_int32
    out, sig, info = (ctypes.c_double * 5)(), (ctypes.c_double * 5)(), (ctypes.c_double * 4)()
    cov = (ctypes.c_double * 25)()
    for i, j, v, rc in ((2, 2, -1.0, RF_E_INVALID), (0, 0, float("nan"), RF_E_INVALID),
                        (1, 3, float("inf"), RF_E_INVALID), (1, 3, 0.5, RF_E_STATE)):
        h0 = (ctypes.c_double * 25)(*[1.0 if a == b else 0.0 for a in range(5) for b in range(5)])
        h0[5 * i + j] = v
        assert fit(p, th, h0, 1e-6, 10, out, sig, cov, info, None) == rc, (i, j, v)
        if rc == RF_E_INVALID:
            assert b"hinv0" in lib.rf_last_error()
    lib.rf_program_free(p)
    g.free()


def test_host_gauss_legendre(lib):
    x, w = (ctypes.c_double * 5)(), (ctypes.c_double * 5)()
    assert lib.rf_gauss_legendre(5, -1.0, 1.0, x, w) == RF_OK
    assert abs(sum(w) - 2.0) < 1e-14
    # exact for x^8 on [-1, 1]: 2/9
    assert abs(sum(wi * xi ** 8 for xi, wi in zip(x, w)) - 2.0 / 9.0) < 1e-14
    assert lib.rf_gauss_legendre(0, -1.0, 1.0, x, w) == RF_E_INVALID


def test_poisson_range_checks(lib):
    """The Poisson leaf needs an observable range with integer ends,
    0 <= lo < hi and at most 2048 values; a good one compiles on the host."""
    op = _consts()
    for lo, hi, ok in [(0.0, 40.0, True), (0.5, 40.0, False), (-1.0, 40.0, False), (0.0, 2047.0, True),
                       (0.0, 2048.0, False), (2.0, 7.5, False)]:
        g = G(lib)
        n = g.obs("n", lo, hi)
        lam = g.par("lam", 0.1, 100.0)
        rc, p = g.node(op["RF_OP_POISSON"], "p", [n, lam])
        if rc == RF_OK:
            rc, prog = _compile(lib, g, p, RF_FP64)
        assert (rc == RF_OK) == ok, (lo, hi, rc, lib.rf_last_error())
        if rc == RF_OK:
            assert "poisson_prologue" in lib.rf_program_source(prog).decode()
            lib.rf_program_free(prog)
        else:
            assert b"poisson" in lib.rf_last_error()
        g.free()


def test_weighted_extended_adds_a_sum(lib):
    """A weighted extended program accumulates the sum of the weights as one
    more event sum; the extended term reads it in place of the event count."""
    op = _consts()
    res = {}
    for flags in (RF_COMPILE_NO_LOAD, RF_COMPILE_NO_LOAD | 4):  # 4: RF_COMPILE_WEIGHTED
        g = G(lib)
        x = g.obs("x", -10.0, 10.0)
        mu, s, nu = g.par("mu", -5, 5), g.par("sigma", 0.05, 10), g.par("nu", 0, 1e9)
        _, gs = g.node(op["RF_OP_GAUSS"], "sig", [x, mu, s])
        _, e = g.node(op["RF_OP_EXTENDED"], "model", [gs, nu])
        rc, p = _compile(lib, g, e, RF_FP64, flags)
        assert rc == RF_OK, lib.rf_last_error()
        npar, ncol, nsum = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.rf_program_info(p, ctypes.byref(npar), ctypes.byref(ncol), ctypes.byref(nsum)) == RF_OK
        res[flags] = (ncol.value, nsum.value, lib.rf_program_source(p).decode())
        lib.rf_program_free(p)
        g.free()
    (c0, s0, src0), (c1, s1, src1) = res.values()
    assert (c1, s1) == (c0 + 1, s0 + 1)
    assert "ext_n = th[3]" in src0 and ("ext_n = (MODE == 2 ? S[%d]" % s0) in src1
