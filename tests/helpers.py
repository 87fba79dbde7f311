"""Shared test helpers: build the same model in the GPU library and the oracle."""
import numpy as np

from oracle import rfo


def build_pair(spec, precision, api, **kw):
    g = api.Graph.from_spec(spec)
    prog = api.Program(g, precision=precision, **kw)
    om, otop, oids = rfo.from_spec(spec)
    return prog, (om, otop, oids)


def to_dev(cols, precision, api):
    import torch
    dt = torch.float32 if precision == api.FP32 else torch.float64
    return [torch.tensor(np.asarray(c), dtype=dt, device="cuda") for c in cols]


def scaled_grad_err(g, g_ref, gabs):
    """|g - g*| / sum_i |d(-log p_i)/d theta| per component (cancellation-aware)."""
    return np.abs(np.asarray(g) - np.asarray(g_ref)) / np.maximum(np.asarray(gabs), 1e-300)


def rel(a, b):
    return abs(a - b) / abs(b)


def oracle_nll_threads(spec, theta, cols, weights=None, mlp_weights=None, threads=16):
    """The oracle's (nll, grad, gabs, n_bad) over all events, evaluated in
    contiguous chunks by independent oracle models on host threads (the
    oracle is single-threaded and its calls release the interpreter lock);
    the chunk results are added exactly rounded (math.fsum).  For full-size
    comparisons that a single thread would take minutes over."""
    import math
    from concurrent.futures import ThreadPoolExecutor

    n = len(cols[0])
    edges = np.linspace(0, n, threads + 1).astype(np.int64)

    def one(k):
        a, b = int(edges[k]), int(edges[k + 1])
        om, otop, oids = rfo.from_spec(spec)
        if mlp_weights is not None:
            for name, w in mlp_weights.items():
                om.set_mlp_weights(oids[name], w)
        w = None if weights is None else np.ascontiguousarray(weights[a:b])
        return om.nll_ex(otop, theta, [np.ascontiguousarray(c[a:b]) for c in cols], weights=w)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, range(threads)))
    nll = math.fsum(p[0] for p in parts)
    P = len(parts[0][1])
    grad = np.array([math.fsum(p[1][k] for p in parts) for k in range(P)])
    gabs = np.array([math.fsum(p[2][k] for p in parts) for k in range(P)])
    return nll, grad, gabs, sum(p[3] for p in parts)


def oracle_hess_threads(spec, theta, cols, weights=None, threads=16):
    """The oracle's (nll, grad, hess, n_bad) over all events in contiguous
    chunks on host threads, each entry added exactly rounded (math.fsum)."""
    import math
    from concurrent.futures import ThreadPoolExecutor

    n = len(cols[0])
    edges = np.linspace(0, n, threads + 1).astype(np.int64)

    def one(k):
        a, b = int(edges[k]), int(edges[k + 1])
        om, otop, _ = rfo.from_spec(spec)
        w = None if weights is None else np.ascontiguousarray(weights[a:b])
        return om.nll_hess(otop, theta, [np.ascontiguousarray(c[a:b]) for c in cols], weights=w)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, range(threads)))
    P = len(parts[0][1])
    nll = math.fsum(p[0] for p in parts)
    grad = np.array([math.fsum(p[1][k] for p in parts) for k in range(P)])
    hess = np.array([[math.fsum(p[2][i, j] for p in parts) for j in range(P)] for i in range(P)])
    return nll, grad, hess, sum(p[3] for p in parts)
