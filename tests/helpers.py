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
