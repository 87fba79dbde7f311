"""Writes the stored expected values under tests/golden/ from the oracle alone.

    python tests/golden/make_golden.py

The paper prints no worked numerical examples (its results are timing
ratios), so the fixtures are small hand-listed samples of each model at its
truth point, evaluated by the FP64 oracle.  Event values are FP32-representable
(as every path reads them).  test_golden.py checks that the oracle still
reproduces them and that the GPU path matches them.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rfo  # noqa: E402
from paper_2003_12861_amd import synth, workloads  # noqa: E402


def f32(v):
    return [float(np.float32(x)) for x in v]


CASES = [
    # (name, spec builder args, theta, columns)
    ("gauss_cheb_one", ("gauss_cheb", {}), workloads.truth_vector(synth.GAUSS_CHEB_TRUTH), [f32([0.7])]),
    ("gauss_cheb_three", ("gauss_cheb", {}), workloads.truth_vector(synth.GAUSS_CHEB_TRUTH), [[-1.0, 0.5, 2.0]]),
    ("gauss_cheb_tails", ("gauss_cheb", {}), [0.3, 0.8, 0.25, 0.15, -0.05], [f32([-9.5, -4.25, 3.75, 9.875])]),
    ("decay_argus_three", ("decay_argus", {}), workloads.truth_vector(synth.DECAY_TRUTH),
     [f32([0.5, 2.0, 7.5]), f32([5.279, 5.25, 5.285])]),
    ("bwcb_exact_three", ("bwcb", {"K": 1024}), workloads.truth_vector(synth.BWCB_TRUTH), [f32([85.0, 91.0, 100.5])]),
    # a lone Gaussian: the two outer events have densities near 1e-33, below
    # the FP32 path's 1e-30 threshold, so that path re-evaluates them in FP64
    ("gauss_far_tail", ("gauss", {}), [0.3, 0.8], [f32([-9.5, 0.1, 9.75])]),
]


def spec_gauss(lo=-10.0, hi=10.0):
    return [("obs", "x", [], [lo, hi]), ("param", "mu", [], [-5.0, 5.0]),
            ("param", "sigma", [], [0.05, 10.0]), ("gauss", "sig", ["x", "mu", "sigma"], [])]


def spec_of(kind, kw):
    return {"gauss_cheb": workloads.spec_gauss_cheb, "decay_argus": workloads.spec_decay_argus,
            "bwcb": workloads.spec_bwcb, "gauss": spec_gauss}[kind](**kw)


def main():
    out = {"note": "values written by tests/golden/make_golden.py from the FP64 oracle", "cases": []}
    for name, (kind, kw), theta, cols in CASES:
        spec = [list(e) for e in spec_of(kind, kw)]
        m, top, _ = rfo.from_spec(spec)
        nll, g, gabs, nb = m.nll_ex(top, list(theta), [np.array(c, dtype=np.float64) for c in cols])
        out["cases"].append(dict(name=name, spec=spec, theta=[float(t) for t in theta], columns=cols,
                                 nll=float(nll), grad=[float(v) for v in g], grad_scale=[float(v) for v in gabs]))
    # binned: a small model with stored tables
    d = synth.make_binned(seed=11, C=2, S=2, B=3, J=2)
    Lp = np.log(d["Tp"] / d["T"][:, :, None, :])
    Lm = np.log(d["Tm"] / d["T"][:, :, None, :])
    theta = [1.1, 0.4, -0.7]
    nll, g = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], theta)
    out["binned"] = dict(T=d["T"].tolist(), Tp=d["Tp"].tolist(), Tm=d["Tm"].tolist(), nobs=d["nobs"].tolist(),
                         theta=theta, nll=float(nll), grad=[float(v) for v in g])
    with open(os.path.join(HERE, "oracle_small.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", os.path.join(HERE, "oracle_small.json"))


if __name__ == "__main__":
    main()
