"""The oracle against its stored small-workload fixture (CPU).

tests/golden/oracle_fit_small.json holds seeded inputs and the FP64
oracle's fit of them, written by tests/golden/make_oracle_golden.py (the
paper prints no worked example of the fit).  The oracle's pins against
closed forms live in test_oracle_pins.py; this test guards the stored
values: the oracle must still reproduce them, so a change to its arithmetic
cannot pass unnoticed, and the fixture's inputs must still be the ones the
generator draws.
"""
import json
import os

import numpy as np
import pytest

from synth import events as ev

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fit_small.json")


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", ["barrel", "disk"])
def test_oracle_reproduces_golden(orc, case):
    c = load_golden()[case]
    i = {k: np.asarray(v, np.float64) for k, v in c["inputs"].items()}
    got = orc.fit_layers(i["par"], i["cov"], i["q"], i["hits"], i["hitcov"], i["surf"], c["kind"], bz=c["bz"])
    e = c["expected"]
    # same FP64 arithmetic on the same inputs: equal up to the compiler's
    # choice of operation order (none is expected at -O2 without fast-math)
    for k in ("par", "cov", "chi2"):
        np.testing.assert_allclose(got[k], np.asarray(e[k]), rtol=1e-12, atol=1e-15, err_msg=f"{case} {k}")
    np.testing.assert_array_equal(got["nused"], np.asarray(e["nused"]))
    np.testing.assert_array_equal(got["status"].astype(np.int64), np.asarray(e["status"]))


def test_golden_inputs_are_the_generator_draws():
    g = load_golden()
    b = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=len(g["barrel"]["inputs"]["q"]))
    d = ev.make_disk_event(ev.P2Z_THROUGHPUT, n_tracks=len(g["disk"]["inputs"]["q"]))
    for case, src in (("barrel", b), ("disk", d)):
        inp = g[case]["inputs"]
        L = len(inp["surf"])
        for k in ("par", "cov", "q"):
            np.testing.assert_array_equal(np.asarray(inp[k]), src[k], err_msg=f"{case} {k}")
        for k in ("hits", "hitcov"):
            np.testing.assert_array_equal(np.asarray(inp[k]), src[k][:, :L], err_msg=f"{case} {k}")
        np.testing.assert_array_equal(np.asarray(inp["surf"]), src["surf"][:L])


def test_golden_values_are_plausible():
    """Every update applied, chi2 near its degrees of freedom per hit, and
    every fitted covariance symmetric positive semi-definite."""
    for case, ndf in (("barrel", 3), ("disk", 2)):
        e = load_golden()[case]["expected"]
        L = len(load_golden()[case]["inputs"]["surf"])
        assert all(n == L for n in e["nused"])
        chi2 = np.asarray(e["chi2"])
        assert np.all(chi2 > 0) and 0.3 * ndf * L < chi2.mean() < 2.0 * ndf * L
        for v in e["cov"]:
            C = ev.unpack21(np.asarray(v))
            assert np.allclose(C, C.T)
            assert np.linalg.eigvalsh(C).min() > -1e-9 * np.abs(C).max()
