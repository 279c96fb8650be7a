"""GPU p2r / p2z on the stored small workloads against the oracle's stored fit.

Inputs and expected values come from tests/golden/oracle_fit_small.json
(written by tests/golden/make_oracle_golden.py with the FP64 oracle only);
the comparison uses the same tolerances as every other parity test.  6
tracks in one block of width W leave a ragged tail of W - 6 masked lanes.
"""
import numpy as np
import pytest

import paper_2401_14221_amd as p2r

from .parity import compare
from .test_gpu_fit import run_p2r, run_p2z
from .test_golden import load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = p2r.Context(0)
    yield c
    c.close()


def _inputs(case):
    c = load_golden()[case]
    d = {k: np.asarray(v, np.float64) for k, v in c["inputs"].items()}
    e = {k: np.asarray(v) for k, v in c["expected"].items()}
    return d, e


@pytest.mark.parametrize("W", [32, 64, 128, 256])
def test_p2r_matches_golden(ctx, W):
    d, e = _inputs("barrel")
    print(f"golden p2r W={W} n={d['par'].shape[0]}", flush=True)
    g = run_p2r(ctx, d, W)
    compare(g, e, ctx=f"golden p2r W={W}")


def test_p2z_matches_golden(ctx):
    d, e = _inputs("disk")
    print(f"golden p2z n={d['par'].shape[0]}", flush=True)
    g = run_p2z(ctx, d)
    compare(g, e, ctx="golden p2z", final_surface="plane")
