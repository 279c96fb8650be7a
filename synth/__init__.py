"""Seeded synthetic event generator shared by the tests, the benchmark and
the training-pair builder.

The module simulates charged particles by numerically integrating the
Lorentz-force equation of motion (classic fourth-order Runge-Kutta in path
length) through a uniform solenoidal field, records where each particle
crosses the detector surfaces, and smears those crossings into hits.  It
holds none of the fit's arithmetic: no analytic helix, no closed-form or
Newton crossing, no Jacobian and no Kalman update.  The workload shapes
follow the paper's mini-app workflow (events x tracks, batched tracks,
Section 2) with the distributions of the five benchmark configurations.
"""
from .events import (  # noqa: F401
    KAPPA, B_TESLA, P2R_PARITY, P2R_THROUGHPUT, P2Z_THROUGHPUT, RAGGED,
    LEARNED_EVAL, EventConfig, make_barrel_event, make_disk_event,
    make_ragged_event, make_mlp_pairs, make_mlp_init, rng, pack21, unpack21,
)
