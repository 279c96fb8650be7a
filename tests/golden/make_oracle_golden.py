"""Write oracle_fit_small.json: a small seeded fit and the FP64 oracle's result.

The paper prints no worked example of the fit (no input state, hit or
fitted value), so the stored expected values here are the oracle's own,
written by this script, which calls only the seeded input generator and
`oracle/`.  The fixture holds its inputs as well, so it does not depend on
the generator staying unchanged:

- barrel: the first 6 tracks of the 1,024-track parity workload, 10
  cylinders at r = linspace(4, 100, 10) cm, B = 3.8 T (propagate to r, then
  the 3D Kalman update, Section 2 of the paper);
- disk: the first 6 tracks of the p2z workload on its first 10 planes
  (|z| = 30 .. 157.9 cm, the side given by the sign of eta).

Run from the repository root: python tests/golden/make_oracle_golden.py
A later change to the oracle's arithmetic that moves these values must
rewrite the fixture in the same commit, naming the passage or reading that
justifies the change.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "oracle_fit_small.json")
N_TRACKS = 6
N_DISKS = 10


def _case(d: dict, kind: str, n_surf: int | None = None) -> dict:
    import oracle

    L = d["hits"].shape[1] if n_surf is None else n_surf
    inp = dict(par=d["par"][:N_TRACKS], cov=d["cov"][:N_TRACKS], q=d["q"][:N_TRACKS],
               hits=d["hits"][:N_TRACKS, :L], hitcov=d["hitcov"][:N_TRACKS, :L], surf=d["surf"][:L])
    ref = oracle.fit_layers(inp["par"], inp["cov"], inp["q"], inp["hits"], inp["hitcov"], inp["surf"], kind)
    tolist = lambda a: np.asarray(a, np.float64).tolist()  # noqa: E731  (repr of a double round-trips)
    return dict(kind=kind, bz=3.8,
                inputs={k: tolist(v) for k, v in inp.items()},
                expected=dict(par=tolist(ref["par"]), cov=tolist(ref["cov"]), chi2=tolist(ref["chi2"]),
                              nused=np.asarray(ref["nused"]).astype(int).tolist(),
                              status=np.asarray(ref["status"]).astype(np.int64).tolist()))


def main() -> None:
    sys.path.insert(0, ROOT)
    from synth import events as ev

    barrel = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=N_TRACKS)
    disk = ev.make_disk_event(ev.P2Z_THROUGHPUT, n_tracks=N_TRACKS)
    doc = {
        "about": "FP64 oracle fit of small seeded workloads; written by make_oracle_golden.py "
                 "(the paper prints no worked example of the fit)",
        "cases": {"barrel": _case(barrel, "barrel"), "disk": _case(disk, "disk", N_DISKS)},
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
