"""Host-side checks of bench.py's helpers (no GPU)."""

import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

torch = pytest.importorskip("torch")


def _golden():
    vel, pres = {}, {}
    with open(bench.ORACLE_SOLUTION_FILE) as fh:
        lines = [ln.split() for ln in fh if not ln.startswith("#")]
    for i, ln in enumerate(lines):
        if ln[0] in ("vel", "p"):
            for r in lines[i + 1:i + 1 + int(ln[1])]:
                (vel if ln[0] == "vel" else pres)[int(r[0])] = [float(v) for v in r[1:]]
    return vel, pres


@pytest.mark.skipif(not os.path.exists(bench.ORACLE_SOLUTION_FILE), reason="golden file absent")
def test_error_vs_stored_oracle_reads_every_sampled_value():
    """The stored oracle values placed in full-size arrays give error 0; a
    perturbation of one sampled node by a known amount gives exactly that
    relative error."""
    vel, pres = _golden()
    n_p2, n_p1 = 129 ** 3, 65 ** 3
    u = np.zeros((1, 3, n_p2))
    p = np.zeros((1, n_p1))
    for k, v in vel.items():
        u[0, :, k] = v
    for k, v in pres.items():
        p[0, k] = v[0]
    e = bench.error_vs_stored_oracle(torch.tensor(u), torch.tensor(p))
    assert e["nodal_rel_l2_u"] == 0.0 and e["nodal_rel_l2_p"] == 0.0
    assert e["nodes"] == len(vel) and e["vertices"] == len(pres)
    ug = np.array(list(vel.values()))
    k = max(vel, key=lambda i: abs(vel[i][0]))
    u[0, 0, k] += 1e-3
    e = bench.error_vs_stored_oracle(torch.tensor(u), torch.tensor(p))
    assert e["nodal_rel_l2_u"] == pytest.approx(1e-3 / np.linalg.norm(ug), rel=1e-9)
