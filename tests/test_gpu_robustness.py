"""Failure handling and observability of the solve entry points (GPU).

* Non-finite input is an error, never convergence: a NaN or Inf in the
  forcing, the boundary data, the initial guess or the adjoint's loss
  gradient returns STOKES_ERR_NONFINITE (-4) from every solve entry point,
  and the context keeps working afterwards.
* The residual history of stokes_solve_info has one entry per outer
  iteration and ends near the final residual; the phase times (profile = 2)
  are positive and fit inside the call's wall time.
"""

import math

import numpy as np
import pytest

from paper_2407_01783_amd import _lib, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NONFINITE = -4


@pytest.fixture(scope="module")
def prob(gpu_lib):
    from paper_2407_01783_amd.stokes import StokesProblem
    print("[case] robustness 3D n=4 seed=2", flush=True)
    P = StokesProblem(3, 4, mesh_seed=2, jitter=0.1, mu=1e-2, alpha=100.0)
    xy, _ = P.mesh()
    f = torch.tensor(inputs.fourier_forcing(xy, inputs.forcing_seed(2))[None], device=P.device)
    return P, f


def _expect_nonfinite(fn):
    with pytest.raises(_lib.StokesError) as e:
        fn()
    assert e.value.status == NONFINITE, e.value


@pytest.mark.parametrize("bad", [math.nan, math.inf])
@pytest.mark.parametrize("where", ["f", "ubc", "x0"])
@pytest.mark.parametrize("method,precision", [("coupled", 1), ("coupled", 0), ("schur", 0)])
def test_nonfinite_input_is_an_error(prob, bad, where, method, precision):
    P, f = prob
    print(f"[case] nonfinite {where}={bad} {method} precision={precision}", flush=True)
    ff, ubc, x0 = f.clone(), None, None
    if where == "f":
        ff[0, 1, P.n_p2 // 2] = bad
    elif where == "ubc":
        ubc = torch.zeros_like(f)
        ubc[0, 0, 0] = bad  # node 0 is a boundary node
    else:
        x0u = torch.zeros_like(f)
        x0u[0, 2, P.n_p2 // 2] = bad
        x0 = (x0u, torch.zeros((1, P.n_p1), dtype=torch.float64, device=P.device))
    _expect_nonfinite(lambda: P.solve(ff, ubc=ubc, x0=x0, method=method, precision=precision, rtol=1e-10,
                                      inner_mode=1))
    u, p, info = P.solve(f, method=method, precision=precision, rtol=1e-10)
    assert info["status"] == 0 and torch.isfinite(u).all() and torch.isfinite(p).all()


def test_nonfinite_projection_and_adjoint(prob):
    P, f = prob
    ff = f.clone()
    ff[0, 0, P.n_p2 // 3] = math.nan
    _expect_nonfinite(lambda: P.projection_step(ff, rtol=1e-10))
    pold = torch.zeros((1, P.n_p1), dtype=torch.float64, device=P.device)
    pold[0, 5] = math.inf
    _expect_nonfinite(lambda: P.projection_step(f, p_old=pold, rtol=1e-10))
    u, _, info = P.solve(f, rtol=1e-10)
    assert info["status"] == 0
    g = torch.zeros_like(u)
    g[0, 1, P.n_p2 // 2] = math.nan
    _expect_nonfinite(lambda: P.adjoint(u, g, rtol=1e-10))
    _, _, _, dmu, info = P.adjoint(u, u, rtol=1e-10)
    assert info["status"] == 0 and torch.isfinite(dmu).all()


@pytest.mark.parametrize("method,precision,inner_mode", [("coupled", 1, 1), ("coupled", 0, 0), ("schur", 0, 0)])
def test_residual_history_and_phase_times(prob, method, precision, inner_mode):
    P, f = prob
    u, p, info = P.solve(f, method=method, precision=precision, inner_mode=inner_mode, rtol=1e-10, profile=2,
                         coupled_pc=1, hist_cap=500)
    print(f"[case] history {method} p{precision}: {info}", flush=True)
    assert info["status"] == 0
    h = np.array(info["res_hist"])
    assert len(h) == info["outer_iters"] == info["res_hist_len"] > 0
    assert np.all(np.isfinite(h)) and np.all(h >= 0)
    assert h[0] < 1.0
    if method == "coupled":
        # the last estimate is the last cycle's least-squares residual: it
        # met the cycle's goal, within a small factor of the true residual
        assert h[-1] <= 20 * max(info["rel_res"], 1e-10)
    t = info["seconds_inner_u"], info["seconds_inner_p"], info["seconds_orth"]
    assert t[0] > 0 and t[1] > 0
    assert (t[2] > 0) == (method == "coupled")
    assert sum(t) <= info["seconds_total"] * 1.05
    # a capped buffer keeps the first entries
    _, _, info2 = P.solve(f, method=method, precision=precision, inner_mode=inner_mode, rtol=1e-10,
                          coupled_pc=1, hist_cap=3)
    assert info2["res_hist_len"] == 3 and np.allclose(info2["res_hist"], h[:3], rtol=1e-12, atol=0)
    assert info2["seconds_inner_u"] == 0.0  # profile off


def test_tuning_cache_file(gpu_lib, tmp_path, monkeypatch):
    """STOKES_TUNE_CACHE: the first context writes its lanes-per-row choices
    (8 right-hand sides, W = 24, where several G compile), a second context
    of the same problem reads them instead of timing, and both solve alike."""
    from paper_2407_01783_amd.stokes import StokesProblem
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("STOKES_TUNE_CACHE", str(path))
    kw = dict(mesh_seed=5, jitter=0.1, mu=1e-2, alpha=100.0)
    P1 = StokesProblem(3, 5, **kw)
    xy, _ = P1.mesh()
    f = torch.tensor(np.stack([inputs.fourier_forcing(xy, inputs.forcing_seed(5, b)) for b in range(8)]),
                     device=P1.device)
    u1, p1, i1 = P1.solve(f, precision=1, rtol=1e-10)
    lines = path.read_text().split()
    assert i1["status"] == 0 and len(lines) >= 6 and len(lines) % 3 == 0, lines
    assert all(g in ("1", "2", "4", "8") for g in lines[2::3])
    del P1
    P2 = StokesProblem(3, 5, **kw)
    u2, p2, i2 = P2.solve(f, precision=1, rtol=1e-10)
    assert i2["status"] == 0
    assert path.read_text().split() == lines  # read, not re-timed and appended
    assert torch.equal(u1, u2) and torch.equal(p1, p2)


@pytest.mark.parametrize("method,precision,inner_mode", [("coupled", 1, 1), ("coupled", 0, 0), ("schur", 1, 0)])
def test_algorithmic_bytes_of_a_solve(prob, method, precision, inner_mode):
    """bytes_alg counts every kernel of the call: the same solve counts the
    same bytes; it covers at least one pass of the stored velocity operator
    per outer iteration; a batch of two right-hand sides reads the operators
    once for both, so it counts less than two single solves."""
    P, f = prob
    kw = dict(method=method, precision=precision, inner_mode=inner_mode, rtol=1e-10)
    _, _, a = P.solve(f, **kw)
    _, _, b = P.solve(f, **kw)
    print(f"[case] bytes {method} p{precision} m{inner_mode}: {a['bytes_alg']:.4g} B in {a['seconds_total']:.4g} s, "
          f"{a['outer_iters']} outer", flush=True)
    assert a["status"] == 0 and a["bytes_alg"] == b["bytes_alg"] > 0
    val = 2 if precision else 8
    assert a["bytes_alg"] >= a["outer_iters"] * P.nnz_A * val
    f2 = torch.cat([f, 0.5 * f])
    _, _, c = P.solve(f2, **kw)
    assert c["status"] == 0 and c["bytes_alg"] < 2 * a["bytes_alg"] * max(1.0, c["outer_iters"] / a["outer_iters"])

