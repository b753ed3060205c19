"""Velocity multigrid (stokes_solve_opts.vel_pc = STOKES_VEL_MG): the V-cycle
for alpha M + mu L against the oracle's assembled operator, and solves with
it against the FP64 oracle.

* one level (<= 1500 interior nodes): the V-cycle is the exact inverse;
* several levels: symmetric positive definite (it preconditions CG), and as
  a stationary iteration on the oracle's A_II it reduces the residual by at
  least 2x per cycle, for mass- and stiffness-dominated A;
* coupled / Schur solves with the multigrid velocity block reach the oracle
  solution (1e-10 FP64, 1e-8 mixed);
* the inner velocity CG iterations per velocity solve do not grow from
  n = 16 to n = 32 at mu = 1 (stiffness dominated), unlike Chebyshev-Jacobi.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import stokes as ostokes
from paper_2407_01783_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _pair(dim, n, seed=3, mu=1.0, alpha=100.0):
    from paper_2407_01783_amd.stokes import StokesProblem
    print(f"[case] vmg dim={dim} n={n} seed={seed} mu={mu} alpha={alpha}", flush=True)
    P = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha)
    S = ostokes.StokesSystem(omesh.KuhnMesh(dim, n, seed=seed, jitter=0.1), mu, alpha)
    return P, S


def _vcycle(P, S, X):
    """Apply op 9 to interior component arrays X (dim, n_I)."""
    full = np.zeros((S.d, S.mesh.n_p2))
    full[:, S.I] = X
    y = P.apply(9, torch.tensor(full.ravel(), device="cuda"), precision=0).cpu().numpy()
    return y.reshape(S.d, -1)[:, S.I]


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 4)])
def test_vcycle_single_level_is_exact(gpu_lib, dim, n):
    P, S = _pair(dim, n)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((dim, S.nI))
    Y = _vcycle(P, S, X)
    A = S.A_II.toarray()
    assert _rel(Y, np.linalg.solve(A, X.T).T) <= 1e-10


@pytest.mark.parametrize("dim,n,mu", [(3, 16, 1.0), (3, 16, 1e-3), (3, 24, 1.0), (2, 64, 1.0)])
def test_vcycle_symmetric_and_contracting(gpu_lib, dim, n, mu):
    P, S = _pair(dim, n, mu=mu)
    rng = np.random.default_rng(2)
    u, v, b = (rng.standard_normal((dim, S.nI)) for _ in range(3))
    Vu, Vv = _vcycle(P, S, u), _vcycle(P, S, v)
    assert abs(np.sum(u * Vv) - np.sum(v * Vu)) <= 1e-11 * abs(np.sum(u * Vv))
    assert np.sum(u * Vu) > 0 and np.sum(v * Vv) > 0
    x = np.zeros_like(b)
    res = [np.linalg.norm(b)]
    for _ in range(4):
        r = b - np.stack([S.A_II @ x[c] for c in range(dim)])
        x = x + _vcycle(P, S, r)
        res.append(np.linalg.norm(b - np.stack([S.A_II @ x[c] for c in range(dim)])))
    rates = np.array(res[1:]) / np.array(res[:-1])
    print(f"[vmg] dim={dim} n={n} mu={mu} rates {rates}", flush=True)
    assert rates.max() <= 0.5, rates


CASES = [("coupled", 0, dict(coupled_pc=0), 1e-13, 1e-10), ("coupled", 1, dict(coupled_pc=1, inner_mode=1), 1e-11, 1e-8),
         ("schur", 0, dict(schur_pc=1), 1e-13, 1e-9)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_solves_with_velocity_multigrid(gpu_lib, case):
    method, precision, extra, rtol, tol = CASES[case]
    P, S = _pair(3, 8, seed=5, mu=0.5, alpha=40.0)
    rng = np.random.default_rng(4)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1005)
    ubc = rng.standard_normal((3, P.n_p2))
    U, Pp = S.solve_direct(*S.rhs(f, ubc))
    u, p, info = P.solve(torch.tensor(f[None], device="cuda"), ubc=torch.tensor(ubc[None], device="cuda"),
                         method=method, precision=precision, rtol=rtol, vel_pc=1, max_outer=2000, max_refine=30,
                         **extra)
    assert info["status"] == 0, info
    assert _rel(u.cpu().numpy()[0], S.full_velocity(U, ubc)) <= tol
    assert _rel(p.cpu().numpy()[0], Pp) <= 10 * tol


def test_inner_iterations_flat_in_h(gpu_lib):
    """Schur CG at mu = 1 (mu dt / h^2 >> 1): velocity CG iterations per
    velocity solve with the multigrid preconditioner stay flat from n = 16
    to n = 32; with Chebyshev-Jacobi they grow."""
    from paper_2407_01783_amd.stokes import StokesProblem
    per = {}
    for n in (16, 32):
        P = StokesProblem(3, n, mesh_seed=0, jitter=0.1, mu=1.0, alpha=100.0)
        xy, _ = P.mesh()
        f = torch.tensor(inputs.fourier_forcing(xy, 1000)[None], device="cuda")
        for vel_pc in (1, 0):
            _, _, info = P.solve(f, method="schur", precision=0, rtol=1e-8, vel_pc=vel_pc, inner_rtol_u=1e-6,
                                 max_outer=2000, max_inner=5000)
            assert info["status"] == 0, info
            solves = info["outer_iters"] + 2 * info["refinements"]
            per[(n, vel_pc)] = info["inner_iters_u"] / max(1, solves)
            print(f"[vmg] n={n} vel_pc={vel_pc} {info}", flush=True)
    assert per[(32, 1)] <= 1.3 * per[(16, 1)], per
    assert per[(32, 0)] >= 1.5 * per[(16, 0)], per
    assert per[(32, 1)] < per[(32, 0)], per
