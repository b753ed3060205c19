"""GPU parity of the Taylor-Hood P3/P2 pair (STOKES_FLAG_P3) against the
P3/P2 oracle (oracle/p3.py), through the C ABI.

The element pair changes, the solvers do not: the same assembled-matrix,
operator, solve, augmented-Lagrangian, adjoint and pressure-correction checks
as for P2/P1, with the same bars (matrices 1e-13 of the max-norm, patterns
bit-exact; operators 1e-13 FP64 / 2e-6 FP32; solution error 1e-10 on the
FP64 path at rel-res 1e-12, 1e-8 on the mixed path at rel-res 1e-10 or
tighter; gradients 1e-8).  The pressure multigrids (ops 6 and 8) coarsen
the P2 pressure to the P1 space of the same mesh first; the velocity
multigrid (op 9) needs the P2/P1 lattices and is refused.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import p3 as op3
from oracle import stokes as ostokes
from paper_2407_01783_amd import _lib, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(dim, n, seed=0, jitter=0.1, mu=1.0, alpha=100.0, gamma=0.0, strain=False):
    from paper_2407_01783_amd.stokes import StokesProblem
    print(f"[case] P3/P2 dim={dim} n={n} seed={seed} jitter={jitter} mu={mu} alpha={alpha} gamma={gamma} "
          f"strain={strain}", flush=True)
    return StokesProblem(dim, n, mesh_seed=seed, jitter=jitter, mu=mu, alpha=alpha, gamma=gamma, strain=strain,
                         p3=True)


def _oracle(dim, n, seed=0, jitter=0.1, mu=1.0, alpha=100.0, gamma=0.0, strain=False):
    m = op3.P3P2Mesh(dim, n, seed=seed, jitter=jitter)
    return ostokes.StokesSystem(m, mu, alpha, gamma, mats=op3.assemble_p3p2(m, grad_div=strain), strain=strain)


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dim,n,jit", [(2, 3, 0.0), (2, 4, 0.1), (3, 2, 0.1), (3, 3, 0.15)])
def test_p3_assembled_matrices_match_oracle(gpu_lib, dim, n, jit):
    P = _problem(dim, n, seed=5, jitter=jit, mu=0.3, alpha=40.0)
    S = _oracle(dim, n, seed=5, jitter=jit, mu=0.3, alpha=40.0)
    assert P.n_p2 == S.mesh.n_vel and P.n_p1 == S.mesh.n_q
    ref = {0: S.mats.Ms, 1: S.mats.Ls, 5: S.mats.MQ, 6: S.mats.LQ, 7: S.A_II}
    for c in range(dim):
        ref[2 + c] = S.mats.B[c]
    for which, A in ref.items():
        rp, cols, vals = P.export_csr(which)
        assert np.array_equal(rp, A.indptr) and np.array_equal(cols, A.indices), which
        scale = np.abs(A.data).max()
        assert np.abs(vals - A.data).max() <= 1e-13 * scale, which
    _, _, lam = P.export_csr(8)
    assert np.abs(lam - S.mats.Lam).max() <= 1e-14 * np.abs(S.mats.Lam).max()
    # the lumped-mass pressure operator B_I Lambda^-1 B_I^T
    Bm = sp.hstack(S.B_I).tocsr()
    lam_i = np.tile(1.0 / S.mats.Lam[S.I], dim)
    X = (Bm @ sp.diags(lam_i) @ Bm.T).tocsr()
    rp, cols, vals = P.export_csr(9)
    Xd = sp.csr_matrix((vals, cols, rp), shape=X.shape).toarray()
    assert np.abs(Xd - X.toarray()).max() <= 1e-13 * np.abs(X).max()
    # the mesh export holds the P3 nodes
    xy, ids = P.mesh()
    assert np.array_equal(ids, S.mesh.vel) and np.array_equal(xy, S.mesh.vel_coords)


@pytest.mark.parametrize("dim,n,nrhs", [(2, 4, 1), (3, 3, 1), (3, 2, 3)])
def test_p3_operator_actions_match_oracle(gpu_lib, dim, n, nrhs):
    P = _problem(dim, n, seed=1)
    S = _oracle(dim, n, seed=1)
    rng = np.random.default_rng(7)
    x_u = rng.standard_normal((nrhs, dim, P.n_p2))
    x_p = rng.standard_normal((nrhs, P.n_p1))
    I, d = S.I, dim
    Bf = [b for b in S.mats.B]
    ref = {}
    xi = x_u[:, :, I]
    y0 = np.zeros_like(x_u)
    y0[:, :, I] = np.einsum("ij,rcj->rci", S.A_II.toarray(), xi)
    ref[0] = y0
    ref[1] = np.stack([sum(S.B_I[c] @ xi[r, c] for c in range(d)) for r in range(nrhs)])
    y2 = np.zeros_like(x_u)
    for r in range(nrhs):
        for c in range(d):
            y2[r, c, I] = S.B_I[c].T @ x_p[r]
    ref[2] = y2
    ref[3] = np.stack([S.mats.MQ @ x_p[r] for r in range(nrhs)])
    ref[4] = np.stack([S.mats.LQ @ x_p[r] for r in range(nrhs)])
    Bm = sp.hstack(S.B_I).tocsr()
    X = Bm @ sp.diags(np.tile(1.0 / S.mats.Lam[I], d)) @ Bm.T
    ref[7] = np.stack([X @ x_p[r] for r in range(nrhs)])
    del Bf
    for op in (0, 1, 2, 3, 4, 7):
        x = x_p if op in (2, 3, 4, 7) else x_u
        for prec, tol in ((0, 1e-13), (1, 2e-6)):
            y = P.apply(op, torch.tensor(x.ravel(), device="cuda"), precision=prec, nrhs=nrhs).cpu().numpy()
            assert _rel(y, ref[op]) <= tol, (op, prec, _rel(y, ref[op]))
    # the velocity multigrid is P2/P1 only
    with pytest.raises(_lib.StokesError) as e:
        P.apply(9, torch.tensor(x_u.ravel(), device="cuda"), precision=0, nrhs=nrhs)
    assert e.value.status == -7


def _p3_pressure_mg_operators(S, dim):
    Bm = sp.hstack(S.B_I).tocsr()
    XL = Bm @ sp.diags(np.tile(1.0 / S.mats.Lam[S.I], dim)) @ Bm.T
    return {6: (S.mats.MQ + S.mats.LQ).tocsr(), 8: (XL + S.mats.MQ).tocsr()}


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 20), (3, 6)])
def test_p3_pressure_multigrid_vcycle(gpu_lib, dim, n):
    """The pressure V-cycles of a P3/P2 context (op 6: eps M_Q + L_Q with
    eps = 1, op 8: B_I Lambda_V^-1 B_I^T + M_Q, both on the P2 pressure) with
    the P1 space of the same mesh as first coarse level.  One level
    ((2n+1)^dim <= 1500 pressure nodes: 2D n=4) is the exact inverse; with
    several (2D n=20: 1,681 -> 441, 3D n=6: 2,197 -> 343 nodes) each cycle is
    symmetric positive definite and, as a stationary iteration on the
    oracle's operator, reduces the residual at every one of eight cycles: by
    at least 2x for op 6; for op 8 by at least 1.25x, since its operator is
    close to the P2 mass matrix, whose low-energy non-smooth modes neither
    the P1 coarse space nor the smoothing interval covers (0.72 per cycle
    measured in 3D, 0.25 in 2D)."""
    P, S = _problem(dim, n, seed=3), _oracle(dim, n, seed=3)
    rng = np.random.default_rng(11)
    u, v, b = rng.standard_normal((3, S.mats.MQ.shape[0]))
    single = (2 * n + 1) ** dim <= 1500
    for op, A in _p3_pressure_mg_operators(S, dim).items():
        V = lambda x: P.apply(op, torch.tensor(x, device="cuda"), precision=0).cpu().numpy()  # noqa: E731
        if single:
            assert _rel(V(b), np.linalg.solve(A.toarray(), b)) <= 1e-10, op
            continue
        Vu, Vv = V(u), V(v)
        assert abs(u @ Vv - v @ Vu) <= 1e-12 * abs(u @ Vv), op
        assert u @ Vu > 0 and v @ Vv > 0
        x = np.zeros_like(b)
        res = [np.linalg.norm(b)]
        for _ in range(8):
            x = x + V(b - A @ x)
            res.append(np.linalg.norm(b - A @ x))
        rates = np.array(res[1:]) / np.array(res[:-1])
        print(f"P3/P2 dim={dim} n={n} op {op}: rates {rates}", flush=True)
        assert rates.max() <= (0.5 if op == 6 else 0.8), (op, rates)


def _solve_and_compare(P, S, f, ubc, method, tol_err, **opts):
    F, g = S.rhs(f, ubc)
    U, Pp = S.solve(F, g)
    u_ref = S.full_velocity(U, ubc)
    fb = torch.tensor(f[None], device="cuda")
    ub = torch.tensor(ubc[None], device="cuda") if ubc is not None else None
    u, p, info = P.solve(fb, ubc=ub, method=method, **opts)
    assert info["status"] == 0, info
    u, p = u.cpu().numpy()[0], p.cpu().numpy()[0]
    eu, ep = _rel(u, u_ref), _rel(p, Pp)
    print(f"[{method}] err_u={eu:.2e} err_p={ep:.2e} info={info}", flush=True)
    assert eu <= tol_err and ep <= tol_err, (eu, ep, info)
    if ubc is not None:
        bnd = S.mesh.p2_boundary
        assert np.array_equal(u[:, bnd], ubc[:, bnd])
    assert abs(S.mQ @ p) <= 1e-12 * max(1.0, np.abs(p).max())
    return info


@pytest.mark.parametrize("coupled_pc", [0, 1, 2])
@pytest.mark.parametrize("inner_mode", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_p3_coupled_solves(gpu_lib, coupled_pc, inner_mode, precision):
    kw = dict(dim=3, n=3, seed=2, mu=1e-2, alpha=100.0)
    P, S = _problem(**kw), _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1002)
    rtol, tol = (1e-12, 1e-10) if precision == 0 else (1e-11, 1e-8)
    _solve_and_compare(P, S, f, None, "coupled", tol, precision=precision, rtol=rtol, coupled_pc=coupled_pc,
                       inner_mode=inner_mode, max_outer=3000, max_refine=40)


@pytest.mark.parametrize("schur_pc", [0, 1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_p3_schur_solves(gpu_lib, schur_pc, precision):
    kw = dict(dim=2, n=5, seed=3, mu=0.1, alpha=100.0)
    P, S = _problem(**kw), _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1003)
    rtol, tol = (1e-13, 1e-10) if precision == 0 else (1e-12, 1e-8)
    _solve_and_compare(P, S, f, None, "schur", tol, precision=precision, rtol=rtol, schur_pc=schur_pc,
                       max_outer=3000, max_refine=40)


@pytest.mark.parametrize("method", ["schur", "coupled"])
def test_p3_dirichlet_data_and_augmented_lagrangian(gpu_lib, method):
    kw = dict(dim=3, n=2, seed=4, mu=0.5, alpha=100.0)
    S = _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1004)
    x = S.mesh.p2coords
    ubc = np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0]), x[:, 0] * x[:, 1]])
    for gamma in (0.0, 5.0):
        P = _problem(gamma=gamma, **kw)
        _solve_and_compare(P, S, f, ubc, method, 1e-10, rtol=1e-14, max_outer=3000, max_refine=30)


def test_p3_manufactured_2d_mixed(gpu_lib):
    mu, alpha = 1.0, 100.0
    S = _oracle(2, 6, jitter=0.0, mu=mu, alpha=alpha)
    _, _, f = inputs.manufactured_2d(S.mesh.p2coords, mu, alpha)
    u, _, _ = inputs.manufactured_2d(S.mesh.p2coords, mu, alpha)
    P = _problem(2, 6, jitter=0.0, mu=mu, alpha=alpha)
    _solve_and_compare(P, S, f, u, "coupled", 1e-8, precision=1, rtol=1e-12, max_outer=3000, max_refine=30)


def test_p3_strain_form(gpu_lib):
    kw = dict(dim=3, n=2, seed=8, mu=0.2, alpha=50.0, strain=True)
    P, S = _problem(**kw), _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1008)
    for precision, rtol, tol in ((0, 1e-13, 1e-10), (1, 1e-12, 1e-8)):
        _solve_and_compare(P, S, f, None, "coupled", tol, precision=precision, rtol=rtol, max_outer=3000,
                           max_refine=40)


def test_p3_adjoint_gradient_matches_oracle(gpu_lib):
    kw = dict(dim=3, n=2, seed=3, mu=0.2, alpha=50.0)
    P, S = _problem(**kw), _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1003)
    ft = inputs.fourier_forcing(S.mesh.p2coords, 9003)
    U, _ = S.solve(*S.rhs(f))
    Ut, _ = S.solve(*S.rhs(ft))
    u, ut = S.full_velocity(U), S.full_velocity(Ut)
    _, dJdu = ostokes.quadratic_loss(S, u, ut)
    w = np.linspace(-1.0, 1.0, S.np1)
    dJdf, dJdmu, _, _ = S.adjoint_gradient(u, dJdu, dJdp=w)
    for precision in (0, 1):
        _, _, gf, gmu, info = P.adjoint(torch.tensor(u[None], device="cuda"),
                                        torch.tensor(dJdu[None], device="cuda"),
                                        torch.tensor(w[None], device="cuda"), precision=precision, rtol=1e-12,
                                        max_outer=3000, max_refine=40)
        assert info["status"] == 0
        assert _rel(gf.cpu().numpy()[0], dJdf) <= 1e-8
        assert abs(float(gmu[0]) - dJdmu) <= 1e-8 * abs(dJdmu)


@pytest.mark.parametrize("precision", [0, 1])
def test_p3_projection_step_matches_oracle(gpu_lib, precision):
    kw = dict(dim=2, n=4, seed=6, mu=0.05, alpha=80.0)
    P, S = _problem(**kw), _oracle(**kw)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1006)
    rng = np.random.default_rng(3)
    pold = rng.standard_normal(S.np1)
    U, Pp = S.projection_step(f, None, pold)
    u, p, info = P.projection_step(torch.tensor(f[None], device="cuda"),
                                   p_old=torch.tensor(pold[None], device="cuda"), precision=precision, rtol=1e-12,
                                   max_inner=5000, max_refine=30)
    assert info["status"] == 0, info
    tol = 1e-10 if precision == 0 else 1e-8
    assert _rel(u.cpu().numpy()[0], S.full_velocity(U)) <= tol
    assert _rel(p.cpu().numpy()[0], Pp) <= tol


def test_p3_velocity_multigrid_refused(gpu_lib):
    P = _problem(2, 3)
    f = torch.zeros((1, 2, P.n_p2), dtype=torch.float64, device="cuda")
    f[0, 0, P.n_p2 // 2] = 1.0
    with pytest.raises(_lib.StokesError) as e:
        P.solve(f, vel_pc=1)
    assert e.value.status == -7


def test_p3_galerkin_multigrid_switch(gpu_lib, monkeypatch):
    """STOKES_MGX_P3=0 leaves the Galerkin hierarchy unbuilt: op 8 is refused,
    the eps M_Q + L_Q cycle (op 6) is bit for bit the one of a default
    context, and a mixed coupled solve (lumped Cahouet-Chabard term, now on
    the op-6 cycle) still converges to the requested residual."""
    b = np.random.default_rng(2).standard_normal((2 * 10 + 1) ** 2)
    ref = _problem(2, 10).apply(6, torch.tensor(b, device="cuda"), precision=0).cpu().numpy()
    monkeypatch.setenv("STOKES_MGX_P3", "0")
    P = _problem(2, 10)
    with pytest.raises(_lib.StokesError) as e:
        P.apply(8, torch.tensor(b, device="cuda"), precision=0)
    assert e.value.status == -7
    y = P.apply(6, torch.tensor(b, device="cuda"), precision=0).cpu().numpy()
    assert np.array_equal(y, ref)
    f = torch.tensor(np.random.default_rng(3).standard_normal((1, 2, P.n_p2)), device="cuda")
    info = P.solve(f, precision=1, rtol=1e-8)[2]
    assert info["status"] == 0 and info["rel_res"] <= 1e-8, info
