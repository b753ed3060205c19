"""GPU adjoint checks beyond the oracle comparison in test_gpu_parity:

* central finite differences of J(f) = 1/2 (u - u*)^T M_V (u - u*) on 16
  seeded unit-RMS directions, from FP64 forward solves at rel-res 1e-13.  J
  is exactly quadratic in f, so the central difference has no truncation
  error at any step; the step h = 1e-3 keeps the rounding noise (forward
  error / h) near 1e-9.  Pass: |FD - d^T grad J| <= 1e-6 |FD| + 1e-12 J.
  For mu (not quadratic) the step is 1e-3 mu (truncation O(h^2)); pass at 1e-5.
* the torch.autograd.Function: grad of an l2 loss through StokesSolve equals
  the oracle's adjoint gradient with dJ/du = u - u*.
"""

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import stokes as ostokes
from paper_2407_01783_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIM, N, SEED, MU, ALPHA = 3, 4, 3, 1e-2, 100.0


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def small(gpu_lib):
    from paper_2407_01783_amd.stokes import StokesProblem
    print(f"[case] adjoint dim={DIM} n={N} seed={SEED} mu={MU} alpha={ALPHA}", flush=True)
    P = StokesProblem(DIM, N, mesh_seed=SEED, jitter=0.1, mu=MU, alpha=ALPHA)
    S = ostokes.StokesSystem(omesh.KuhnMesh(DIM, N, seed=SEED, jitter=0.1), MU, ALPHA)
    return P, S


def test_adjoint_gradient_finite_differences(small):
    P, S = small
    f = inputs.fourier_forcing(S.mesh.p2coords, inputs.forcing_seed(SEED, 0))
    Ut, _ = S.solve(*S.rhs(inputs.fourier_forcing(S.mesh.p2coords, inputs.target_seed(SEED))))
    ut = S.full_velocity(Ut)
    fwd = dict(method="coupled", precision=0, rtol=1e-13)

    def J(fv, mu=None):
        if mu is not None:
            P.set_mu(mu)
        u, _, info = P.solve(torch.tensor(fv[None], device="cuda"), **fwd)
        assert info["status"] == 0, info
        return ostokes.quadratic_loss(S, u.cpu().numpy()[0], ut)[0], u

    J0, u = J(f)
    _, dJdu = ostokes.quadratic_loss(S, u.cpu().numpy()[0], ut)
    _, _, gf, gmu, info = P.adjoint(u, torch.tensor(dJdu[None], device="cuda"), rtol=1e-13)
    assert info["status"] == 0
    gf, gmu = gf.cpu().numpy()[0], float(gmu[0])
    h = 1e-3
    for j, d in enumerate(inputs.fd_directions(f.shape, 16, 77)):
        fd = (J(f + h * d)[0] - J(f - h * d)[0]) / (2 * h)
        an = float(np.sum(d * gf))
        assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12 * J0, (j, fd, an)
    hm = 1e-3 * MU
    fdm = (J(f, MU + hm)[0] - J(f, MU - hm)[0]) / (2 * hm)
    P.set_mu(MU)
    assert abs(fdm - gmu) <= 1e-5 * abs(fdm), (fdm, gmu)


def test_autograd_function_matches_oracle_gradient(small):
    from paper_2407_01783_amd.stokes import StokesSolve
    P, S = small
    f = inputs.fourier_forcing(S.mesh.p2coords, inputs.forcing_seed(SEED, 1))
    ut = S.full_velocity(S.solve(*S.rhs(inputs.fourier_forcing(S.mesh.p2coords, inputs.target_seed(SEED))))[0])
    ft = torch.tensor(f, device="cuda", requires_grad=True)
    mu = torch.tensor(MU, dtype=torch.float64, requires_grad=True)
    u, p = StokesSolve.apply(ft, mu, P, dict(method="coupled", precision=1, rtol=1e-12))
    target = torch.tensor(ut, device="cuda")
    loss = 0.5 * ((u - target) ** 2).sum()
    loss.backward()
    un = u.detach().cpu().numpy()
    dJdf, dJdmu, _, _ = S.adjoint_gradient(un, un - ut)
    assert ft.grad is not None and mu.grad is not None
    assert _rel(ft.grad.cpu().numpy(), dJdf) <= 1e-8
    assert abs(float(mu.grad) - dJdmu) <= 1e-8 * abs(dJdmu)
    assert p.shape == (S.np1,)


def test_autograd_two_solves_at_different_mu(small):
    """Two StokesSolve calls on one problem at different mu, backpropagated
    together: each backward must run the adjoint with its own forward
    operator (mu saved by the forward pass), and the problem's mu is left as
    the caller set it."""
    from paper_2407_01783_amd.stokes import StokesSolve
    P, S = small
    mesh_ = S.mesh
    f = inputs.fourier_forcing(mesh_.p2coords, inputs.forcing_seed(SEED, 2))
    ut = S.full_velocity(S.solve(*S.rhs(inputs.fourier_forcing(mesh_.p2coords, inputs.target_seed(SEED))))[0])
    target = torch.tensor(ut, device="cuda")
    ft = torch.tensor(f, device="cuda", requires_grad=True)
    mus = (MU, 3.0 * MU)
    mut = [torch.tensor(m, dtype=torch.float64, requires_grad=True) for m in mus]
    opts = dict(method="coupled", precision=0, rtol=1e-12)
    us = [StokesSolve.apply(ft, m, P, opts)[0] for m in mut]
    assert P.mu == mus[1]
    loss = sum(0.5 * ((u - target) ** 2).sum() for u in us)
    loss.backward()
    assert P.mu == mus[1]
    gf = np.zeros_like(f)
    for m, u, mt in zip(mus, us, mut):
        Sm = ostokes.StokesSystem(mesh_, m, ALPHA)
        un = u.detach().cpu().numpy()
        dJdf, dJdmu, _, _ = Sm.adjoint_gradient(un, un - ut)
        gf += dJdf
        assert abs(float(mt.grad) - dJdmu) <= 1e-8 * abs(dJdmu), (m, float(mt.grad), dJdmu)
    assert _rel(ft.grad.cpu().numpy(), gf) <= 1e-8
    P.set_mu(MU)
