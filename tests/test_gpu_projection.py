"""GPU pressure-correction step (stokes_projection_step, the comparator of
Sec. 7.5) against the oracle's step: FP64 to 1e-10, mixed to 1e-8 (each of
the three solves at rel-res 1e-12 / 1e-11), with Dirichlet data and a given
p_old; the coupled solution is its fixed point."""

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


@pytest.mark.parametrize("dim,n,strain", [(2, 6, False), (3, 4, False), (3, 4, True)])
@pytest.mark.parametrize("precision,rtol,tol", [(0, 1e-13, 1e-10), (1, 1e-12, 1e-8)])
@pytest.mark.parametrize("vel_pc", [0, 1])
def test_projection_step_matches_oracle(gpu_lib, dim, n, strain, precision, rtol, tol, vel_pc):
    from paper_2407_01783_amd.stokes import StokesProblem
    print(f"[case] projection dim={dim} n={n} strain={strain} precision={precision} vel_pc={vel_pc}", flush=True)
    mu, alpha = 0.3, 60.0
    P = StokesProblem(dim, n, mesh_seed=8, jitter=0.1, mu=mu, alpha=alpha, strain=strain)
    S = ostokes.StokesSystem(omesh.KuhnMesh(dim, n, seed=8, jitter=0.1), mu, alpha, strain=strain)
    rng = np.random.default_rng(12)
    f = inputs.fourier_forcing(S.mesh.p2coords, 1008)
    ubc = rng.standard_normal((dim, P.n_p2))
    p_old = rng.standard_normal(P.n_p1)
    U, Pp = S.projection_step(f, ubc, p_old)
    u, p, info = P.projection_step(torch.tensor(f[None], device="cuda"), torch.tensor(p_old[None], device="cuda"),
                                   torch.tensor(ubc[None], device="cuda"), precision=precision, rtol=rtol,
                                   vel_pc=vel_pc, max_inner=5000, max_refine=30)
    assert info["status"] == 0 and info["rel_res"] <= rtol, info
    assert _rel(u.cpu().numpy()[0], S.full_velocity(U, ubc)) <= tol
    assert _rel(p.cpu().numpy()[0], Pp) <= tol


def test_coupled_solution_is_fixed_point(gpu_lib):
    from paper_2407_01783_amd.stokes import StokesProblem
    P = StokesProblem(3, 4, mesh_seed=9, jitter=0.1, mu=0.1, alpha=80.0)
    xy, _ = P.mesh()
    f = torch.tensor(inputs.fourier_forcing(xy, 1009)[None], device="cuda")
    u, p, info = P.solve(f, method="coupled", precision=0, rtol=1e-13)
    assert info["status"] == 0
    u2, p2, info2 = P.projection_step(f, p, precision=0, rtol=1e-13)
    assert info2["status"] == 0
    assert _rel(u2.cpu().numpy(), u.cpu().numpy()) <= 1e-10
    assert _rel(p2.cpu().numpy(), p.cpu().numpy()) <= 1e-9
