"""Full-size checks on the benchmark workload (3D unit cube, 64^3 cells, Kuhn
tetrahedra, jitter 0.1 h seed 1, mu = 1e-3, dt = 5e-3: 6,714,692 DOFs), in the
solver configuration the benchmark times.

The oracle cannot solve this size in seconds, so it checks sampled outputs it
computes one by one from the incident elements:
* mesh coordinates and connectivity: bit-exact, every entry;
* rows of the assembled M_s and L_s: same columns, values within 1e-13 of
  the row's largest magnitude;
* rows of the coupled operator (A u - B^T p, B u) in FP64 (1e-12) and FP32
  (2e-6), relative to the sampled reference norm;
* the solution: the oracle's residual rows, scaled to a norm estimate, stay
  below 2 x 1e-8 of the right-hand-side norm estimate (the solver stops at
  a true relative residual of 1e-8; the factor 2 covers the sampling).
"""

import os
import sys

import numpy as np
import pytest

from oracle import fem as ofem
from oracle import mesh as omesh
from paper_2407_01783_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402  (the workload table and solver options it times)

DIM, N, SEED, MU, DT, FSEED, _ = bench.WORKLOADS["cube64"]
ALPHA = 1.0 / DT


@pytest.fixture(scope="module")
def cube64(gpu_lib):
    from paper_2407_01783_amd.stokes import StokesProblem
    print(f"[case] full size dim={DIM} n={N} seed={SEED} mu={MU} alpha={ALPHA}", flush=True)
    prob = StokesProblem(DIM, N, mesh_seed=SEED, jitter=0.1, mu=MU, alpha=ALPHA)
    m = omesh.KuhnMesh(DIM, N, seed=SEED, jitter=0.1)
    return prob, m


def _sample(rng, pool, k):
    return np.sort(rng.choice(pool, size=k, replace=False))


def test_fullsize_mesh_bit_exact(cube64):
    prob, m = cube64
    xy, p2 = prob.mesh()
    assert xy.shape == m.p2coords.shape and np.array_equal(xy, m.p2coords)
    assert np.array_equal(p2, m.p2)


def test_fullsize_matrix_rows(cube64):
    prob, m = cube64
    rng = np.random.default_rng(11)
    rows = np.concatenate([_sample(rng, m.n_p2, 40), [0, m.n_p2 - 1, m.interior_nodes[0]]])
    ref = ofem.assemble_rows(m, rows)
    for which, k in ((0, 1), (1, 2)):   # 0: M_s, 1: L_s (all P2 nodes)
        rp, cols, vals = prob.export_csr(which)
        for r in rows:
            rc, rv = cols[rp[r]:rp[r + 1]], vals[rp[r]:rp[r + 1]]
            assert np.array_equal(rc, ref[r][0]), (which, r)
            assert np.abs(rv - ref[r][k]).max() <= 1e-13 * np.abs(ref[r][k]).max(), (which, r)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-6)])
def test_fullsize_coupled_operator_rows(cube64, precision, tol):
    prob, m = cube64
    rng = np.random.default_rng(5 + precision)
    u = rng.standard_normal((DIM, m.n_p2))
    u[:, m.p2_boundary] = 0.0          # the operator ignores boundary entries
    p = rng.standard_normal(m.n_p1)
    x = torch.tensor(np.concatenate([u.ravel(), p]), device="cuda")
    y = prob.apply(5, x, precision=precision).cpu().numpy()
    yu, yp = y[:DIM * m.n_p2].reshape(DIM, m.n_p2), y[DIM * m.n_p2:]
    nodes = _sample(rng, m.interior_nodes, 60)
    vrows = [(c, i) for c in range(DIM) for i in nodes]
    prow = _sample(rng, m.n_p1, 60)
    rm, rpr, _ = ofem.residual_rows(m, MU, ALPHA, np.zeros((DIM, m.n_p2)), u, p, vrows, prow)
    got_u = np.array([yu[c, i] for c, i in vrows])
    assert np.linalg.norm(got_u + rm) <= tol * np.linalg.norm(rm)
    assert np.linalg.norm(yp[prow] + rpr) <= tol * np.linalg.norm(rpr)


@pytest.mark.parametrize("precision", [1, 0])
def test_fullsize_benchmark_solve_residual_rows(cube64, precision):
    prob, m = cube64
    opts = dict(bench.SOLVER)
    method = opts.pop("method")
    f = inputs.fourier_forcing(m.p2coords, FSEED)
    u, p, info = prob.solve(torch.tensor(f[None], device="cuda"), method=method, precision=precision, **opts)
    print(f"[solve] precision={precision} {info}", flush=True)
    assert info["status"] == 0 and info["rel_res"] <= opts["rtol"]
    uf, pp = u.cpu().numpy()[0], p.cpu().numpy()[0]
    assert np.all(uf[:, m.p2_boundary] == 0.0)
    rng = np.random.default_rng(17 + precision)
    nodes = _sample(rng, m.interior_nodes, 120)
    vrows = [(c, i) for c in range(DIM) for i in nodes]
    prow = _sample(rng, m.n_p1, 120)
    rm, rpr, rf = ofem.residual_rows(m, MU, ALPHA, f, uf, pp, vrows, prow)
    n_u, n_p = DIM * m.n_free_nodes, m.n_p1
    res_est = np.sqrt(n_u * np.mean(rm ** 2) + n_p * np.mean(rpr ** 2))
    rhs_est = np.sqrt(n_u * np.mean(rf ** 2))
    print(f"[solve] sampled residual estimate {res_est / rhs_est:.2e}", flush=True)
    assert res_est <= 2.0 * opts["rtol"] * rhs_est


# ------------------------------------------------------- error vs the oracle
# tests/golden/cube64_oracle.txt holds the FP64 oracle solution of this
# workload (MINRES at rtol 1e-14 plus a correction sweep, written by
# tests/golden/make_cube64_golden.py, which calls only oracle/) on the nodes of
# 400 seeded elements.  The relative error in the M-norm (the paper's error
# measure; u in M_V = I_3 (x) M_s, p in M_Q) is estimated on those elements:
#     sum_K e_K^T M_K e_K / sum_K u_K^T M_K u_K
# with the oracle's element mass matrices.  Bars: 1e-8 for the mixed path
# solved to rel-res 1e-10 (the parity setting).  The benchmark's own solve at
# rel-res 1e-8 has its error reported, with a bar of 10 x rtol: the error can
# exceed the relative residual by up to the condition number of the coupled
# operator (about 4x here: 1.7e-8 at rel-res 4.4e-9).

GOLDEN = os.path.join(ROOT, "tests", "golden", "cube64_oracle.txt")


def _read_golden():
    out = {}
    with open(GOLDEN) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    it = iter(lines)
    for ln in it:
        key, val = ln.split()[:2]
        if key in ("rel_res", "unorm_M", "pnorm_MQ"):
            out[key] = float(val)
        elif key == "elems":
            out["elems"] = np.array([int(v) for v in next(it).split()])
        elif key == "vel":
            rows = [next(it).split() for _ in range(int(val))]
            out["vel"] = {int(r[0]): np.array([float(v) for v in r[1:]]) for r in rows}
        elif key == "p":
            rows = [next(it).split() for _ in range(int(val))]
            out["p"] = {int(r[0]): float(r[1]) for r in rows}
    return out


@pytest.mark.parametrize("rtol,bar", [(1e-8, 1e-7), (1e-10, 1e-8)])
def test_fullsize_error_vs_oracle_m_norm(cube64, rtol, bar):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden oracle solution not generated")
    prob, m = cube64
    gold = _read_golden()
    assert gold["rel_res"] <= 1e-12
    opts = dict(bench.SOLVER, rtol=rtol)
    method = opts.pop("method")
    f = inputs.fourier_forcing(m.p2coords, FSEED)
    u, p, info = prob.solve(torch.tensor(f[None], device="cuda"), method=method, precision=1, **opts)
    print(f"[solve] rtol={rtol} {info}", flush=True)
    assert info["status"] == 0 and info["rel_res"] <= rtol
    uf, pp = u.cpu().numpy()[0], p.cpu().numpy()[0]
    nu = du = npp = dpp = 0.0
    for e in gold["elems"]:
        em = ofem.element_matrices(m, int(e))
        nodes, verts = m.p2[e], m.elems[e]
        ug = np.stack([gold["vel"][int(v)] for v in nodes], axis=1)   # (3, 10)
        eu = uf[:, nodes] - ug
        du += float(np.einsum("ci,ij,cj->", eu, em["M"], eu))
        nu += float(np.einsum("ci,ij,cj->", ug, em["M"], ug))
        pg = np.array([gold["p"][int(v)] for v in verts])
        ep = pp[verts] - pg
        dpp += float(ep @ em["MQ"] @ ep)
        npp += float(pg @ em["MQ"] @ pg)
    err_u, err_p = np.sqrt(du / nu), np.sqrt(dpp / npp)
    # the sampled norms scale to the oracle's global norms (a check that the
    # sample and the golden values belong together)
    frac = len(gold["elems"]) / m.n_e
    assert 0.5 < np.sqrt(nu / frac) / gold["unorm_M"] < 2.0
    print(f"[error] rtol={rtol}: M-norm relative error u {err_u:.3e}, p {err_p:.3e} "
          f"(rel res {info['rel_res']:.2e})", flush=True)
    assert err_u <= bar and err_p <= bar, (err_u, err_p)


# ------------------------------------------------------------------ cube32 sweep
# 3D n = 32 (jitter seed 0, dt = 1e-2, forcing seed 1000): both methods and
# the preconditioner variants across the paper's mu range, with and without
# the augmented Lagrangian (the solution does not depend on gamma); every
# solve is checked on sampled residual rows of the plain system.

C2_N, C2_SEED, C2_DT, C2_FSEED = 32, 0, 1e-2, 1000


@pytest.fixture(scope="module")
def cube32_mesh():
    return omesh.KuhnMesh(3, C2_N, seed=C2_SEED, jitter=0.1)


def _sampled_rel_res(m, mu, alpha, f, uf, pp, seed):
    rng = np.random.default_rng(seed)
    nodes = _sample(rng, m.interior_nodes, 100)
    vrows = [(c, i) for c in range(3) for i in nodes]
    prow = _sample(rng, m.n_p1, 100)
    rm, rpr, rf = ofem.residual_rows(m, mu, alpha, f, uf, pp, vrows, prow)
    n_u, n_p = 3 * m.n_free_nodes, m.n_p1
    return np.sqrt(n_u * np.mean(rm ** 2) + n_p * np.mean(rpr ** 2)) / np.sqrt(n_u * np.mean(rf ** 2))


C2_CASES = [
    # (method, precision, options)
    ("coupled", 1, dict(coupled_pc=1, inner_mode=1, cheb_degree=6)),
    ("coupled", 0, dict(coupled_pc=0)),   # full block factorisation (Sec. 2.4)
    ("coupled", 0, dict(coupled_pc=1)),   # upper block triangular
    ("coupled", 0, dict(coupled_pc=2)),   # lower block triangular, the "incomplete Full" of Sec. 6.2
    ("schur", 0, dict(schur_pc=1)),
]


@pytest.mark.parametrize("mu", [1.0, 1e-2, 1e-4])
@pytest.mark.parametrize("gamma", [0.0, 1.0, 10.0])
@pytest.mark.parametrize("case", range(len(C2_CASES)))
def test_cube32_mu_gamma_sweep_residual_rows(gpu_lib, cube32_mesh, mu, gamma, case):
    from paper_2407_01783_amd.stokes import StokesProblem
    method, precision, extra = C2_CASES[case]
    m = cube32_mesh
    alpha = 1.0 / C2_DT
    print(f"[case] cube32 mu={mu} gamma={gamma} {method} precision={precision} {extra}", flush=True)
    prob = StokesProblem(3, C2_N, mesh_seed=C2_SEED, jitter=0.1, mu=mu, alpha=alpha, gamma=gamma)
    f = inputs.fourier_forcing(m.p2coords, C2_FSEED)
    # the augmented velocity block at mu = 1 is the hard case of the paper
    # (its condition number grows with gamma): allow more refinement sweeps
    u, p, info = prob.solve(torch.tensor(f[None], device="cuda"), method=method, precision=precision, rtol=1e-8,
                            max_outer=3000, max_refine=40, **extra)
    print(f"[solve] {info}", flush=True)
    assert info["status"] == 0 and info["rel_res"] <= 1e-8
    est = _sampled_rel_res(m, mu, alpha, f, u.cpu().numpy()[0], p.cpu().numpy()[0], 31)
    assert est <= 2e-8, est


# ------------------------------------------------------------- adjoint, 64^3
# 3D n = 64 (jitter seed 3, mu = 1e-2, dt = 1e-2, forcing seed 1003): the
# gradient of J(f) = 1/2 (u - u*)^T M_V (u - u*) from the adjoint solve
# against central finite differences of forward solves (rtol 1e-13) on 16
# seeded directions, and dJ/dmu against a central difference in mu (step
# 1e-4 mu: truncation O(1e-8) relative, rounding noise O(1e-13 / 1e-4)).
# Both the FP64 path and the mixed path (FP32 inner solves, FP64 refinement)
# run the forward and adjoint solves.  M_V is the oracle's mass matrix; u* is
# the solution for the seeded target forcing (seed 9003), solved on the GPU
# in FP64 to rtol 1e-13 (an oracle solve at this size takes tens of minutes;
# any fixed u* serves the finite-difference check).


@pytest.fixture(scope="module")
def c5_mass():
    from oracle import fem
    n, seed = 64, 3
    print(f"[case] adjoint n={n} seed={seed}: oracle assembly of M_V", flush=True)
    m = omesh.KuhnMesh(3, n, seed=seed, jitter=0.1)
    return m, fem.assemble(m).Ms


@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_gradient_finite_differences_64(gpu_lib, c5_mass, precision):
    from paper_2407_01783_amd.stokes import StokesProblem
    n, seed, mu, alpha = 64, 3, 1e-2, 100.0
    m, Ms = c5_mass
    print(f"[case] adjoint n={n} seed={seed} mu={mu} alpha={alpha} precision={precision}", flush=True)
    P = StokesProblem(3, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha)
    x = m.p2coords
    fwd = dict(method="coupled", precision=precision, rtol=1e-13, max_outer=3000, max_refine=40)
    ut_dev, _, info_t = P.solve(torch.tensor(inputs.fourier_forcing(x, inputs.target_seed(seed))[None],
                                             device="cuda"), method="coupled", precision=0, rtol=1e-13,
                                max_outer=3000)
    assert info_t["status"] == 0, info_t
    ut = ut_dev.cpu().numpy()[0]
    f = inputs.fourier_forcing(x, inputs.forcing_seed(seed, 0))

    def J(fv, mu_v=None):
        if mu_v is not None:
            P.set_mu(mu_v)
        u, _, info = P.solve(torch.tensor(fv[None], device="cuda"), **fwd)
        assert info["status"] == 0, info
        d = u.cpu().numpy()[0] - ut
        return 0.5 * float(sum(d[c] @ (Ms @ d[c]) for c in range(3))), u, d

    J0, u, d = J(f)
    dJdu = np.stack([Ms @ d[c] for c in range(3)])
    _, _, gf, gmu, info = P.adjoint(u, torch.tensor(dJdu[None], device="cuda"), precision=precision, rtol=1e-13,
                                    max_outer=3000, max_refine=40)
    assert info["status"] == 0, info
    gf, gmu = gf.cpu().numpy()[0], float(gmu[0])
    h = 1e-3
    for j, dj in enumerate(inputs.fd_directions(f.shape, 16, 1003)):
        fd = (J(f + h * dj)[0] - J(f - h * dj)[0]) / (2 * h)
        an = float(np.sum(dj * gf))
        print(f"[fd] direction {j}: fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12 * J0, (j, fd, an)
    hm = 1e-4 * mu
    fdm = (J(f, mu + hm)[0] - J(f, mu - hm)[0]) / (2 * hm)
    P.set_mu(mu)
    print(f"[fd] mu: fd {fdm:.10e} adjoint {gmu:.10e} rel {abs(fdm - gmu) / abs(fdm):.2e}", flush=True)
    assert abs(fdm - gmu) <= 1e-6 * abs(fdm), (fdm, gmu)


# --------------------------------------------------------- 128^3, 8 rhs batched
# The batched workload (3D n = 128, jitter seed 2, mu = 1e-4, dt = 2e-3,
# forcing seeds 1002 + 100 b, b < 8) in the benchmark's solver configuration;
# every right-hand side is checked on the oracle's sampled residual rows.


def test_cube128_eight_rhs_batched_residual_rows(gpu_lib):
    from paper_2407_01783_amd.stokes import StokesProblem
    dim, n, seed, mu, dt, fseed, _ = bench.WORKLOADS["cube128"]
    alpha = 1.0 / dt
    opts = dict(bench.SOLVER)
    opts.update(bench.WORKLOAD_SOLVER["cube128"])
    method = opts.pop("method")
    print(f"[case] cube128 x 8 rhs mu={mu} alpha={alpha} {opts}", flush=True)
    m = omesh.KuhnMesh(dim, n, seed=seed, jitter=0.1)
    P = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha)
    fs = [inputs.fourier_forcing(m.p2coords, inputs.forcing_seed(seed, b)) for b in range(8)]
    assert inputs.forcing_seed(seed, 0) == fseed
    u, p, info = P.solve(torch.tensor(np.stack(fs), device="cuda"), method=method, precision=1, **opts)
    print(f"[solve] {info}", flush=True)
    assert info["status"] == 0 and info["rel_res"] <= opts["rtol"]
    un, pn = u.cpu().numpy(), p.cpu().numpy()
    del u, p
    for b in range(8):
        est = _sampled_rel_res(m, mu, alpha, fs[b], un[b], pn[b], 100 + b)
        print(f"[solve] rhs {b}: sampled residual estimate {est:.2e}", flush=True)
        assert est <= 2.0 * opts["rtol"], (b, est)
