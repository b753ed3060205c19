"""Pins of the FP64 CPU oracle against facts the mathematics fixes.

Each test checks the oracle by a route other than its own code: published
generator outputs, closed forms, an independent nodal-interpolation +
Gauss-quadrature construction of the element matrices, invariants of the
continuous operators, dense least squares, the paper's exact block
factorisation and augmented-Lagrangian identity (Sec. 2.3, 2.4), manufactured
convergence rates and finite differences.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse as sp

from oracle import fem, mesh, stokes
from paper_2407_01783_amd import inputs


# ----------------------------------------------------------------- generators


def test_splitmix64_published_outputs():
    # SplitMix64 from state 0 (Steele, Lea & Flood 2014): first two outputs.
    assert int(mesh.splitmix64_mix(np.uint64(0x9E3779B97F4A7C15))) == 0xE220A8397B1DCDAF
    assert int(mesh.splitmix64_mix(np.uint64((2 * 0x9E3779B97F4A7C15) % 2 ** 64))) == 0x6E789E6AA1B965F4
    assert int(mesh.jitter_unit(0, 0) * 2 ** 53) == 0xE220A8397B1DCDAF >> 11
    r = inputs.SplitMix64(0)
    assert r.next_u64() == 0xE220A8397B1DCDAF
    assert r.next_u64() == 0x6E789E6AA1B965F4


# ----------------------------------------------------------------------- mesh


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 3), (2, 16), (3, 1), (3, 2), (3, 5)])
def test_mesh_counts_and_volume(dim, n):
    m = mesh.KuhnMesh(dim, n, seed=7, jitter=0.1)
    assert m.n_e == math.factorial(dim) * n ** dim
    assert m.n_p1 == (n + 1) ** dim
    assert m.n_p2 == (2 * n + 1) ** dim
    assert m.n_free_nodes == (2 * n - 1) ** dim
    vol, _, detJ = fem.element_geometry(m)
    assert abs(vol.sum() - 1.0) < 1e-13
    m0 = mesh.KuhnMesh(dim, n, seed=7, jitter=0.0)
    _, _, det0 = fem.element_geometry(m0)
    assert np.all(np.sign(detJ) == np.sign(det0))       # no inverted simplex
    assert np.all(np.abs(det0) > 0)
    assert np.allclose(vol, vol.mean()) or n > 1        # jitter changes volumes


def test_mesh_unjittered_coordinates_and_midpoints():
    m = mesh.KuhnMesh(3, 3, seed=1, jitter=0.0)
    assert np.array_equal(m.vcoords, m.vgrid / 3.0)
    assert np.allclose(m.p2coords, m.p2grid / 6.0, atol=0, rtol=1e-15)
    mj = mesh.KuhnMesh(3, 3, seed=1, jitter=0.1)
    bnd = np.any((mj.vgrid == 0) | (mj.vgrid == 3), axis=1)
    assert np.array_equal(mj.vcoords[bnd], m.vcoords[bnd])        # boundary does not move
    shift = (mj.vcoords - m.vcoords) * 3.0
    assert np.all(np.abs(shift) <= 0.1 + 1e-12) and np.abs(shift[~bnd]).max() > 0.05
    # every edge node is the midpoint of its edge's two vertices
    for q, (a, b) in enumerate(mesh.local_edges(3)):
        node = mj.p2[:, 4 + q]
        mid = (mj.vcoords[mj.elems[:, a]] + mj.vcoords[mj.elems[:, b]]) * 0.5
        assert np.array_equal(mj.p2coords[node], mid)


def test_jitter_counter_layout():
    # x_c of vertex g uses counter d*g + c: check one interior vertex by hand.
    n, seed, jit = 4, 123, 0.1
    m = mesh.KuhnMesh(3, n, seed=seed, jitter=jit)
    g = 1 + 5 * (2 + 5 * 3)                     # vertex (1, 2, 3)
    for c, ic in enumerate((1, 2, 3)):
        z = (seed + (3 * g + c + 1) * 0x9E3779B97F4A7C15) % 2 ** 64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % 2 ** 64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % 2 ** 64
        z ^= z >> 31
        u = (z >> 11) * 2.0 ** -53
        assert m.vcoords[g, c] == (ic + (2.0 * u - 1.0) * jit) / n


def test_pattern_sizes_closed_form():
    # nnz of the interior scalar P2 matrix, of one B plane (pressure rows x
    # interior velocity columns) and of the P1 matrices on the Kuhn cube.
    for n in (2, 3, 4, 6):
        s = stokes.StokesSystem(mesh.KuhnMesh(3, n), 1.0, 1.0)
        assert s.A_II.nnz == 230 * n ** 3 - 690 * n ** 2 + 732 * n - 273
        assert s.B_I[0].nnz == 65 * n ** 3 - 111 * n ** 2 + 69 * n - 15
        assert s.mats.MQ.nnz == 15 * n ** 3 + 21 * n ** 2 + 9 * n + 1


# ---------------------------------------------------------- element matrices


def _duffy_rule(dim, q=6):
    """Gauss-Legendre tensor rule collapsed onto the reference simplex."""
    x, w = np.polynomial.legendre.leggauss(q)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    pts, wts = [], []
    for idx in itertools.product(range(q), repeat=dim):
        u = [x[i] for i in idx]
        ww = np.prod([w[i] for i in idx])
        if dim == 2:
            xi = (u[0], u[1] * (1 - u[0]))
            jac = 1 - u[0]
        else:
            xi = (u[0], u[1] * (1 - u[0]), u[2] * (1 - u[0]) * (1 - u[1]))
            jac = (1 - u[0]) ** 2 * (1 - u[1])
        pts.append(xi)
        wts.append(ww * jac)
    return np.array(pts), np.array(wts)


def _monomials(dim, deg):
    return [e for e in itertools.product(range(deg + 1), repeat=dim) if sum(e) <= deg]


def _lagrange(nodes, deg):
    """Coefficients of the nodal Lagrange basis in monomials of degree <= deg."""
    mons = _monomials(nodes.shape[1], deg)
    V = np.array([[np.prod(p ** np.array(e)) for e in mons] for p in nodes])
    return mons, np.linalg.inv(V)       # column i of inv(V) = coefficients of phi_i


def _eval(mons, C, x):
    vals = np.array([np.prod(x ** np.array(e)) for e in mons])
    grads = []
    for c in range(x.size):
        g = []
        for e in mons:
            if e[c] == 0:
                g.append(0.0)
            else:
                e2 = list(e)
                e2[c] -= 1
                g.append(e[c] * np.prod(x ** np.array(e2)))
        grads.append(g)
    return vals @ C, np.array(grads) @ C          # (nb,), (dim, nb)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrices_vs_nodal_quadrature(dim):
    m = mesh.KuhnMesh(dim, 3, seed=11, jitter=0.1)
    pts, wts = _duffy_rule(dim)
    for e in (0, 7, m.n_e - 1):
        X = m.vcoords[m.elems[e]]
        J = np.stack([X[a + 1] - X[0] for a in range(dim)], axis=1)
        nodes2 = np.vstack([X] + [0.5 * (X[a] + X[b]) for a, b in mesh.local_edges(dim)])
        mons2, C2 = _lagrange(nodes2, 2)
        mons1, C1 = _lagrange(X, 1)
        nl, nv = nodes2.shape[0], dim + 1
        M, L = np.zeros((nl, nl)), np.zeros((nl, nl))
        Dq = np.zeros((dim, dim, nl, nl))
        B = np.zeros((dim, nv, nl))
        MQ, LQ = np.zeros((nv, nv)), np.zeros((nv, nv))
        absphi = np.zeros(nl)
        detJ = abs(np.linalg.det(J))
        for xi, w in zip(pts, wts):
            x = X[0] + J @ xi
            p2, g2 = _eval(mons2, C2, x)
            p1, g1 = _eval(mons1, C1, x)
            ww = w * detJ
            M += ww * np.outer(p2, p2)
            L += ww * g2.T @ g2
            Dq += ww * np.einsum("ai,bj->abij", g2, g2)
            for c in range(dim):
                B[c] += ww * np.outer(p1, g2[c])
            MQ += ww * np.outer(p1, p1)
            LQ += ww * g1.T @ g1
        em = fem.element_matrices(m, e)
        scale = np.abs(em["M"]).max()
        assert np.allclose(em["M"], M, rtol=0, atol=1e-13 * scale)
        assert np.allclose(em["L"], L, rtol=0, atol=1e-12 * np.abs(L).max())
        assert np.allclose(em["D"], Dq, rtol=0, atol=1e-12 * np.abs(Dq).max())   # grad-div blocks
        assert np.allclose(em["B"], B, rtol=0, atol=1e-12 * np.abs(B).max())
        assert np.allclose(em["MQ"], MQ, rtol=0, atol=1e-13 * np.abs(MQ).max())
        assert np.allclose(em["LQ"], LQ, rtol=0, atol=1e-12 * np.abs(LQ).max())
        # P1 mass closed form |K| (1 + delta_kl) / ((d+1)(d+2))
        vol = detJ / math.factorial(dim)
        assert np.allclose(em["MQ"], vol * (np.ones((nv, nv)) + np.eye(nv)) / ((dim + 1) * (dim + 2)),
                           rtol=1e-14, atol=0)
        del absphi


@pytest.mark.parametrize("dim", [2, 3])
def test_lumped_abs_mass_closed_form_and_quadrature(dim):
    ref = fem.reference_tensors(dim)
    # Closed forms: int |phi_vertex| / |K| = 3/32 (3D), 1/8 (2D); edges 1/5, 1/3.
    want_v, want_e = (3 / 32, 1 / 5) if dim == 3 else (1 / 8, 1 / 3)
    assert np.allclose(ref["absphi"][: dim + 1], want_v, rtol=1e-15)
    assert np.allclose(ref["absphi"][dim + 1:], want_e, rtol=1e-15)
    # numerical quadrature of the 1D marginal integral, split at the kink
    dens = lambda t: dim * (1 - t) ** (dim - 1)  # noqa: E731
    f = lambda t: abs(t * (2 * t - 1)) * dens(t)  # noqa: E731
    val = scipy.integrate.quad(f, 0, 0.5, epsabs=1e-15)[0] + scipy.integrate.quad(f, 0.5, 1, epsabs=1e-15)[0]
    assert abs(val - ref["absphi"][0]) < 1e-13
    # row sums of the mass = integral of each basis function (partition of unity)
    assert np.allclose(ref["M"].sum(axis=1), ref["phi"], atol=1e-15)
    assert np.allclose(ref["phi"][: dim + 1], -1 / 20 if dim == 3 else 0.0, atol=1e-15)


# --------------------------------------------------------- global invariants


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2), (3, 3)])
def test_global_invariants(dim, n):
    m = mesh.KuhnMesh(dim, n, seed=3, jitter=0.1)
    mats = fem.assemble(m)
    for A in (mats.Ms, mats.Ls, mats.MQ, mats.LQ):
        assert abs(A - A.T).max() <= 1e-15 * abs(A).max()     # symmetric to rounding
    one2, one1 = np.ones(m.n_p2), np.ones(m.n_p1)
    assert abs(one2 @ mats.Ms @ one2 - 1.0) < 1e-13
    assert abs(one1 @ mats.MQ @ one1 - 1.0) < 1e-13
    assert np.abs(mats.Ls @ one2).max() < 1e-11
    assert np.abs(mats.LQ @ one1).max() < 1e-12
    for c in range(dim):
        assert np.abs(mats.B[c] @ one2).max() < 1e-15     # div(const) = 0
        xc = m.p2coords[:, c]
        assert np.allclose(mats.B[c] @ xc, mats.MQ @ one1, atol=1e-15)   # div(x_c e_c) = 1
    s = stokes.StokesSystem(m, 1.0, 10.0)
    for c in range(dim):
        assert np.abs(s.B_I[c].T @ one1).max() < 1e-15    # B_I^T 1 = 0 (Dirichlet)
    Bm = sp.hstack(s.B_I).toarray()
    assert np.linalg.matrix_rank(Bm) == m.n_p1 - 1
    # Lambda_V: total |phi| mass and positivity
    assert np.all(mats.Lam > 0)


def test_assembly_rows_match_element_sums():
    m = mesh.KuhnMesh(3, 3, seed=5, jitter=0.1)
    mats = fem.assemble(m)
    rows = [0, 17, m.n_p2 // 2, m.n_p2 - 1]
    for r, (cols, mv, lv) in fem.assemble_rows(m, rows).items():
        Mr, Lr = mats.Ms[r], mats.Ls[r]
        assert np.array_equal(Mr.indices, cols)
        assert np.allclose(Mr.data, mv, rtol=1e-14, atol=1e-18)
        assert np.allclose(Lr.data, lv, rtol=1e-13, atol=1e-14)


def test_residual_rows_match_assembled_system():
    """Row-by-row residuals (used at full size) == the assembled operators;
    and they vanish on a direct solution with Dirichlet data."""
    for dim, n in ((2, 4), (3, 3)):
        m = mesh.KuhnMesh(dim, n, seed=2, jitter=0.1)
        mats = fem.assemble(m)
        rng = np.random.default_rng(dim)
        mu, alpha = 0.3, 7.0
        f = rng.standard_normal((dim, m.n_p2))
        u = rng.standard_normal((dim, m.n_p2))
        p = rng.standard_normal(m.n_p1)
        A = alpha * mats.Ms + mu * mats.Ls
        mom = np.stack([mats.Ms @ f[c] - A @ u[c] + mats.B[c].T @ p for c in range(dim)])
        con = -sum(mats.B[c] @ u[c] for c in range(dim))
        vrows = [(c, i) for c in range(dim) for i in (0, 5, m.n_p2 // 2, m.n_p2 - 2)]
        prow = [0, 3, m.n_p1 - 1]
        rm, rp, rf = fem.residual_rows(m, mu, alpha, f, u, p, vrows, prow)
        assert np.allclose(rm, [mom[c, i] for c, i in vrows], rtol=1e-12, atol=1e-12)
        assert np.allclose(rp, con[prow], rtol=1e-12, atol=1e-13)
        assert np.allclose(rf, [(mats.Ms @ f[c])[i] for c, i in vrows], rtol=1e-13, atol=1e-14)
        # at a solution with nonzero Dirichlet data every interior row vanishes
        s = stokes.StokesSystem(m, mu, alpha, mats=mats)
        ubc = rng.standard_normal((dim, m.n_p2))
        ubc[:, m.interior_nodes] = 0
        F, g = s.rhs(f, ubc)
        U, P = s.solve_direct(F, g)
        uf = s.full_velocity(U, ubc)
        inner = [(c, int(i)) for c in range(dim) for i in m.interior_nodes[[0, -1]]]
        rm, rp, _ = fem.residual_rows(m, mu, alpha, f, uf, P, inner, range(m.n_p1))
        scale = np.abs(F).max()
        assert np.abs(rm).max() <= 1e-10 * scale
        # continuity holds up to the l2-mean removed from g (compatibility)
        assert np.abs(rp - rp.mean()).max() <= 1e-10 * scale


def test_grad_div_identities():
    """The grad-div blocks D[a][b]_ij = int d_a phi_i d_b phi_j against facts
    that do not depend on how they were computed:
    * H^1_0 identity (integration by parts twice, Sec. 3.2): for interior
      nodes i, j, int d_b phi_i d_a phi_j = int d_a phi_i d_b phi_j, i.e.
      D[b][a]_II = D[a][b]_II -- but not between two boundary nodes;
    * rigid motions have zero strain: (I (x) L_s + T) u = 0 on every row, with
      T[a][b] = D[b][a] the transposed-gradient form;
    * a divergence-free linear field u = (y, z, x) has D u = 0 on every row;
    * sum_a D[a][a] restricted to one component of a linear field x_a e_a
      gives int d_a phi_i = 0 for interior i."""
    for dim, n in ((2, 4), (3, 3)):
        m = mesh.KuhnMesh(dim, n, seed=4, jitter=0.15)
        mats = fem.assemble(m, grad_div=True)
        D, I = mats.D, m.interior_nodes
        scale = max(abs(D[a][b]).max() for a in range(dim) for b in range(dim))
        for a in range(dim):
            for b in range(dim):
                assert abs(D[a][b] - D[b][a].T).max() <= 1e-14 * scale          # symmetric operator
                dII = (D[a][b][I][:, I] - D[b][a][I][:, I])
                assert abs(dII).max() <= 1e-12 * scale, (a, b)
        Gm = np.nonzero(m.p2_boundary)[0]                                          # both nodes on the boundary:
        assert abs(D[0][1][Gm][:, Gm] - D[1][0][Gm][:, Gm]).max() > 1e-3 * scale  # the identity fails
        x = m.p2coords
        rigid = [np.stack([-x[:, 1], x[:, 0]] + ([np.zeros(m.n_p2)] if dim == 3 else []))]
        if dim == 3:
            rigid += [np.stack([np.zeros(m.n_p2), -x[:, 2], x[:, 1]]), np.stack([x[:, 2], np.zeros(m.n_p2), -x[:, 0]])]
        rigid += [np.stack([np.ones(m.n_p2) if c == k else np.zeros(m.n_p2) for c in range(dim)]) for k in range(dim)]
        lscale = abs(mats.Ls).max()
        for u in rigid:
            for a in range(dim):
                Eu = mats.Ls @ u[a] + sum(D[b][a] @ u[b] for b in range(dim))
                assert np.abs(Eu).max() <= 1e-12 * lscale * np.abs(u).max()
        cyc = np.stack([x[:, (c + 1) % dim] for c in range(dim)])                 # (y, x) / (y, z, x)
        for a in range(dim):
            assert np.abs(sum(D[a][b] @ cyc[b] for b in range(dim))).max() <= 1e-13 * scale
        for a in range(dim):
            assert np.abs((D[a][a] @ x[:, a])[I]).max() <= 1e-13 * scale


def test_strain_system_solutions_agree():
    """Strain form A = alpha M + mu (L + D): direct, dense least squares and
    MINRES reach the same solution, with Dirichlet data; the momentum residual
    vanishes row by row (residual_rows with the grad-div term)."""
    for dim, n in ((2, 3), (3, 2)):
        m = mesh.KuhnMesh(dim, n, seed=2, jitter=0.1)
        s = stokes.StokesSystem(m, 0.3, 20.0, strain=True)
        rng = np.random.default_rng(dim)
        f = inputs.fourier_forcing(m.p2coords, 1000 + dim)
        ubc = rng.standard_normal((dim, m.n_p2))
        F, g = s.rhs(f, ubc)
        U1, P1 = s.solve_direct(F, g)
        U2, P2 = s.solve_dense_lstsq(F, g)
        U3, P3, _ = s.solve_minres(F, g, rtol=1e-13)
        for U, P in ((U2, P2), (U3, P3)):
            assert np.abs(U - U1).max() <= 1e-9 * np.abs(U1).max()
            assert np.abs(P - P1).max() <= 1e-8 * np.abs(P1).max()
        assert s.residual(U1, P1, F, g) < 1e-12
        uf = s.full_velocity(U1, ubc)
        rows = [(c, int(i)) for c in range(dim) for i in m.interior_nodes]
        rm, _, _ = fem.residual_rows(m, s.mu, s.alpha, f, uf, P1, rows, [], strain=True)
        assert np.abs(rm).max() <= 1e-10 * np.abs(F).max()
        # the strain form differs from the vector-Laplacian form
        s0 = stokes.StokesSystem(m, 0.3, 20.0, mats=s.mats)
        U0, _ = s0.solve_direct(*s0.rhs(f, ubc))
        assert np.abs(U0 - U1).max() > 1e-6 * np.abs(U1).max()


def test_strain_manufactured_rates_2d():
    """For a divergence-free exact solution the strain form has the same
    forcing (-mu div(2 eps(u)) = -mu Lap u when div u = 0): O(h^3) / O(h^2)."""
    mu, alpha = 1.0, 100.0
    pi = math.pi

    def u_ex(x):
        return np.stack([np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]),
                         np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])], axis=1)

    def p_ex(x):
        return np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])

    errs = []
    for n in (4, 8, 16):
        m = mesh.KuhnMesh(2, n)
        s = stokes.StokesSystem(m, mu, alpha, strain=True)
        u, p, f = inputs.manufactured_2d(m.p2coords, mu, alpha)
        F, g = s.rhs(f, u)
        U, P = s.solve_direct(F, g)
        errs.append(_l2_errors_2d(m, s, U, P, u, u_ex, p_ex))
    ru = [math.log2(errs[i][0] / errs[i + 1][0]) for i in range(2)]
    rp = [math.log2(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert min(ru) > 2.7, (errs, ru)
    assert min(rp) > 1.7, (errs, rp)


def test_strain_adjoint_gradient_vs_finite_differences():
    m = mesh.KuhnMesh(3, 2, seed=6, jitter=0.1)
    s = stokes.StokesSystem(m, 0.4, 25.0, strain=True)
    f = inputs.fourier_forcing(m.p2coords, 1006)
    U, _ = s.solve_direct(*s.rhs(f))
    u = s.full_velocity(U)
    Ut, _ = s.solve_direct(*s.rhs(inputs.fourier_forcing(m.p2coords, 9006)))
    ut = s.full_velocity(Ut)
    _, dJdu = stokes.quadratic_loss(s, u, ut)
    dJdf, dJdmu, _, _ = s.adjoint_gradient(u, dJdu)

    def J_of(fv, mu):
        s2 = stokes.StokesSystem(m, mu, s.alpha, mats=s.mats, strain=True)
        U2, _ = s2.solve_direct(*s2.rhs(fv))
        return stokes.quadratic_loss(s2, s2.full_velocity(U2), ut)[0]

    for dvec in inputs.fd_directions(f.shape, 3, seed=8):
        h = 1e-3
        fd = (J_of(f + h * dvec, s.mu) - J_of(f - h * dvec, s.mu)) / (2 * h)
        assert abs(fd - np.sum(dJdf * dvec)) <= 1e-8 * abs(fd)
    h = 1e-5 * s.mu
    fd = (J_of(f, s.mu + h) - J_of(f, s.mu - h)) / (2 * h)
    assert abs(fd - dJdmu) <= 1e-6 * abs(fd)


def test_projection_step_fixed_point_and_pieces():
    """The coupled solution is the fixed point of the pressure-correction step
    (with p_old = P*, U = U* and the divergence data vanish); away from it the
    pressure Laplacian is solvable (1^T d = 0) and the step matches a dense
    minimum-norm computation of the same three solves."""
    for dim, n, strain in ((2, 4, False), (3, 2, False), (3, 2, True)):
        m = mesh.KuhnMesh(dim, n, seed=7, jitter=0.1)
        s = stokes.StokesSystem(m, 0.3, 40.0, strain=strain)
        rng = np.random.default_rng(dim)
        f = inputs.fourier_forcing(m.p2coords, 1000 + dim)
        ubc = rng.standard_normal((dim, m.n_p2))
        F, g = s.rhs(f, ubc)
        Us, Ps = s.solve_direct(F, g)
        U, P = s.projection_step(f, ubc, Ps)
        assert np.abs(U - Us).max() <= 1e-10 * np.abs(Us).max()
        assert np.abs(P - Ps).max() <= 1e-9 * np.abs(Ps).max()
        # from p_old = 0: dense route
        U1, P1 = s.projection_step(f, ubc, None)
        Ad = s.Avel_II.toarray()
        U2 = np.linalg.solve(Ad, F.ravel()).reshape(dim, -1)
        d = sum(s.B_I[c] @ U2[c] for c in range(dim)) - g
        assert abs(d.sum()) <= 1e-12 * np.abs(d).max()
        phi = np.linalg.lstsq(s.mats.LQ.toarray(), -s.alpha * d, rcond=None)[0]
        psi = np.linalg.solve(s.mats.MQ.toarray(), d)
        P2 = s.normalize_pressure(phi - s.mu * psi)
        assert np.abs(U1 - U2).max() <= 1e-10 * np.abs(U2).max()
        assert np.abs(P1 - P2).max() <= 1e-8 * np.abs(P2).max()


def _inf_sup_range(s, limit):
    """Spectrum on 1-perp of L_Q^-1 B M_V^-1 B^T (limit "mass") or of
    M_Q^-1 B L_V^-1 B^T (limit "visc"), by dense generalized eigenvalues.

    Integration by parts over V_h in H^1_0 bounds both above by 1
    (p^T B M^-1 B^T p = sup_v (grad p, v)^2 / |v|^2 <= |grad p|^2, and
    p^T B L^-1 B^T p <= |p|^2 |div v|^2 / |grad v|^2 <= |p|^2); the discrete
    inf-sup condition of the Taylor-Hood pair bounds them below by beta^2 > 0."""
    import scipy.linalg as sla
    Bm = sp.hstack(s.B_I).toarray()
    blk = (s.mats.Ms if limit == "mass" else s.mats.Ls)[s.I][:, s.I].toarray()
    X = Bm @ np.linalg.solve(sla.block_diag(*([blk] * s.d)), Bm.T)
    Y = (s.mats.LQ if limit == "mass" else s.mats.MQ).toarray()
    n = X.shape[0]
    Q = np.linalg.qr(np.hstack([np.ones((n, 1)), np.eye(n)[:, : n - 1]]))[0][:, 1:]
    ev = sla.eigh(Q.T @ X @ Q, Q.T @ Y @ Q, eigvals_only=True)
    return ev.min(), ev.max()


class _MutatedProjection(stokes.StokesSystem):
    """The pressure-correction step with one deliberate mistake (for the pin
    below): the sign of phi, the sign of the mu psi term, or alpha dropped
    from phi's right-hand side."""

    def __init__(self, *a, mutation, **kw):
        super().__init__(*a, **kw)
        self.mutation = mutation

    def projection_step(self, f, ubc=None, p_old=None):
        import scipy.sparse.linalg as spla
        F, g = self.rhs(f, ubc)
        p0 = np.zeros(self.np1) if p_old is None else p_old
        bu = F + np.stack([self.B_I[c].T @ p0 for c in range(self.d)])
        U = spla.spsolve(self.Avel_II.tocsc(), bu.ravel()).reshape(self.d, self.nI)
        dv = sum(self.B_I[c] @ U[c] for c in range(self.d)) - g
        scale = 1.0 if self.mutation == "drop_alpha" else self.alpha
        phi = np.linalg.lstsq(self.mats.LQ.toarray(), -scale * dv, rcond=None)[0]
        psi = np.linalg.solve(self.mats.MQ.toarray(), dv)
        sphi = -1.0 if self.mutation == "flip_phi" else 1.0
        spsi = 1.0 if self.mutation == "flip_psi" else -1.0
        return U, self.normalize_pressure(p0 + sphi * phi + spsi * self.mu * psi)


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_projection_step_contracts_at_the_inf_sup_rate(dim, n):
    """Iterating the pressure-correction step from p = 0 is a Richardson
    iteration on the Schur complement S = B A^-1 B^T: with exact solves the
    pressure error obeys e+ = (I - C S) e, C = alpha L_Q^-1 + mu M_Q^-1 (the
    Cahouet-Chabard operator of Sec. 4.1).  In the mass limit (mu -> 0,
    A = alpha M) C S = L_Q^-1 B M^-1 B^T and in the viscous limit (alpha -> 0,
    A = mu L) C S = M_Q^-1 B L^-1 B^T; both have spectrum [beta^2, <= 1]
    (see _inf_sup_range), so C S is self-adjoint in the S inner product and
    every step shrinks ||e||_S by at least the factor 1 - beta^2.

    A flipped sign of phi or of mu psi, or alpha dropped from phi's
    right-hand side, breaks this bound in one of the two limits (the error
    grows, or shrinks by a factor near 1); each mutant is run to show it."""
    m = mesh.KuhnMesh(dim, n, seed=1, jitter=0.1)
    f = inputs.fourier_forcing(m.p2coords, inputs.forcing_seed(1))

    def ratios(s, steps=6):
        F, g = s.rhs(f)
        _, Ps = s.solve_direct(F, g)
        Bm = sp.hstack(s.B_I).toarray()
        Ad = s.Avel_II.toarray()

        def snorm(e):
            return math.sqrt(float(e @ (Bm @ np.linalg.solve(Ad, Bm.T @ e))))

        p = np.zeros(s.np1)
        e0 = snorm(p - Ps)
        out = []
        for _ in range(steps):
            _, p = s.projection_step(f, None, p)
            e1 = snorm(p - Ps)
            out.append(e1 / e0)
            e0 = e1
        return np.array(out)

    for limit, mu, alpha, mutations in (("mass", 1e-9, 1e3, ("flip_phi", "drop_alpha")),
                                        ("visc", 50.0, 1e-9, ("flip_psi",))):
        s = stokes.StokesSystem(m, mu, alpha)
        lo, hi = _inf_sup_range(s, limit)
        assert 0 < lo and hi <= 1 + 1e-10, (limit, lo, hi)
        r = ratios(s)
        assert np.all(r <= 1 - lo + 1e-8), (limit, lo, r)
        for mut in mutations:
            rm = ratios(_MutatedProjection(m, mu, alpha, mutation=mut), steps=3)
            assert np.any(rm > 1 - lo + 1e-3), (limit, mut, lo, rm)


# ------------------------------------------------------------------- solves


def _random_problem(dim, n, mu=1.0, alpha=10.0, seed=0, ubc=False):
    m = mesh.KuhnMesh(dim, n, seed=seed, jitter=0.1)
    s = stokes.StokesSystem(m, mu, alpha)
    f = inputs.fourier_forcing(m.p2coords, 1000 + seed)
    bc = None
    if ubc:
        x = m.p2coords
        bc = np.stack([np.sin(2 * x[:, 1]), np.cos(x[:, 0]), x[:, 0] * x[:, 1]])[:dim]
    F, g = s.rhs(f, bc)
    return m, s, f, bc, F, g


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 4), (3, 2)])
def test_direct_matches_dense_least_squares(dim, n):
    _, s, _, _, F, g = _random_problem(dim, n, ubc=True)
    U1, P1 = s.solve_direct(F, g)
    U2, P2 = s.solve_dense_lstsq(F, g)
    assert np.allclose(U1, U2, rtol=0, atol=1e-12 * np.abs(U2).max())
    assert np.allclose(P1, P2, rtol=0, atol=1e-11 * np.abs(P2).max())
    assert s.residual(U1, P1, F, g) < 1e-13
    assert abs(s.mQ @ P1) < 1e-13


def test_exact_block_factorisation_one_step():
    # Sec. 2.4, Eq. "exact_factorization": the three-factor product equals the
    # inverse of the coupled matrix (on the space where P has zero mean).
    _, s, _, _, F, g = _random_problem(2, 3, mu=0.1, alpha=50.0)
    d, nI = s.d, s.nI
    A = sp.block_diag([s.A_II] * d).toarray()
    Bm = sp.hstack(s.B_I).toarray()
    Ainv = np.linalg.inv(A)
    S = Bm @ Ainv @ Bm.T
    Sp = np.linalg.pinv(S)
    ru, rp = F.ravel(), g
    y_p = rp - Bm @ Ainv @ ru
    w_u, w_p = Ainv @ ru, Sp @ y_p
    z_u, z_p = w_u + Ainv @ Bm.T @ w_p, w_p
    U, P = s.solve_direct(F, g)
    assert np.allclose(z_u, U.ravel(), atol=1e-12 * np.abs(U).max())
    assert np.allclose(s.normalize_pressure(z_p), P, atol=1e-11 * np.abs(P).max())
    # Schur form (Sec. 2.3): S P = g - B A^{-1} F, A U = F + B^T P
    P2 = Sp @ (g - Bm @ Ainv @ ru)
    assert np.allclose(s.normalize_pressure(P2), P, atol=1e-11 * np.abs(P).max())
    del nI


def test_augmented_lagrangian_identity_and_invariance():
    # Sec. 2.3, Prop. "Augmented Lagrangian": S_rho^{-1} = rho M_Q^{-1} + S^{-1}
    # (rho = lambda mu), checked with one pressure row removed so that S is
    # invertible; and the AL system has the same solution as the plain one.
    m, s, _, _, F, g = _random_problem(2, 3, mu=0.3, alpha=20.0)
    d = s.d
    A = sp.block_diag([s.A_II] * d).toarray()
    Bm = sp.hstack(s.B_I).toarray()[1:]
    MQ = s.mats.MQ.toarray()[1:, 1:]
    for lam in (1.0, 10.0):
        rho = lam * s.mu
        Arho = A + rho * Bm.T @ np.linalg.solve(MQ, Bm)
        S = Bm @ np.linalg.solve(A, Bm.T)
        Srho = Bm @ np.linalg.solve(Arho, Bm.T)
        lhs = np.linalg.inv(Srho)
        rhs = rho * np.linalg.inv(MQ) + np.linalg.inv(S)
        assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(rhs).max())
    # AL invariance of the solution (full pressure space, g = 0 here)
    s_al = stokes.StokesSystem(m, s.mu, s.alpha, gamma=10.0, mats=s.mats)
    F2, g2 = s_al.rhs(inputs.fourier_forcing(m.p2coords, 1000), None, gamma_rhs=True)
    BmF = sp.hstack(s.B_I).toarray()
    Agam = A + 10.0 * s.mu * BmF.T @ np.linalg.solve(s.mats.MQ.toarray(), BmF)
    K = np.block([[Agam, -BmF.T], [BmF, np.zeros((s.np1, s.np1))]])
    x = np.linalg.lstsq(K, np.concatenate([F2.ravel(), g2]), rcond=None)[0]
    U0, P0 = s.solve_direct(F2, g2)
    assert np.allclose(x[: d * s.nI], U0.ravel(), atol=1e-11 * np.abs(U0).max())
    assert np.allclose(s.normalize_pressure(x[d * s.nI:]), P0, atol=1e-10 * np.abs(P0).max())
    del F, g


def test_minres_matches_direct_3d():
    _, s, _, _, F, g = _random_problem(3, 3, mu=0.5, alpha=100.0)
    U1, P1 = s.solve_direct(F, g)
    U2, P2, info = s.solve_minres(F, g, rtol=1e-13)
    assert info == 0
    assert np.linalg.norm(U2 - U1) <= 1e-10 * np.linalg.norm(U1)
    assert np.linalg.norm(P2 - P1) <= 1e-9 * np.linalg.norm(P1)


def _l2_errors_2d(m, s, U, P, ubc, u_exact, p_exact):
    """Exact-solution L2 errors by a Duffy Gauss rule on every triangle."""
    pts, wts = _duffy_rule(2, q=5)
    u_full = s.full_velocity(U, ubc)
    vol, _, _ = fem.element_geometry(m)
    X = m.element_vertices()
    eu = nu = ep = npp = 0.0
    lam = np.stack([1 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)  # (q, 3)
    phi2 = np.concatenate([lam * (2 * lam - 1)] + [4 * lam[:, [a]] * lam[:, [b]] for a, b in mesh.local_edges(2)],
                          axis=1)
    for e in range(m.n_e):
        x = X[e, 0] + (pts @ np.stack([X[e, 1] - X[e, 0], X[e, 2] - X[e, 0]]))
        w = wts * 2 * vol[e]
        uh = phi2 @ u_full[:, m.p2[e]].T
        ph = lam @ P[m.elems[e]]
        ue, pe = u_exact(x), p_exact(x)
        eu += np.sum(w[:, None] * (uh - ue) ** 2)
        nu += np.sum(w[:, None] * ue ** 2)
        ep += np.sum(w * (ph - pe) ** 2)
        npp += np.sum(w * pe ** 2)
    return math.sqrt(eu / nu), math.sqrt(ep / npp)


def test_manufactured_rates_2d():
    # P2/P1 Taylor-Hood: O(h^3) velocity and O(h^2) pressure in L2
    # (paper Sec. 3.3 reports the velocity rate on its meshes).
    mu, alpha = 1.0, 100.0
    pi = math.pi

    def u_ex(x):
        return np.stack([np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]),
                         np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])], axis=1)

    def p_ex(x):
        return np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])

    errs = []
    for n in (4, 8, 16):
        m = mesh.KuhnMesh(2, n)
        s = stokes.StokesSystem(m, mu, alpha)
        u, p, f = inputs.manufactured_2d(m.p2coords, mu, alpha)
        F, g = s.rhs(f, u)
        U, P = s.solve_direct(F, g)
        errs.append(_l2_errors_2d(m, s, U, P, u, u_ex, p_ex))
    ru = [math.log2(errs[i][0] / errs[i + 1][0]) for i in range(2)]
    rp = [math.log2(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert min(ru) > 2.7, (errs, ru)
    assert min(rp) > 1.7, (errs, rp)


def test_adjoint_gradient_vs_finite_differences():
    m, s, f, _, F, g = _random_problem(2, 3, mu=0.7, alpha=30.0)
    U, P = s.solve_direct(F, g)
    u = s.full_velocity(U)
    f_t = inputs.fourier_forcing(m.p2coords, 9000)
    Ut, _ = s.solve_direct(*s.rhs(f_t))
    ut = s.full_velocity(Ut)
    J, dJdu = stokes.quadratic_loss(s, u, ut)
    dJdf, dJdmu, lam_u, _ = s.adjoint_gradient(u, dJdu)

    def J_of(fv, mu):
        s2 = stokes.StokesSystem(m, mu, s.alpha, mats=s.mats)
        U2, _ = s2.solve_direct(*s2.rhs(fv))
        return stokes.quadratic_loss(s2, s2.full_velocity(U2), ut)[0]

    for dvec in inputs.fd_directions(f.shape, 4, seed=5):
        h = 1e-3  # J is quadratic in f: central differences are exact up to rounding
        fd = (J_of(f + h * dvec, s.mu) - J_of(f - h * dvec, s.mu)) / (2 * h)
        assert abs(fd - np.sum(dJdf * dvec)) <= 1e-8 * abs(fd)
    h = 1e-5 * s.mu
    fd = (J_of(f, s.mu + h) - J_of(f, s.mu - h)) / (2 * h)
    assert abs(fd - dJdmu) <= 1e-6 * abs(fd)
    del J, lam_u


def test_adjoint_pressure_loss_gradient():
    # loss on the (zero-mean) pressure output: checks the normalisation term
    m, s, f, _, F, g = _random_problem(2, 3, mu=0.7, alpha=30.0)
    w = np.linspace(-1, 2, s.np1)

    def J_of(fv):
        U2, P2 = s.solve_direct(*s.rhs(fv))
        return float(w @ P2), s.full_velocity(U2)

    _, u = J_of(f)
    dJdf, _, _, _ = s.adjoint_gradient(u, np.zeros_like(u), dJdp=w)
    for dvec in inputs.fd_directions(f.shape, 3, seed=9):
        h = 1e-3
        fd = (J_of(f + h * dvec)[0] - J_of(f - h * dvec)[0]) / (2 * h)
        assert abs(fd - np.sum(dJdf * dvec)) <= 1e-8 * max(abs(fd), 1e-12)


# ------------------------------------------- Chebyshev-Jacobi closed form

def _chebyshev_recurrence(A, lo, hi, k, r):
    """Saad's Chebyshev acceleration (Iterative Methods, Alg. 12.1) on
    D^-1 A x = D^-1 r from x = 0: k iterates, one product per step."""
    A = np.asarray(A)
    d = np.diag(A)
    b = r / d
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    dvec = b / theta
    x = dvec.copy()
    for _ in range(1, k):
        res = b - (A @ x) / d
        rho_new = 1.0 / (2.0 * sigma - rho)
        dvec = rho_new * rho * dvec + (2.0 * rho_new / delta) * res
        rho = rho_new
        x = x + dvec
    return x


def test_chebyshev_jacobi_matches_recurrence_and_error_bound():
    """The closed form equals the textbook three-term iteration, meets the
    Chebyshev error bound 2 rho^k in the A-norm when [lo, hi] holds the
    spectrum of D^-1 A, and reaches A^-1 r for large k."""
    rng = np.random.default_rng(11)
    Bm = rng.standard_normal((40, 40))
    A = Bm @ Bm.T + 40 * np.eye(40)
    d = np.diag(A)
    ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
    lo, hi = 0.9 * ev.min(), 1.05 * ev.max()
    r = rng.standard_normal(40)
    x_star = np.linalg.solve(A, r)
    anorm = lambda v: np.sqrt(v @ A @ v)  # noqa: E731
    kappa = hi / lo
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    for k in (1, 2, 3, 6, 9):
        z = stokes.chebyshev_jacobi(A, lo, hi, k, r)
        assert np.allclose(z, _chebyshev_recurrence(A, lo, hi, k, r), rtol=1e-12, atol=1e-14), k
        assert anorm(z - x_star) <= 2 * rho ** k * anorm(x_star) * (1 + 1e-12), k
    assert np.allclose(stokes.chebyshev_jacobi(A, lo, hi, 60, r), x_star, rtol=1e-10)
    # several right-hand sides along the leading axis
    R = rng.standard_normal((3, 40))
    Z = stokes.chebyshev_jacobi(A, lo, hi, 6, R)
    assert np.allclose(Z[1], stokes.chebyshev_jacobi(A, lo, hi, 6, R[1]), rtol=1e-13)
