"""Pins of the Taylor-Hood P3/P2 oracle (oracle/p3.py), CPU only.

What fixes each part independently of the oracle's own arithmetic:
* numbering: (3n+1)^d lattice counts, every lattice point reached, nodes of
  the unjittered mesh at lattice / (3n), shared nodes identical;
* element matrices: an independent Duffy (collapsed Gauss-Legendre) rule
  applied to Lagrange bases fitted by a Vandermonde solve at the physical
  P3 / P2 nodes of each element;
* Lambda_V = int |phi_i|: exact integration on the Kuhn subdivision of the
  reference simplex into 6^d pieces (the sign changes of the P3 functions lie
  on the planes lambda_a = 1/3, 2/3, which are faces of that subdivision, so
  |phi| is a polynomial on every piece);
* global invariants: symmetry, 1^T M 1 = 1 for both masses, zero stiffness
  row sums, B (constant) = 0, B (x_c e_c) = M_Q 1, B_I^T 1 = 0 and
  rank B_I = n_q - 1 (the discrete inf-sup of the pair);
* the P2 pressure as the vertex lattice of the mesh with 2n cells (what the
  pressure multigrid of a P3/P2 context builds on): same coordinates, and a
  P1 function of the mesh evaluated there by locating the containing
  simplex by brute force equals its P2 nodal values (vertex values, edge
  means);
* the solve: direct = dense least squares, the exact block factorisation,
  and the convergence rates the paper reports for P3 velocities (Sec. 3.3,
  Table 4): O(h^4) for the velocity and O(h^3) for the pressure in L2 on a
  manufactured 2D solution.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import p3, stokes
from oracle.mesh import KuhnMesh, local_edges
from test_oracle_pins import _duffy_rule, _eval, _lagrange


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 3), (3, 1), (3, 2)])
def test_p3_numbering(dim, n):
    m = p3.P3P2Mesh(dim, n)
    assert m.n_vel == (3 * n + 1) ** dim and m.n_q == (2 * n + 1) ** dim
    assert m.vel.shape == (m.n_e, 20 if dim == 3 else 10)
    assert np.array_equal(np.unique(m.vel), np.arange(m.n_vel))
    # unjittered: node coordinates are the lattice points over 3n
    assert np.allclose(m.vel_coords, m.vel_grid / (3.0 * n), rtol=0, atol=4e-16)
    # every simplex's local nodes are the barycentric points sum c_a x_a / 3
    mi = np.array(p3.p3_multi_indices(dim))
    X = m.vcoords[m.elems]
    want = np.einsum("la,ead->eld", mi / 3.0, X)
    assert np.allclose(m.vel_coords[m.vel], want, rtol=0, atol=4e-16)
    nb = (3 * n + 1) ** dim - (3 * n - 1) ** dim
    assert m.vel_boundary.sum() == nb


def test_p3_jittered_shared_nodes_consistent():
    m = p3.P3P2Mesh(3, 3, seed=4, jitter=0.15)
    mi = np.array(p3.p3_multi_indices(3))
    X = m.vcoords[m.elems]
    want = np.einsum("la,ead->eld", mi / 3.0, X)
    # the canonical per-node formula agrees with every simplex's own
    # barycentric point to rounding
    assert np.abs(m.vel_coords[m.vel] - want).max() <= 4e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_p3p2_element_matrices_vs_nodal_quadrature(dim):
    m = p3.P3P2Mesh(dim, 2, seed=11, jitter=0.12)
    mats = p3.assemble_p3p2(m)
    ref = p3.reference_tensors_p3p2(dim)
    pts, wts = _duffy_rule(dim, q=7)
    for e in (0, 5, m.n_e - 1):
        X = m.vcoords[m.elems[e]]
        J = np.stack([X[a + 1] - X[0] for a in range(dim)], axis=1)
        mi = np.array(p3.p3_multi_indices(dim))
        nodes3 = (mi / 3.0) @ X
        nodes2 = np.vstack([X] + [0.5 * (X[a] + X[b]) for a, b in local_edges(dim)])
        mons3, C3 = _lagrange(nodes3, 3)
        mons2, C2 = _lagrange(nodes2, 2)
        nl, nq = nodes3.shape[0], nodes2.shape[0]
        M, L = np.zeros((nl, nl)), np.zeros((nl, nl))
        B = np.zeros((dim, nq, nl))
        MQ, LQ = np.zeros((nq, nq)), np.zeros((nq, nq))
        phi_int = np.zeros(nl)
        detJ = abs(np.linalg.det(J))
        for xi, w in zip(pts, wts):
            x = X[0] + J @ xi
            f3, g3 = _eval(mons3, C3, x)
            f2, g2 = _eval(mons2, C2, x)
            ww = w * detJ
            M += ww * np.outer(f3, f3)
            L += ww * g3.T @ g3
            for c in range(dim):
                B[c] += ww * np.outer(f2, g3[c])
            MQ += ww * np.outer(f2, f2)
            LQ += ww * g2.T @ g2
            phi_int += ww * f3
        # the assembled element contributions: rebuild from the reference
        # tensors with this element's geometry
        vol = mats.vol[e]
        G = mats.grad[e] @ mats.grad[e].T
        Me = vol * ref["M"]
        Le = vol * np.einsum("ab,iajb->ij", G, ref["T"])
        Be = vol * np.einsum("ac,kia->cki", mats.grad[e], ref["W"])
        MQe = vol * ref["MQ"]
        LQe = vol * np.einsum("ab,kalb->kl", G, ref["TQ"])
        assert np.allclose(Me, M, rtol=0, atol=1e-13 * np.abs(M).max())
        assert np.allclose(Le, L, rtol=0, atol=1e-11 * np.abs(L).max())
        assert np.allclose(Be, B, rtol=0, atol=1e-12 * np.abs(B).max())
        assert np.allclose(MQe, MQ, rtol=0, atol=1e-13 * np.abs(MQ).max())
        assert np.allclose(LQe, LQ, rtol=0, atol=1e-12 * np.abs(LQ).max())
        assert np.allclose(vol * ref["phi"], phi_int, rtol=0, atol=1e-13 * np.abs(phi_int).max())
    # row sums of the mass reference = int phi (partition of unity)
    assert np.allclose(ref["M"].sum(axis=1), ref["phi"], atol=1e-15)
    assert abs(ref["phi"].sum() - 1.0) < 1e-14


def _kuhn_subsimplices(dim, k):
    """Barycentric vertices (d+1, d+1) of the k^d * d! Kuhn pieces of the
    reference simplex {xi >= 0, sum xi <= 1} (pieces of the cube that lie in
    the simplex, mapped by the order-preserving cumulative map)."""
    out = []
    for cell in itertools.product(range(k), repeat=dim):
        for perm in itertools.permutations(range(dim)):
            pos = [np.array(cell, dtype=float)]
            for ax in perm:
                p = pos[-1].copy()
                p[ax] += 1
                pos.append(p)
            pos = np.array(pos) / k          # cube points in [0,1]^d
            # map the cube [0,1]^d onto the simplex by sorting: the Kuhn
            # pieces with a decreasing coordinate chain are the simplex
            # t1 >= t2 >= ... ; keep pieces inside 1 >= y_1 >= ... >= y_d >= 0
            if np.all(np.diff(pos, axis=1) <= 1e-12):
                lam = np.concatenate([1 - pos[:, :1], pos[:, :-1] - pos[:, 1:], pos[:, -1:]], axis=1)
                out.append(lam)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_abs_integrals_by_subdivision(dim):
    # the sign changes of every P3 basis function lie on lambda_a = 1/3 or
    # 2/3: faces of the Kuhn subdivision with k = 3 along the chain
    # coordinates; on each piece |phi| is a cubic, integrated exactly by a
    # Duffy rule of 6 points per direction
    pieces = _kuhn_subsimplices(dim, 6)
    vol_ref = 1.0 / math.factorial(dim)
    assert abs(len(pieces) - 6 ** dim) == 0
    pts, wts = _duffy_rule(dim, q=6)
    lam_ref = np.concatenate([1 - pts.sum(axis=1, keepdims=True), pts], axis=1)
    total = np.zeros(20 if dim == 3 else 10)
    vol_sum = 0.0
    for lam_v in pieces:
        # barycentric coordinates of the piece's points in the reference simplex
        lam = lam_ref @ lam_v
        Jp = np.stack([lam_v[a + 1, 1:] - lam_v[0, 1:] for a in range(dim)], axis=1)
        det = abs(np.linalg.det(Jp))
        vals = p3.p3_basis_values(dim, lam)
        signs = np.sign(p3.p3_basis_values(dim, lam_v.mean(axis=0, keepdims=True)))[0]
        # one sign per piece: no basis function changes sign inside a piece
        assert np.all(np.sign(vals) * signs >= 0)
        total += det * (wts @ np.abs(vals))
        vol_sum += det * wts.sum()
    assert abs(vol_sum - vol_ref) < 1e-14
    exact = np.array([float(v) for v in p3.p3_abs_integrals(dim)])
    assert np.allclose(total / vol_ref, exact, rtol=1e-13, atol=0)
    ref = p3.reference_tensors_p3p2(dim)
    assert np.allclose(ref["absphi"], exact, rtol=0, atol=1e-16)
    assert np.all(ref["absphi"] >= np.abs(ref["phi"]) - 1e-16)


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 3), (3, 1), (3, 2)])
def test_p3p2_global_invariants(dim, n):
    m = p3.P3P2Mesh(dim, n, seed=3, jitter=0.1)
    mats = p3.assemble_p3p2(m)
    for A in (mats.Ms, mats.Ls, mats.MQ, mats.LQ):
        assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    onev, oneq = np.ones(m.n_vel), np.ones(m.n_q)
    assert abs(onev @ mats.Ms @ onev - 1.0) < 1e-13
    assert abs(oneq @ mats.MQ @ oneq - 1.0) < 1e-13
    assert np.abs(mats.Ls @ onev).max() < 1e-11
    assert np.abs(mats.LQ @ oneq).max() < 1e-11
    for c in range(dim):
        assert np.abs(mats.B[c] @ onev).max() < 1e-15
        assert np.allclose(mats.B[c] @ m.vel_coords[:, c], mats.MQ @ oneq, atol=1e-15)
    s = stokes.StokesSystem(m, 1.0, 10.0, mats=mats)
    for c in range(dim):
        assert np.abs(s.B_I[c].T @ oneq).max() < 1e-15
    Bm = sp.hstack(s.B_I).toarray()
    if n >= 2:  # one cell has too few interior velocity nodes for a unique pressure
        assert np.linalg.matrix_rank(Bm) == m.n_q - 1
    assert np.all(mats.Lam > 0)


def _p3_problem(dim, n, mu=1.0, alpha=10.0, seed=0, ubc=True):
    m = p3.P3P2Mesh(dim, n, seed=seed, jitter=0.1)
    s = stokes.StokesSystem(m, mu, alpha, mats=p3.assemble_p3p2(m))
    rng = np.random.default_rng(seed + 7)
    f = rng.standard_normal((dim, m.n_vel))
    bc = rng.standard_normal((dim, m.n_vel)) if ubc else None
    F, g = s.rhs(f, bc)
    return m, s, f, bc, F, g


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 3), (3, 2)])
def test_p3p2_direct_matches_dense_least_squares(dim, n):
    _, s, _, _, F, g = _p3_problem(dim, n)
    U1, P1 = s.solve_direct(F, g)
    U2, P2 = s.solve_dense_lstsq(F, g)
    assert np.allclose(U1, U2, rtol=0, atol=1e-11 * np.abs(U2).max())
    assert np.allclose(P1, P2, rtol=0, atol=1e-10 * np.abs(P2).max())
    assert s.residual(U1, P1, F, g) < 1e-13
    assert abs(s.mQ @ P1) < 1e-12


def test_p3p2_exact_block_factorisation_one_step():
    _, s, _, _, F, g = _p3_problem(2, 2, mu=0.1, alpha=50.0)
    A = sp.block_diag([s.A_II] * s.d).toarray()
    Bm = sp.hstack(s.B_I).toarray()
    Ainv = np.linalg.inv(A)
    Sp = np.linalg.pinv(Bm @ Ainv @ Bm.T)
    ru, rp = F.ravel(), g
    w_p = Sp @ (rp - Bm @ Ainv @ ru)
    z_u = Ainv @ ru + Ainv @ Bm.T @ w_p
    U, P = s.solve_direct(F, g)
    assert np.allclose(z_u, U.ravel(), atol=1e-11 * np.abs(U).max())
    assert np.allclose(s.normalize_pressure(w_p), P, atol=1e-10 * np.abs(P).max())


def _l2_errors_2d_p3(m, s, U, P, ubc, u_exact, p_exact):
    """Exact-solution L2 errors by a Duffy Gauss rule on every triangle."""
    pts, wts = _duffy_rule(2, q=7)
    u_full = s.full_velocity(U, ubc)
    X = m.element_vertices()
    lam = np.stack([1 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)
    phi3 = p3.p3_basis_values(2, lam)
    phi2 = np.concatenate([lam * (2 * lam - 1)] + [4 * lam[:, [a]] * lam[:, [b]] for a, b in local_edges(2)],
                          axis=1)
    eu = nu = ep = npp = 0.0
    for e in range(m.n_e):
        J = np.stack([X[e, 1] - X[e, 0], X[e, 2] - X[e, 0]])
        x = X[e, 0] + pts @ J
        w = wts * abs(np.linalg.det(J))
        uh = phi3 @ u_full[:, m.vel[e]].T
        ph = phi2 @ P[m.q[e]]
        ue, pe = u_exact(x), p_exact(x)
        eu += np.sum(w[:, None] * (uh - ue) ** 2)
        nu += np.sum(w[:, None] * ue ** 2)
        ep += np.sum(w * (ph - pe) ** 2)
        npp += np.sum(w * pe ** 2)
    return math.sqrt(eu / nu), math.sqrt(ep / npp)


def test_p3p2_manufactured_rates_2d():
    # P3/P2 Taylor-Hood: O(h^4) velocity (the rate the paper observes for its
    # P3 runs, Sec. 3.3) and O(h^3) pressure in L2
    mu, alpha = 1.0, 100.0
    pi = math.pi

    def u_ex(x):
        return np.stack([np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]),
                         np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])], axis=1)

    def p_ex(x):
        return np.cos(pi * x[:, 0]) * np.cos(pi * x[:, 1])

    def f_ex(x):
        u = u_ex(x)
        gp = np.stack([-pi * np.sin(pi * x[:, 0]) * np.cos(pi * x[:, 1]),
                       -pi * np.cos(pi * x[:, 0]) * np.sin(pi * x[:, 1])], axis=1)
        return (alpha + 2 * pi * pi * mu) * u + gp

    errs = []
    for n in (2, 4, 8):
        m = p3.P3P2Mesh(2, n, seed=0, jitter=0.0)
        s = stokes.StokesSystem(m, mu, alpha, mats=p3.assemble_p3p2(m))
        x = m.vel_coords
        f = f_ex(x).T
        ubc = u_ex(x).T
        F, g = s.rhs(f, ubc)
        U, P = s.solve_direct(F, g)
        errs.append(_l2_errors_2d_p3(m, s, U, P, ubc, u_ex, p_ex))
    eu = np.array([e[0] for e in errs])
    ep = np.array([e[1] for e in errs])
    ru, rp = np.log2(eu[:-1] / eu[1:]), np.log2(ep[:-1] / ep[1:])
    # the forcing enters as M_V f_nodal (P3 interpolant, reading c-5): its
    # error is O(h^4) too, so the rates are not spoilt
    assert ru[-1] > 3.7, (eu, ru)
    assert rp[-1] > 2.7, (ep, rp)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_p2_nodes_are_the_refined_vertex_lattice(dim, n):
    """The P2 nodes of the Kuhn mesh with n cells per side sit at the vertices
    of the mesh with 2n cells, id for id, and the P1 functions of the coarse
    mesh are the P2 functions whose edge nodes carry the mean of the edge's
    two end values: evaluating a random P1 function at every refined vertex
    through a brute-force search for a simplex that contains it gives the P2
    nodal values built from the element table."""
    m1, m2 = KuhnMesh(dim, n, jitter=0.0), KuhnMesh(dim, 2 * n, jitter=0.0)
    assert m1.n_p2 == m2.n_p1
    np.testing.assert_allclose(m1.p2coords, m2.vcoords, rtol=0, atol=1e-15)
    v = np.random.default_rng(5).standard_normal(m1.n_p1)
    u2 = np.full(m1.n_p2, np.nan)
    for e in range(m1.n_e):
        for a in range(dim + 1):
            u2[m1.p2[e, a]] = v[m1.elems[e, a]]
        for q, (a, b) in enumerate(local_edges(dim)):
            u2[m1.p2[e, dim + 1 + q]] = 0.5 * (v[m1.elems[e, a]] + v[m1.elems[e, b]])
    X = m1.vcoords
    for i, x in enumerate(m2.vcoords):
        val = None
        for e in range(m1.n_e):
            P = X[m1.elems[e]]
            lam = np.linalg.solve((P[1:] - P[0]).T, x - P[0])
            bary = np.concatenate([[1.0 - lam.sum()], lam])
            if bary.min() >= -1e-12:
                val = bary @ v[m1.elems[e]]
                break
        assert val is not None, i
        assert abs(val - u2[i]) <= 1e-12, (i, val, u2[i])
