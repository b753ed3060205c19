"""Taylor-Hood P2/P1 element matrices by exact barycentric integration, and assembly.

Test infrastructure only (see the package header).

Definitions followed (paper, Sec. 2.2 "Discrete problem" and Sec. 3.2, 4.1):

* velocity mass      M_ij   = int phi_i phi_j                    (Sec. 2.2)
* vector Laplacian   L_ij   = int grad phi_i : grad phi_j         (Sec. 3.2, L_V)
* divergence         B_kj   = b(phi_j, psi_k) = int psi_k div phi_j   (Sec. 2.2)
* pressure mass      MQ_kl  = int psi_k psi_l                     (Sec. 2.2)
* pressure Laplacian LQ_kl  = int grad psi_k . grad psi_l          (Sec. 4.1, Eq. "pressure_Laplacian")
* lumped mass        Lambda_ii = int |phi_i|                      (Sec. 4.1, Lambda_V)

The velocity is vector valued with one scalar P2 basis per component, so M_V =
I_d (x) M_s and L_V = I_d (x) L_s; only the scalar matrices are assembled, and B
is stored as d scalar planes B^c_{k,i} = int psi_k d(phi_i)/dx_c.

Integration is exact: every integrand is a polynomial in the barycentric
coordinates lambda_0..lambda_d, and on a simplex K
    int_K prod_a lambda_a^{k_a} = |K| d! prod_a k_a! / (d + sum_a k_a)!.
The reference tensors are computed once with rational arithmetic; element
matrices follow from |K| and the barycentric gradients (chain rule
grad phi = sum_a (d phi / d lambda_a) grad lambda_a).
"""

from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np
import scipy.sparse as sp

from .mesh import local_edges

# ---------------------------------------------------------------- polynomials
# A polynomial in lambda_0..lambda_d is a dict {exponent tuple: Fraction}.


def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, Fraction(0)) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _poly_diff(p, a):
    out = {}
    for e, c in p.items():
        if e[a] == 0:
            continue
        e2 = list(e)
        e2[a] -= 1
        e2 = tuple(e2)
        out[e2] = out.get(e2, Fraction(0)) + c * e[a]
    return out


def _mono_integral(e, dim):
    """int_K prod lambda^e / |K| (barycentric monomial formula)."""
    num = factorial(dim)
    for k in e:
        num *= factorial(k)
    return Fraction(num, factorial(dim + sum(e)))


def _poly_integral(p, dim):
    return sum((c * _mono_integral(e, dim) for e, c in p.items()), Fraction(0))


def _lam(a, dim, power=1):
    e = [0] * (dim + 1)
    e[a] = power
    return {tuple(e): Fraction(1)}


def p2_basis(dim):
    """P2 Lagrange basis in barycentric form: vertex a -> lambda_a (2 lambda_a - 1),
    edge (a, b) -> 4 lambda_a lambda_b, in the local node order of the mesh."""
    basis = []
    for a in range(dim + 1):
        p = {}
        for e, c in _lam(a, dim, 2).items():
            p[e] = 2 * c
        for e, c in _lam(a, dim, 1).items():
            p[e] = p.get(e, Fraction(0)) - c
        basis.append(p)
    for (a, b) in local_edges(dim):
        e = [0] * (dim + 1)
        e[a] += 1
        e[b] += 1
        basis.append({tuple(e): Fraction(4)})
    return basis


def _abs_vertex_integral(dim):
    """int_K |lambda (2 lambda - 1)| / |K|.

    The barycentric coordinate lambda of a point drawn uniformly in K has the
    density d (1 - t)^(d - 1) on [0, 1]; the integrand changes sign at t = 1/2,
    so the integral is split there and each piece integrated exactly."""
    # g(t) = 2 t^2 - t ; w(t) = d (1 - t)^(d-1), as coefficient lists in t
    g = [Fraction(0), Fraction(-1), Fraction(2)]
    w = [Fraction(0)] * dim
    for k in range(dim):  # binomial expansion of (1 - t)^(d-1)
        if k <= dim - 1:
            w[k] = Fraction(dim) * Fraction(
                factorial(dim - 1), factorial(k) * factorial(dim - 1 - k)) * (-1) ** k
    prod = [Fraction(0)] * (len(g) + len(w) - 1)
    for i, gi in enumerate(g):
        for j, wj in enumerate(w):
            prod[i + j] += gi * wj

    def prim(t):
        return sum(c * t ** (k + 1) / (k + 1) for k, c in enumerate(prod))

    half = Fraction(1, 2)
    neg = prim(half) - prim(Fraction(0))   # integral over [0, 1/2], integrand <= 0
    pos = prim(Fraction(1)) - prim(half)   # integral over [1/2, 1], integrand >= 0
    return pos - neg


@lru_cache(maxsize=None)
def reference_tensors(dim):
    """Shape-independent integrals (all divided by |K|), as float64 arrays.

    Returns dict with
      M  [i, j]       int phi_i phi_j
      T  [i, a, j, b] int (d phi_i / d lambda_a)(d phi_j / d lambda_b)
      W  [k, i, a]    int lambda_k (d phi_i / d lambda_a)
      MQ [k, l]       int lambda_k lambda_l
      absphi [i]      int |phi_i|
      phi [i]         int phi_i
    """
    basis = p2_basis(dim)
    nl, nv = len(basis), dim + 1
    M = np.zeros((nl, nl))
    T = np.zeros((nl, nv, nl, nv))
    W = np.zeros((nv, nl, nv))
    MQ = np.zeros((nv, nv))
    phi = np.zeros(nl)
    absphi = np.zeros(nl)
    dphi = [[_poly_diff(p, a) for a in range(nv)] for p in basis]
    for i in range(nl):
        phi[i] = float(_poly_integral(basis[i], dim))
        for j in range(nl):
            M[i, j] = float(_poly_integral(_poly_mul(basis[i], basis[j]), dim))
            for a in range(nv):
                for b in range(nv):
                    T[i, a, j, b] = float(_poly_integral(_poly_mul(dphi[i][a], dphi[j][b]), dim))
        for k in range(nv):
            for a in range(nv):
                W[k, i, a] = float(_poly_integral(_poly_mul(_lam(k, dim), dphi[i][a]), dim))
    for k in range(nv):
        for l in range(nv):
            MQ[k, l] = float(_poly_integral(_poly_mul(_lam(k, dim), _lam(l, dim)), dim))
    av = float(_abs_vertex_integral(dim))
    for i in range(nl):
        # edge functions 4 lambda_a lambda_b are non-negative on K
        absphi[i] = av if i < nv else phi[i]
    return dict(M=M, T=T, W=W, MQ=MQ, phi=phi, absphi=absphi)


# ------------------------------------------------------------------ geometry


def element_geometry(mesh):
    """|K| and barycentric gradients for every simplex.

    J = [x_1 - x_0, ..., x_d - x_0]; lambda_{1..d}(x) = J^{-1}(x - x_0), so
    grad lambda_a (a >= 1) is row a-1 of J^{-1} and grad lambda_0 = -sum.
    Returns vol (n_e,), grad (n_e, d+1, d), detJ (n_e,)."""
    X = mesh.element_vertices()
    d = mesh.dim
    J = np.stack([X[:, a + 1, :] - X[:, 0, :] for a in range(d)], axis=2)  # (n_e, d, d) columns
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    grad = np.empty((X.shape[0], d + 1, d))
    grad[:, 1:, :] = Jinv
    grad[:, 0, :] = -Jinv.sum(axis=1)
    vol = np.abs(detJ) / factorial(d)
    return vol, grad, detJ


# ------------------------------------------------------------------ assembly


class Matrices:
    """Globally assembled matrices (all P2 / P1 nodes, no boundary conditions).

    Ms, Ls : (n_p2, n_p2) CSR   scalar P2 mass and stiffness
    B      : list of d (n_p1, n_p2) CSR planes sharing one pattern
    MQ, LQ : (n_p1, n_p1) CSR
    Lam    : (n_p2,) lumped |phi| mass
    D      : d x d list of (n_p2, n_p2) CSR grad-div blocks on the Ms pattern,
             D[a][b][i, j] = int d_a phi_i d_b phi_j (only with grad_div=True)
    """

    def __init__(self, Ms, Ls, B, MQ, LQ, Lam, vol, grad, D=None):
        self.Ms, self.Ls, self.B, self.MQ, self.LQ, self.Lam = Ms, Ls, B, MQ, LQ, Lam
        self.vol, self.grad = vol, grad
        self.D = D


def _coo_to_csr(rows, cols, vals, shape):
    A = sp.coo_matrix((vals, (rows, cols)), shape=shape).tocsr()
    A.sum_duplicates()   # explicit zeros are kept: the pattern is structural
    A.sort_indices()
    return A


def assemble(mesh, grad_div=False):
    """Assemble every matrix of Sec. 2.2 / 3.2 / 4.1 on ``mesh`` (COO -> CSR).

    grad_div=True also assembles the grad-div blocks D of Sec. 3.2
    (D_ij = int div phi_i div phi_j for vector basis functions phi_i = phi e_a),
    as the d x d scalar blocks D[a][b][i, j] = int d_a phi_i d_b phi_j."""
    d = mesh.dim
    ref = reference_tensors(d)
    vol, grad, _ = element_geometry(mesh)
    G = np.einsum("eac,ebc->eab", grad, grad)                    # grad lambda_a . grad lambda_b
    Me = vol[:, None, None] * ref["M"][None]
    Le = vol[:, None, None] * np.einsum("eab,iajb->eij", G, ref["T"])
    Be = vol[:, None, None, None] * np.einsum("eac,kia->ckei", grad, ref["W"]).transpose(2, 0, 1, 3)
    # Be: (n_e, d, d+1, n_loc)  [e, c, k, i] = |K| sum_a (grad lambda_a)_c W[k, i, a]
    MQe = vol[:, None, None] * ref["MQ"][None]
    LQe = vol[:, None, None] * G

    P2, P1 = mesh.p2, mesh.elems
    nl, nv = P2.shape[1], d + 1
    r2 = np.repeat(P2, nl, axis=1).ravel()
    c2 = np.tile(P2, (1, nl)).ravel()
    shape2 = (mesh.n_p2, mesh.n_p2)
    Ms = _coo_to_csr(r2, c2, Me.ravel(), shape2)
    Ls = _coo_to_csr(r2, c2, Le.ravel(), shape2)

    rb = np.repeat(P1, nl, axis=1).ravel()
    cb = np.tile(P2, (1, nv)).ravel()
    B = [_coo_to_csr(rb, cb, Be[:, c].ravel(), (mesh.n_p1, mesh.n_p2)) for c in range(d)]

    r1 = np.repeat(P1, nv, axis=1).ravel()
    c1 = np.tile(P1, (1, nv)).ravel()
    shape1 = (mesh.n_p1, mesh.n_p1)
    MQ = _coo_to_csr(r1, c1, MQe.ravel(), shape1)
    LQ = _coo_to_csr(r1, c1, LQe.ravel(), shape1)

    Lam = np.zeros(mesh.n_p2)
    np.add.at(Lam, P2.ravel(), (vol[:, None] * ref["absphi"][None]).ravel())
    D = None
    if grad_div:
        D = [[None] * d for _ in range(d)]
        for a in range(d):
            for b in range(d):
                De = vol[:, None, None] * np.einsum("ep,eq,ipjq->eij", grad[:, :, a], grad[:, :, b], ref["T"])
                D[a][b] = _coo_to_csr(r2, c2, De.ravel(), shape2)
    return Matrices(Ms, Ls, B, MQ, LQ, Lam, vol, grad, D)


def element_matrices(mesh, e):
    """Dense element matrices of simplex ``e`` (for row-by-row spot checks)."""
    d = mesh.dim
    ref = reference_tensors(d)
    X = mesh.vcoords[mesh.elems[e]]
    J = np.stack([X[a + 1] - X[0] for a in range(d)], axis=1)
    Jinv = np.linalg.inv(J)
    grad = np.vstack([-Jinv.sum(axis=0), Jinv])
    vol = abs(np.linalg.det(J)) / factorial(d)
    G = grad @ grad.T
    return dict(
        M=vol * ref["M"],
        L=vol * np.einsum("ab,iajb->ij", G, ref["T"]),
        D=vol * np.einsum("pa,qb,ipjq->abij", grad, grad, ref["T"]),
        B=vol * np.einsum("ac,kia->cki", grad, ref["W"]),
        MQ=vol * ref["MQ"],
        LQ=vol * G,
        absphi=vol * ref["absphi"],
        vol=vol,
    )


def assemble_rows(mesh, rows):
    """Rows of M_s and L_s computed one by one from the incident elements.

    Returns {row: (cols sorted, M values, L values)}; used to spot-check
    matrices at sizes where a full assembly is too slow."""
    rows = [int(r) for r in rows]
    want = set(rows)
    acc = {r: {} for r in rows}
    hit = np.isin(mesh.p2, list(want))
    for e in np.nonzero(hit.any(axis=1))[0]:
        em = element_matrices(mesh, e)
        nodes = mesh.p2[e]
        for i, r in enumerate(nodes):
            if int(r) not in want:
                continue
            for j, cnode in enumerate(nodes):
                m, l = acc[int(r)].get(int(cnode), (0.0, 0.0))
                acc[int(r)][int(cnode)] = (m + em["M"][i, j], l + em["L"][i, j])
    out = {}
    for r in rows:
        cols = np.array(sorted(acc[r]))
        out[r] = (cols, np.array([acc[r][c][0] for c in cols]), np.array([acc[r][c][1] for c in cols]))
    return out


def residual_rows(mesh, mu, alpha, f, u_full, p, vel_rows, p_rows, strain=False):
    """Rows of the coupled residual computed one by one from incident elements.

    Discrete problem of Sec. 2.2 with the velocity block alpha M_V + mu L_V
    (the A~_{lambda,3} form of Sec. 3.2; strain=True: alpha M_V + mu (L_V + D),
    the matrix A of Sec. 3.2) and F = M_V f:
      momentum row (node i, component c):
          (M f_c)_i - ((alpha M + mu L) u_c)_i + sum_k B_c[k, i] p_k
      continuity row k:   - sum_c (B_c u_c)_k
    where u_full holds every P2 node (boundary values included), so the
    Dirichlet lifting is implicit.  f, u_full: (d, n_p2); p: (n_p1,).
    vel_rows: iterable of (c, node); p_rows: iterable of P1 vertex ids.
    Returns (momentum residuals, continuity residuals, momentum right-hand
    sides (M f_c)_i) as arrays in the order given."""
    d = mesh.dim
    vel_rows = [(int(c), int(i)) for c, i in vel_rows]
    p_rows = [int(k) for k in p_rows]
    nodes = {i for _, i in vel_rows}
    verts = set(p_rows)
    rm = {r: 0.0 for r in vel_rows}
    rf = {r: 0.0 for r in vel_rows}
    rp = {k: 0.0 for k in p_rows}
    hit = np.isin(mesh.p2, list(nodes)).any(axis=1) if nodes else np.zeros(mesh.n_e, bool)
    if verts:
        hit |= np.isin(mesh.elems, list(verts)).any(axis=1)
    for e in np.nonzero(hit)[0]:
        em = element_matrices(mesh, e)
        loc = mesh.p2[e]
        vs = mesh.elems[e]
        A = alpha * em["M"] + mu * em["L"]
        for a, i in enumerate(loc):
            for c in range(d):
                key = (c, int(i))
                if key not in rm:
                    continue
                mf = em["M"][a] @ f[c, loc]
                rf[key] += mf
                rm[key] += mf - A[a] @ u_full[c, loc] + em["B"][c, :, a] @ p[vs]
                if strain:
                    rm[key] -= mu * sum(em["D"][c, b, a] @ u_full[b, loc] for b in range(d))
        for kk, k in enumerate(vs):
            if int(k) in rp:
                rp[int(k)] -= sum(em["B"][c, kk, :] @ u_full[c, loc] for c in range(d))
    return (np.array([rm[r] for r in vel_rows]), np.array([rp[k] for k in p_rows]),
            np.array([rf[r] for r in vel_rows]))
