"""Taylor-Hood P3/P2 on the Kuhn mesh: numbering, exact element integrals and
assembly (TEST INFRASTRUCTURE ONLY, see the package header).

The paper runs its velocity experiments with P2/P1 and with P3/P2 Taylor-Hood
elements (Sec. 1, and Sec. 3.3, Table 4, the P3 rows); the pressure is the
continuous P2 space, the velocity the continuous P3 space.  Everything the
P2/P1 oracle states about the problem carries over; only the element pair
changes.  Readings (listed with the others in the design notes):

* nodes: the P3 velocity nodes of the Kuhn mesh with n cells per side are
  the points of the (3n+1)^d lattice: a node with barycentric multi-index c
  (|c| = 3) of a simplex with vertex lattice points V_a sits at sum_a c_a V_a
  in units of h/3.  Id = I + (3n+1) J [+ (3n+1)^2 K], x fastest.  The P2
  pressure nodes are the (2n+1)^d lattice of the P2/P1 oracle, with its ids
  and local order.
* local P3 order: vertices 0..d; then for each local edge (a, b) in the mesh
  order ((0,1),(0,2),(0,3),(1,2),(1,3),(2,3) / (0,1),(0,2),(1,2)) the node
  next to a (c = 2 e_a + e_b), then the node next to b; then, in 3D, the face
  nodes e_a + e_b + e_c of the faces (0,1,2),(0,1,3),(0,2,3),(1,2,3), and in
  2D the interior node e_0 + e_1 + e_2.  20 nodes per tetrahedron, 10 per
  triangle.
* coordinates: a vertex node copies the vertex; the edge node next to a is
  (2 x_a + x_b) / 3; a face (2D: interior) node is ((x_p + x_q) + x_r) / 3
  with p < q < r the global vertex ids, so nodes shared by several simplices
  get one value.
* basis (barycentric Lagrange functions of degree 3):
      vertex a:      lambda_a (3 lambda_a - 1)(3 lambda_a - 2) / 2
      edge, near a:  9/2 lambda_a lambda_b (3 lambda_a - 1)
      face a, b, c:  27 lambda_a lambda_b lambda_c
* Lambda_V = int |phi_i| per element in closed form (below).

The system object of ``oracle.stokes`` is reused unchanged: ``P3P2Mesh``
exposes the attribute names it reads (n_p2, n_p1, p2_boundary,
interior_nodes, p2coords), which here mean the velocity (P3) and pressure
(P2) spaces.
"""

from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np

from .fem import Matrices, _coo_to_csr, _lam, _poly_diff, _poly_integral, _poly_mul, element_geometry, p2_basis
from .mesh import KuhnMesh, local_edges


def local_faces(dim):
    """Faces (3D) / the single interior triple (2D) of the local P3 order."""
    if dim == 3:
        return [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    return [(0, 1, 2)]


def p3_multi_indices(dim):
    """Barycentric multi-indices c (|c| = 3) of the local P3 nodes, in order."""
    nv = dim + 1
    out = []
    for a in range(nv):
        c = [0] * nv
        c[a] = 3
        out.append(tuple(c))
    for (a, b) in local_edges(dim):
        for near, far in ((a, b), (b, a)):
            c = [0] * nv
            c[near] = 2
            c[far] = 1
            out.append(tuple(c))
    for f in local_faces(dim):
        c = [0] * nv
        for a in f:
            c[a] = 1
        out.append(tuple(c))
    return out


def p3_basis(dim):
    """P3 Lagrange basis in barycentric form, in the local node order."""
    basis = []
    for c in p3_multi_indices(dim):
        nz = [a for a in range(dim + 1) if c[a] > 0]
        if len(nz) == 1:            # vertex: lambda (3 lambda - 1)(3 lambda - 2) / 2
            a = nz[0]
            lam = _lam(a, dim)
            p = _poly_mul(_poly_mul(lam, _affine(a, dim, 3, -1)), _affine(a, dim, 3, -2))
            basis.append({e: v / 2 for e, v in p.items()})
        elif len(nz) == 2:          # edge node next to a: 9/2 lambda_a lambda_b (3 lambda_a - 1)
            a = nz[0] if c[nz[0]] == 2 else nz[1]
            b = nz[1] if a == nz[0] else nz[0]
            p = _poly_mul(_poly_mul(_lam(a, dim), _lam(b, dim)), _affine(a, dim, 3, -1))
            basis.append({e: v * Fraction(9, 2) for e, v in p.items()})
        else:                       # face / interior: 27 lambda_a lambda_b lambda_c
            p = _lam(nz[0], dim)
            for a in nz[1:]:
                p = _poly_mul(p, _lam(a, dim))
            basis.append({e: v * 27 for e, v in p.items()})
    return basis


def _affine(a, dim, s, t):
    """s lambda_a + t (t times the constant 1 = sum of all lambdas)."""
    p = {}
    for e, v in _lam(a, dim).items():
        p[e] = Fraction(s) * v
    for b in range(dim + 1):
        for e, v in _lam(b, dim).items():
            p[e] = p.get(e, Fraction(0)) + Fraction(t) * v
    return {e: v for e, v in p.items() if v != 0}


def _density_integral(g, dim, lo, hi):
    """int_lo^hi g(t) d (1 - t)^(d-1) dt for a polynomial g (coefficient list in
    t): the integral over a simplex of a function of one barycentric
    coordinate, divided by |K| (that coordinate has density d (1 - t)^(d-1))."""
    w = [Fraction(dim) * Fraction(factorial(dim - 1), factorial(k) * factorial(dim - 1 - k)) * (-1) ** k
         for k in range(dim)]
    prod = [Fraction(0)] * (len(g) + len(w) - 1)
    for i, gi in enumerate(g):
        for j, wj in enumerate(w):
            prod[i + j] += Fraction(gi) * wj

    def prim(t):
        return sum(c * t ** (k + 1) / (k + 1) for k, c in enumerate(prod))

    return prim(Fraction(hi)) - prim(Fraction(lo))


def p3_abs_integrals(dim):
    """int_K |phi_i| / |K| for the local P3 basis (exact rationals).

    * vertex: the function of t = lambda_a, t (3t - 1)(3t - 2) / 2, changes sign
      at t = 1/3 and 2/3; integrate against the density of lambda_a piecewise.
    * edge node next to a: 9/2 lambda_a lambda_b (3 lambda_a - 1) has the sign
      of 3 lambda_a - 1.  Given lambda_a = t, the other d coordinates are
      uniform on a simplex of total 1 - t, so E[lambda_b | t] = (1 - t) / d,
      and int |phi| = |K| int 9/2 t (1 - t)/d |3t - 1| d (1 - t)^(d-1) dt.
    * face / interior: 27 lambda_a lambda_b lambda_c >= 0, int |phi| = int phi."""
    third, two3 = Fraction(1, 3), Fraction(2, 3)
    # vertex: g(t) = (9 t^3 - 9 t^2 + 2 t) / 2
    gv = [Fraction(0), Fraction(1), Fraction(-9, 2), Fraction(9, 2)]
    v_abs = (_density_integral(gv, dim, 0, third) - _density_integral(gv, dim, third, two3)
             + _density_integral(gv, dim, two3, 1))
    # edge: h(t) = 9/2 t (3t - 1) (1 - t) / d  (E[lambda_b | t] folded in)
    # = 9/(2d) (-3 t^3 + 4 t^2 - t)
    k = Fraction(9, 2 * dim)
    ge = [Fraction(0), -k, 4 * k, -3 * k]
    e_abs = _density_integral(ge, dim, third, 1) - _density_integral(ge, dim, 0, third)
    basis = p3_basis(dim)
    out = []
    for i, c in enumerate(p3_multi_indices(dim)):
        nz = sum(1 for x in c if x > 0)
        if nz == 1:
            out.append(v_abs)
        elif nz == 2:
            out.append(e_abs)
        else:
            out.append(_poly_integral(basis[i], dim))
    return out


@lru_cache(maxsize=None)
def reference_tensors_p3p2(dim):
    """Shape-independent integrals of the P3/P2 pair (divided by |K|), float64.

      M  [i, j]       int phi_i phi_j                       (P3 x P3)
      T  [i, a, j, b] int (d phi_i / d lambda_a)(d phi_j / d lambda_b)
      W  [k, i, a]    int psi_k (d phi_i / d lambda_a)      (P2 pressure psi_k)
      MQ [k, l]       int psi_k psi_l                       (P2 x P2)
      TQ [k, a, l, b] int (d psi_k / d lambda_a)(d psi_l / d lambda_b)
      absphi [i]      int |phi_i|
      phi [i]         int phi_i
    """
    vb, qb = p3_basis(dim), p2_basis(dim)
    nl, nq, nv = len(vb), len(qb), dim + 1
    dv = [[_poly_diff(p, a) for a in range(nv)] for p in vb]
    dq = [[_poly_diff(p, a) for a in range(nv)] for p in qb]
    M = np.zeros((nl, nl))
    T = np.zeros((nl, nv, nl, nv))
    W = np.zeros((nq, nl, nv))
    MQ = np.zeros((nq, nq))
    TQ = np.zeros((nq, nv, nq, nv))
    phi = np.zeros(nl)
    for i in range(nl):
        phi[i] = float(_poly_integral(vb[i], dim))
        for j in range(nl):
            M[i, j] = float(_poly_integral(_poly_mul(vb[i], vb[j]), dim))
            for a in range(nv):
                for b in range(nv):
                    T[i, a, j, b] = float(_poly_integral(_poly_mul(dv[i][a], dv[j][b]), dim))
        for k in range(nq):
            for a in range(nv):
                W[k, i, a] = float(_poly_integral(_poly_mul(qb[k], dv[i][a]), dim))
    for k in range(nq):
        for l_ in range(nq):
            MQ[k, l_] = float(_poly_integral(_poly_mul(qb[k], qb[l_]), dim))
            for a in range(nv):
                for b in range(nv):
                    TQ[k, a, l_, b] = float(_poly_integral(_poly_mul(dq[k][a], dq[l_][b]), dim))
    absphi = np.array([float(v) for v in p3_abs_integrals(dim)])
    return dict(M=M, T=T, W=W, MQ=MQ, TQ=TQ, absphi=absphi, phi=phi)


class P3P2Mesh:
    """Kuhn mesh with Taylor-Hood P3 velocity / P2 pressure numbering.

    Attributes (besides those of the underlying vertex mesh: dim, n, vcoords,
    vgrid, elems, n_e, seed, jitter):
      vel      (n_e, n_loc)   P3 node ids of each simplex, local P3 order
      vel_grid (n_vel, dim)   lattice position (units h/3)
      vel_coords (n_vel, dim) node coordinates
      q        (n_e, nq_loc)  P2 pressure node ids (the P2/P1 oracle's p2)
      n_vel, n_q, n_loc, nq_loc
    Aliases read by oracle.stokes.StokesSystem: n_p2 = n_vel (velocity nodes),
    n_p1 = n_q (pressure nodes), p2coords = vel_coords, p2_boundary,
    interior_nodes, n_free_nodes (velocity)."""

    def __init__(self, dim, n, seed=0, jitter=0.0):
        base = KuhnMesh(dim, n, seed=seed, jitter=jitter)
        self.base = base
        self.dim, self.n, self.seed, self.jitter = dim, n, base.seed, base.jitter
        self.vcoords, self.vgrid, self.elems, self.n_e = base.vcoords, base.vgrid, base.elems, base.n_e
        self.q = base.p2
        self.n_q = base.n_p2
        self.nq_loc = base.n_loc
        self.q_coords = base.p2coords
        n3 = 3 * n + 1
        self.n_vel = n3 ** dim
        stride = np.array([n3 ** c for c in range(dim)], dtype=np.int64)
        mi = np.array(p3_multi_indices(dim), dtype=np.int64)          # (n_loc, d+1)
        self.n_loc = mi.shape[0]
        eg = self.vgrid[self.elems]                                     # (n_e, d+1, d)
        pos = np.einsum("la,ead->eld", mi, eg)                          # (n_e, n_loc, d)
        self.vel = pos @ stride
        rem = np.arange(self.n_vel)
        grid = np.empty((self.n_vel, dim), dtype=np.int64)
        for c in range(dim):
            grid[:, c] = rem % n3
            rem //= n3
        self.vel_grid = grid
        # coordinates, canonical per node (see the module header)
        vc = self.vcoords
        xc = np.full((self.n_vel, dim), np.nan)
        nv = dim + 1
        for li, c in enumerate(mi):
            nodes = self.vel[:, li]
            nz = [a for a in range(nv) if c[a] > 0]
            if len(nz) == 1:
                x = vc[self.elems[:, nz[0]]]
            elif len(nz) == 2:
                near = nz[0] if c[nz[0]] == 2 else nz[1]
                far = nz[1] if near == nz[0] else nz[0]
                x = (2.0 * vc[self.elems[:, near]] + vc[self.elems[:, far]]) / 3.0
            else:
                ids = np.sort(self.elems[:, nz], axis=1)
                x = ((vc[ids[:, 0]] + vc[ids[:, 1]]) + vc[ids[:, 2]]) / 3.0
            xc[nodes] = x
        if np.isnan(xc).any():
            raise AssertionError("P3 numbering is not onto the (3n+1)^d lattice")
        self.vel_coords = xc
        self.vel_boundary = np.any((grid == 0) | (grid == 3 * n), axis=1)
        # aliases for oracle.stokes.StokesSystem
        self.n_p2, self.n_p1 = self.n_vel, self.n_q
        self.p2coords = self.vel_coords
        self.p2_boundary = self.vel_boundary
        self.p2_interior = ~self.vel_boundary
        self.interior_nodes = np.nonzero(self.p2_interior)[0]
        self.n_free_nodes = self.interior_nodes.size

    def element_vertices(self):
        return self.vcoords[self.elems]


def assemble_p3p2(mesh, grad_div=False):
    """Assemble the Taylor-Hood P3/P2 matrices (Sec. 2.2 / 3.2 / 4.1 with the
    P3/P2 pair): P3 scalar mass Ms and stiffness Ls, the d planes of B
    (P2 pressure rows x P3 velocity columns), the P2 pressure mass MQ and
    Laplacian LQ, and the lumped Lambda_V = int |phi_i| (COO -> CSR with
    explicit zeros kept); grad_div=True adds the d x d grad-div blocks
    D[a][b][i, j] = int d_a phi_i d_b phi_j of Sec. 3.2.  Returns an
    ``oracle.fem.Matrices``."""
    d = mesh.dim
    ref = reference_tensors_p3p2(d)
    vol, grad, _ = element_geometry(mesh)
    G = np.einsum("eac,ebc->eab", grad, grad)
    Me = vol[:, None, None] * ref["M"][None]
    Le = vol[:, None, None] * np.einsum("eab,iajb->eij", G, ref["T"])
    Be = vol[:, None, None, None] * np.einsum("eac,kia->ckei", grad, ref["W"]).transpose(2, 0, 1, 3)
    MQe = vol[:, None, None] * ref["MQ"][None]
    LQe = vol[:, None, None] * np.einsum("eab,kalb->ekl", G, ref["TQ"])
    V, Q = mesh.vel, mesh.q
    nl, nq = V.shape[1], Q.shape[1]
    rv = np.repeat(V, nl, axis=1).ravel()
    cv = np.tile(V, (1, nl)).ravel()
    shape_v = (mesh.n_vel, mesh.n_vel)
    Ms = _coo_to_csr(rv, cv, Me.ravel(), shape_v)
    Ls = _coo_to_csr(rv, cv, Le.ravel(), shape_v)
    rb = np.repeat(Q, nl, axis=1).ravel()
    cb = np.tile(V, (1, nq)).ravel()
    B = [_coo_to_csr(rb, cb, Be[:, c].ravel(), (mesh.n_q, mesh.n_vel)) for c in range(d)]
    rq = np.repeat(Q, nq, axis=1).ravel()
    cq = np.tile(Q, (1, nq)).ravel()
    MQ = _coo_to_csr(rq, cq, MQe.ravel(), (mesh.n_q, mesh.n_q))
    LQ = _coo_to_csr(rq, cq, LQe.ravel(), (mesh.n_q, mesh.n_q))
    Lam = np.zeros(mesh.n_vel)
    np.add.at(Lam, V.ravel(), (vol[:, None] * ref["absphi"][None]).ravel())
    D = None
    if grad_div:
        D = [[None] * d for _ in range(d)]
        for a in range(d):
            for b in range(d):
                De = vol[:, None, None] * np.einsum("ep,eq,ipjq->eij", grad[:, :, a], grad[:, :, b], ref["T"])
                D[a][b] = _coo_to_csr(rv, cv, De.ravel(), shape_v)
    return Matrices(Ms, Ls, B, MQ, LQ, Lam, vol, grad, D)


def p3_basis_values(dim, lam):
    """Values of the local P3 basis at barycentric points lam (npts, d+1),
    evaluated from the factored forms of the module header; (npts, n_loc)."""
    lam = np.asarray(lam, dtype=np.float64)
    out = []
    for c in p3_multi_indices(dim):
        nz = [a for a in range(dim + 1) if c[a] > 0]
        if len(nz) == 1:
            t = lam[:, nz[0]]
            out.append(0.5 * t * (3 * t - 1) * (3 * t - 2))
        elif len(nz) == 2:
            a = nz[0] if c[nz[0]] == 2 else nz[1]
            b = nz[1] if a == nz[0] else nz[0]
            out.append(4.5 * lam[:, a] * lam[:, b] * (3 * lam[:, a] - 1))
        else:
            out.append(27.0 * lam[:, nz[0]] * lam[:, nz[1]] * lam[:, nz[2]])
    return np.stack(out, axis=1)
