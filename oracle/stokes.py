"""Generalized Stokes saddle-point system, its direct / MINRES solution, the true
residual and the adjoint gradient (TEST INFRASTRUCTURE ONLY).

The paper's discrete problem (Sec. 2.2, Eq. "Saddle_point_A_BT_B"):

    A U - B^T P = F,   B U = 0,      A = (1/dt) M_V + mu E_V.

Readings used here (listed with the others in the design notes):

* viscous block: mu L_V, the vector Laplacian (the paper's A~_{lambda,3} =
  dt^-1 M_V + mu L_V of Sec. 3.2); alpha = 1/dt.  strain=True uses the
  paper's own matrix A = dt^-1 M_V + mu (L_V + D) of Sec. 3.2 (D the grad-div
  matrix), which equals the strain-rate form 2 mu eps:eps on H^1_0; the
  Dirichlet lifting uses the same A.
* Dirichlet data on the whole boundary (Sec. 3.1, V = H^1_0): the velocity
  is eliminated on boundary nodes with nodal values G and lifted,
      F~ = (M_V f)_I - A_{I,Gamma} G,    g = -B_Gamma G,
  where f is the forcing given at every P2 node (F = M_V f, exact).
* g is made compatible by removing its l2 mean (1^T g = 0 is required since
  B_I^T 1 = 0); the pressure is returned with zero integral (1^T M_Q P = 0).
* augmented Lagrangian (Sec. 2.3, Eq. "def_of_Alambda"): A_gamma = A +
  gamma mu B^T M_Q^{-1} B with right-hand side F~ + gamma mu B^T M_Q^{-1} g.
  Because B U = g at the solution, the solution does not depend on gamma, so
  the oracle solves the gamma = 0 system; ``apply_coupled`` still applies
  the gamma operator for residual checks.
* "relative residual": the unpreconditioned l2 residual of the plain (gamma
  = 0) coupled FP64 system, ||b - K x|| / ||b|| with b = (F~, g).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import assemble


class StokesSystem:
    """Assembled and boundary-reduced generalized Stokes system on a mesh.

    Unknown layout: U is (d, n_I) (component-major over interior P2 nodes in
    increasing node id), P is (n_p1,)."""

    def __init__(self, mesh, mu, alpha, gamma=0.0, mats=None, strain=False):
        self.mesh = mesh
        self.mu, self.alpha, self.gamma = float(mu), float(alpha), float(gamma)
        self.strain = bool(strain)
        self.mats = assemble(mesh, grad_div=self.strain) if mats is None else mats
        m = self.mats
        if self.strain and m.D is None:
            raise ValueError("strain=True needs matrices assembled with grad_div=True")
        self.d = mesh.dim
        self.I = mesh.interior_nodes
        self.nI = self.I.size
        self.np1 = mesh.n_p1
        # A_s = alpha M_s + mu L_s on the shared structural pattern (a sparse sum
        # would drop entries that cancel exactly, e.g. on right triangles)
        if not (np.array_equal(m.Ms.indptr, m.Ls.indptr) and np.array_equal(m.Ms.indices, m.Ls.indices)):
            raise AssertionError("M_s and L_s must share one pattern")
        self.As_full = m.Ms.copy()
        self.As_full.data = self.alpha * m.Ms.data + self.mu * m.Ls.data
        self.A_II = self.As_full[self.I][:, self.I].tocsr()
        self.A_Iall = self.As_full[self.I].tocsr()
        self.B_I = [b[:, self.I].tocsr() for b in m.B]
        self.mQ = m.MQ @ np.ones(self.np1)   # M_Q 1 (pressure integral weights)
        self._MQ_lu = None
        # velocity operator on component-major vectors (index c * n_p2 + node):
        # I_d (x) A_s, plus mu D (strain) and the viscous part E for dJ/dmu
        d, n2 = self.d, mesh.n_p2
        blocks, eblocks = [], []
        for a in range(d):
            row, erow = [], []
            for b in range(d):
                if a == b:
                    Ab, Eb = self.As_full.copy(), m.Ls.copy()
                    if self.strain:
                        Ab.data = Ab.data + self.mu * m.D[a][a].data
                        Eb.data = Eb.data + m.D[a][a].data
                elif self.strain:
                    Ab, Eb = self.mu * m.D[a][b], m.D[a][b]
                else:
                    Ab = Eb = None
                row.append(Ab)
                erow.append(Eb)
            blocks.append(row)
            eblocks.append(erow)
        self.Avel_full = sp.bmat(blocks, format="csr")
        Evel_full = sp.bmat(eblocks, format="csr")
        self.Iv = np.concatenate([c * n2 + self.I for c in range(d)])
        self.Avel_II = self.Avel_full[self.Iv][:, self.Iv].tocsr()
        self.Avel_Iall = self.Avel_full[self.Iv].tocsr()
        self.Evel_Iall = Evel_full[self.Iv].tocsr()

    # ------------------------------------------------------------- helpers
    def MQ_solve(self, r):
        if self._MQ_lu is None:
            self._MQ_lu = spla.splu(self.mats.MQ.tocsc())
        return self._MQ_lu.solve(r)

    def lift(self, ubc):
        """Nodal lifting G: ubc on boundary nodes, zero inside. (d, n_p2)."""
        G = np.zeros((self.d, self.mesh.n_p2))
        if ubc is not None:
            bnd = self.mesh.p2_boundary
            G[:, bnd] = np.asarray(ubc, dtype=np.float64).reshape(self.d, -1)[:, bnd]
        return G

    def rhs(self, f, ubc=None, gamma_rhs=False):
        """(F~, g) of the reduced system; f, ubc are (d, n_p2) nodal arrays.

        gamma_rhs=True adds the augmented-Lagrangian term gamma mu B^T M_Q^{-1} g."""
        f = np.asarray(f, dtype=np.float64).reshape(self.d, -1)
        G = self.lift(ubc)
        F = np.empty((self.d, self.nI))
        AG = (self.Avel_Iall @ G.ravel()).reshape(self.d, self.nI)
        for c in range(self.d):
            F[c] = (self.mats.Ms @ f[c])[self.I] - AG[c]
        g = np.zeros(self.np1)
        for c in range(self.d):
            g -= self.mats.B[c] @ G[c]
        g -= g.mean()
        if gamma_rhs and self.gamma != 0.0:
            w = self.MQ_solve(g)
            for c in range(self.d):
                F[c] += self.gamma * self.mu * (self.B_I[c].T @ w)
        return F, g

    def apply_coupled(self, U, P, gamma=None):
        """K_gamma (U, P) = (A_gamma U - B^T P, B U) for U (d, n_I), P (n_p1,)."""
        gamma = self.gamma if gamma is None else gamma
        U = np.asarray(U).reshape(self.d, self.nI)
        BU = sum(self.B_I[c] @ U[c] for c in range(self.d))
        RU = (self.Avel_II @ U.ravel()).reshape(self.d, self.nI)
        w = self.MQ_solve(BU) if gamma != 0.0 else None
        for c in range(self.d):
            RU[c] = RU[c] - self.B_I[c].T @ P
            if w is not None:
                RU[c] += gamma * self.mu * (self.B_I[c].T @ w)
        return RU, BU

    def residual(self, U, P, F, g):
        """True relative residual ||b - K x||_2 / ||b||_2 of the plain system."""
        RU, RP = self.apply_coupled(U, P, gamma=0.0)
        num = np.sqrt(np.sum((F - RU) ** 2) + np.sum((g - RP) ** 2))
        den = np.sqrt(np.sum(F ** 2) + np.sum(g ** 2))
        return num / den if den > 0 else num

    def normalize_pressure(self, P):
        """Shift P so that int p_h = 1^T M_Q P = 0."""
        return P - (self.mQ @ P) / self.mQ.sum()

    def full_velocity(self, U, ubc=None):
        """Scatter interior U (d, n_I) and the boundary data to all P2 nodes."""
        u = self.lift(ubc)
        u[:, self.I] = U
        return u

    # ------------------------------------------------------------- operators
    def coupled_matrix(self, bordered=True):
        """Sparse K = [[I_d (x) A_II, -B_I^T], [B_I, 0]], optionally bordered with
        the zero-mean constraint [0, m^T] / column [0; m] (m = M_Q 1)."""
        d = self.d
        Ablk = self.Avel_II
        BT = sp.vstack([b.T for b in self.B_I], format="csr")
        Bm = sp.hstack(self.B_I, format="csr")
        if not bordered:
            return sp.bmat([[Ablk, -BT], [Bm, None]], format="csc")
        mcol = sp.csr_matrix(self.mQ[:, None])
        return sp.bmat([[Ablk, -BT, None], [Bm, None, mcol], [None, mcol.T, None]],
                       format="csc")

    # ------------------------------------------------------------- solvers
    def solve_direct(self, F, g):
        """Sparse LU of the bordered system (small meshes)."""
        K = self.coupled_matrix(bordered=True)
        b = np.concatenate([F.ravel(), g, [0.0]])
        x = spla.spsolve(K, b)
        U = x[: self.d * self.nI].reshape(self.d, self.nI)
        P = self.normalize_pressure(x[self.d * self.nI: self.d * self.nI + self.np1])
        return U, P

    def solve_dense_lstsq(self, F, g):
        """Minimum-norm least-squares solution of the singular unbordered system
        (tiny meshes only) -- an independent route to the same (U, P)."""
        K = self.coupled_matrix(bordered=False).toarray()
        b = np.concatenate([F.ravel(), g])
        x = np.linalg.lstsq(K, b, rcond=None)[0]
        U = x[: self.d * self.nI].reshape(self.d, self.nI)
        P = self.normalize_pressure(x[self.d * self.nI:])
        return U, P

    def solve_minres(self, F, g, rtol=1e-13, maxiter=5000, inner_rtol=1e-14, callback=None):
        """Preconditioned MINRES on the symmetric form [[A, B^T], [B, 0]] (U, -P).

        Block-diagonal SPD preconditioner: CG on the velocity block (Jacobi,
        tight tolerance) and mu M_Q^{-1} + alpha (M_Q + L_Q)^{-1} on the
        pressure, both by CG.  Only the iteration count depends on it."""
        d, nI, np1 = self.d, self.nI, self.np1
        Ablk = self.Avel_II
        Bm = sp.hstack(self.B_I, format="csr")
        Ksym = sp.bmat([[Ablk, Bm.T], [Bm, None]], format="csr")
        Dinv_A = 1.0 / Ablk.diagonal()
        MQ, XQ = self.mats.MQ, (self.mats.MQ + self.mats.LQ).tocsr()
        Dinv_MQ, Dinv_XQ = 1.0 / MQ.diagonal(), 1.0 / XQ.diagonal()

        def cg(A, b, dinv):
            x, _ = spla.cg(A, b, rtol=inner_rtol, atol=0.0, maxiter=10000,
                           M=spla.LinearOperator(A.shape, lambda v: dinv * v))
            return x

        def prec(v):
            out = np.empty_like(v)
            out[:d * nI] = cg(Ablk, v[:d * nI], Dinv_A)
            vp = v[d * nI:]
            out[d * nI:] = self.mu * cg(MQ, vp, Dinv_MQ) + self.alpha * cg(XQ, vp, Dinv_XQ)
            return out

        n = d * nI + np1
        b = np.concatenate([F.ravel(), g])
        x, info = spla.minres(Ksym, b, M=spla.LinearOperator((n, n), prec), rtol=rtol,
                              maxiter=maxiter, callback=callback)
        U = x[: d * nI].reshape(d, nI)
        P = self.normalize_pressure(-x[d * nI:])
        return U, P, info

    def solve(self, F, g, method="auto", **kw):
        if method == "auto":
            method = "direct" if self.d * self.nI + self.np1 <= 150_000 else "minres"
        if method == "direct":
            return self.solve_direct(F, g)
        if method == "lstsq":
            return self.solve_dense_lstsq(F, g)
        U, P, _ = self.solve_minres(F, g, **kw)
        return U, P

    # ------------------------------------------------------------- projection
    def projection_step(self, f, ubc=None, p_old=None):
        """One rotational incremental pressure-correction step, the comparator
        of Sec. 7.5 and Table 8: a momentum solve, then a pressure Poisson
        solve and a pressure-mass solve, each done directly:
            A U = F~ + B_I^T p_old,   d = B_I U - g,
            L_Q phi = -alpha d (zero mean),   M_Q psi = d,
            P = p_old + phi - mu psi  (zero integral).
        The coupled solution is its fixed point: with p_old = P*, U = U*
        and d = 0."""
        d_ = self.d
        F, g = self.rhs(f, ubc)
        p0 = np.zeros(self.np1) if p_old is None else np.asarray(p_old, dtype=np.float64)
        bu = F + np.stack([self.B_I[c].T @ p0 for c in range(d_)])
        U = spla.spsolve(self.Avel_II.tocsc(), bu.ravel()).reshape(d_, self.nI)
        dvec = sum(self.B_I[c] @ U[c] for c in range(d_)) - g
        one = sp.csr_matrix(np.ones((self.np1, 1)))
        K = sp.bmat([[self.mats.LQ, one], [one.T, None]], format="csc")
        phi = spla.spsolve(K, np.concatenate([-self.alpha * dvec, [0.0]]))[: self.np1]
        psi = spla.spsolve(self.mats.MQ.tocsc(), dvec)
        P = self.normalize_pressure(p0 + phi - self.mu * psi)
        return U, P

    # ------------------------------------------------------------- adjoint
    def adjoint_gradient(self, u_full, dJdu_full, dJdp=None, method="auto", **kw):
        """Gradient of a loss J(u, p) w.r.t. the nodal forcing f and mu.

        The transposed system K^T (lam_u, lam_p) = (dJ/dU_I, Pi^T dJ/dP), with
        K^T = [[A, B^T], [-B, 0]], becomes the forward system after the
        substitution q = -lam_p:  A lam_u - B^T q = j_u,  B lam_u = -j_p.
        Then dJ/df_c = M_s[:, I] lam_u,c (all P2 nodes) and
        dJ/dmu = -lam_u . (E[I, :] u) with E the viscous matrix (I_d (x) L_s,
        plus D with strain).  Pi is the zero-mean normalisation of the
        pressure output."""
        d = self.d
        ju = np.asarray(dJdu_full).reshape(d, -1)[:, self.I]
        jp = np.zeros(self.np1) if dJdp is None else np.asarray(dJdp, dtype=np.float64)
        # Pi = I - 1 m^T / (1^T m); its transpose applied to jp:
        jp = jp - self.mQ * jp.sum() / self.mQ.sum()
        lam_u, q = self.solve(ju, -jp, method=method, **kw)
        lam_p = -q
        dJdf = np.zeros((d, self.mesh.n_p2))
        u_full = np.asarray(u_full).reshape(d, -1)
        for c in range(d):
            ext = np.zeros(self.mesh.n_p2)
            ext[self.I] = lam_u[c]
            dJdf[c] = self.mats.Ms @ ext
        dJdmu = -float(lam_u.ravel() @ (self.Evel_Iall @ u_full.ravel()))
        return dJdf, dJdmu, lam_u, lam_p


def quadratic_loss(sysm, u_full, u_target_full):
    """J = 1/2 (u - u*)^T M_V (u - u*) over all P2 nodes, and dJ/du."""
    diff = np.asarray(u_full).reshape(sysm.d, -1) - np.asarray(u_target_full).reshape(sysm.d, -1)
    Md = np.stack([sysm.mats.Ms @ diff[c] for c in range(sysm.d)])
    return 0.5 * float(np.sum(diff * Md)), Md


def chebyshev_jacobi(A, lo, hi, k, r):
    """z = q_k(D^-1 A) D^-1 r, the degree-k Chebyshev-Jacobi polynomial
    preconditioner (the FIXED inner velocity operator, standing in for the
    paper's fixed inner cycles of Sec. 3.3; Saad, Iterative Methods for Sparse
    Linear Systems, Sec. 12.1): k steps of the Chebyshev iteration for
    D^-1 A z = D^-1 r from z = 0 on the interval [lo, hi] of D^-1 A (D = diag A).

    Written in closed form rather than as the three-term recurrence: the
    iteration's error after k steps is T_k((theta - M)/delta) / T_k(theta/delta)
    times the initial error (theta = (hi + lo)/2, delta = (hi - lo)/2, T_k the
    Chebyshev polynomial of the first kind), so
        z = (1 - T_k((theta - lambda)/delta) / T_k(theta/delta)) / lambda
    on every eigenpair of the symmetric S = D^-1/2 A D^-1/2, evaluated by a
    dense eigendecomposition (small A only).  r: [..., n] (rows along the last
    axis)."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=float)
    dh = 1.0 / np.sqrt(np.diag(A))
    S = dh[:, None] * A * dh[None, :]
    lam, Q = np.linalg.eigh(0.5 * (S + S.T))
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
    q = (1.0 - Tk((theta - lam) / delta) / Tk(theta / delta)) / lam
    r = np.asarray(r, dtype=float)
    y = (r * dh) @ Q          # rows of r in the eigenbasis of S
    return ((y * q) @ Q.T) * dh
