"""PyTorch-facing wrapper of the C ABI: device tensors in, device tensors out.

Only argument marshalling happens here; every step of the solve runs in the
HIP library.  Tensors are float64 on the context's device, in the caller
layout of ``include/stokes.h``: velocity-shaped [nrhs, dim, n_p2], pressure
[nrhs, n_p1].
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, ptr


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class StokesProblem:
    """An assembled generalized Stokes operator on the Kuhn mesh (one GPU)."""

    def __init__(self, dim, n, mesh_seed=0, jitter=0.0, mu=1.0, alpha=1.0, gamma=0.0, strain=False, p3=False):
        """strain=True: velocity matrix alpha M + mu (L + D) (the strain-rate
        form); otherwise alpha M + mu L (vector Laplacian).  p3=True: the
        Taylor-Hood P3/P2 pair (velocity arrays over the (3n+1)^dim P3 nodes,
        pressure over the (2n+1)^dim P2 nodes); otherwise P2/P1."""
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("StokesProblem needs a HIP device")
        self.strain = bool(strain)
        self.p3 = bool(p3)
        self.prob = _lib.make_problem(dim, n, mesh_seed, jitter, mu, alpha, gamma,
                                      (_lib.FLAG_STRAIN if strain else 0) | (_lib.FLAG_P3 if p3 else 0))
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(self.lib.stokes_assemble(ctypes.byref(self.prob), _stream_handle(), ctypes.byref(h)),
              "stokes_assemble")
        self.ctx = h
        s = (ctypes.c_int64 * 12)()
        check(self.lib.stokes_query(self.ctx, s), "stokes_query")
        (self.n_p2, self.n_p1, self.n_free_nodes, self.nnz_A, self.nnz_B, self.nnz_Q, self.n_elem, self.dim,
         self.nnz_full, self.nnz_Bfull, self.nnz_X, self.affine_slices) = [int(v) for v in s]
        if self.p3:
            self.n_loc = 20 if self.dim == 3 else 10
        else:
            self.n_loc = 10 if self.dim == 3 else 6

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.lib.stokes_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    # ----------------------------------------------------------- metadata
    @property
    def mu(self):
        return self.prob.mu

    def set_mu(self, mu):
        check(self.lib.stokes_set_mu(self.ctx, float(mu)), "stokes_set_mu")
        self.prob.mu = float(mu)

    def total_dofs(self):
        """Velocity (all P2 nodes x dim) plus pressure degrees of freedom."""
        return self.dim * self.n_p2 + self.n_p1

    def mesh(self):
        """P2 node coordinates (n_p2, dim) and simplex P2 ids (n_elem, n_loc), numpy."""
        xy = np.empty((self.n_p2, self.dim))
        p2 = np.empty((self.n_elem, self.n_loc), dtype=np.int32)
        check(self.lib.stokes_export_mesh(self.ctx, ptr(xy), ptr(p2)), "stokes_export_mesh")
        return xy, p2

    def export_csr(self, which):
        """(rowptr, cols, vals) numpy arrays of an assembled FP64 matrix."""
        if which >= 10:
            nrows, nnz = self.n_p2, self.nnz_full
            rp = np.empty(nrows + 1, dtype=np.int32)
            cols = np.empty(nnz, dtype=np.int32)
            vals = np.empty(nnz)
            check(self.lib.stokes_export_csr(self.ctx, int(which), ptr(rp), ptr(cols), ptr(vals)), "stokes_export_csr")
            return rp, cols, vals
        if which == 8:
            vals = np.empty(self.n_p2)
            check(self.lib.stokes_export_csr(self.ctx, 8, None, None, ptr(vals)), "stokes_export_csr")
            return None, None, vals
        if which in (0, 1):
            nrows, nnz = self.n_p2, self.nnz_full
        elif which in (2, 3, 4):
            nrows, nnz = self.n_p1, self.nnz_Bfull
        elif which in (5, 6):
            nrows, nnz = self.n_p1, self.nnz_Q
        elif which == 9:
            nrows, nnz = self.n_p1, self.nnz_X
        else:
            nrows, nnz = self.n_free_nodes, self.nnz_A
        rp = np.empty(nrows + 1, dtype=np.int32)
        cols = np.empty(nnz, dtype=np.int32)
        vals = np.empty(nnz)
        check(self.lib.stokes_export_csr(self.ctx, int(which), ptr(rp), ptr(cols), ptr(vals)), "stokes_export_csr")
        return rp, cols, vals

    def bounds(self):
        b = (ctypes.c_double * 8)()
        check(self.lib.stokes_bounds(self.ctx, b), "stokes_bounds")
        return list(b)

    # ----------------------------------------------------------- tensors
    def _vel(self, x, nrhs):
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        if x.numel() != nrhs * self.dim * self.n_p2:
            raise ValueError(f"velocity array must have {nrhs} x {self.dim} x {self.n_p2} entries")
        return x.view(nrhs, self.dim, self.n_p2)

    def _pres(self, x, nrhs):
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        if x.numel() != nrhs * self.n_p1:
            raise ValueError(f"pressure array must have {nrhs} x {self.n_p1} entries")
        return x.view(nrhs, self.n_p1)

    def _nrhs(self, f):
        f = torch.as_tensor(f)
        if f.dim() == 2:
            return 1
        return int(f.shape[0])

    # ----------------------------------------------------------- solves
    def solve(self, f, ubc=None, method="coupled", x0=None, hist_cap=0, **opts):
        """Solve for (u, p); returns (u, p, info dict).  f: [nrhs,] dim, n_p2.
        hist_cap > 0 returns up to that many residual-history entries as
        info["res_hist"]."""
        nrhs = self._nrhs(f)
        f = self._vel(f, nrhs)
        ubc = self._vel(ubc, nrhs) if ubc is not None else None
        u = torch.empty_like(f)
        p = torch.empty((nrhs, self.n_p1), dtype=torch.float64, device=self.device)
        x0u = x0p = None
        if x0 is not None:
            x0u, x0p = self._vel(x0[0], nrhs), self._pres(x0[1], nrhs)
        o = _lib.default_opts(**opts)
        info = _lib.SolveInfo()
        if hist_cap > 0:
            info.attach_history(hist_cap)
        fn = self.lib.stokes_solve_coupled if method == "coupled" else self.lib.stokes_solve_schur
        if method not in ("coupled", "schur"):
            raise ValueError("method must be 'coupled' or 'schur'")
        check(self.lib.stokes_set_stream(self.ctx, _stream_handle()))
        status = check(fn(self.ctx, nrhs, ptr(f), ptr(ubc), ptr(x0u), ptr(x0p), ptr(u), ptr(p),
                          ctypes.byref(o), ctypes.byref(info)), f"stokes_solve_{method}")
        d = info.as_dict()
        d["status"] = status
        return u, p, d

    def projection_step(self, f, p_old=None, ubc=None, **opts):
        """One pressure-correction step (stokes_projection_step); returns (u, p, info)."""
        nrhs = self._nrhs(f)
        f = self._vel(f, nrhs)
        ubc = self._vel(ubc, nrhs) if ubc is not None else None
        p_old = self._pres(p_old, nrhs) if p_old is not None else None
        u = torch.empty_like(f)
        p = torch.empty((nrhs, self.n_p1), dtype=torch.float64, device=self.device)
        o = _lib.default_opts(**opts)
        info = _lib.SolveInfo()
        check(self.lib.stokes_set_stream(self.ctx, _stream_handle()))
        status = check(self.lib.stokes_projection_step(self.ctx, nrhs, ptr(f), ptr(ubc), ptr(p_old), ptr(u), ptr(p),
                                                       ctypes.byref(o), ctypes.byref(info)), "stokes_projection_step")
        d = info.as_dict()
        d["status"] = status
        return u, p, d

    def adjoint(self, u, dJdu, dJdp=None, **opts):
        """Adjoint solve; returns (lam_u, lam_p, dJdf, dJdmu, info)."""
        nrhs = self._nrhs(u)
        u = self._vel(u, nrhs)
        dJdu = self._vel(dJdu, nrhs)
        dJdp = self._pres(dJdp, nrhs) if dJdp is not None else None
        lam_u = torch.empty_like(u)
        dJdf = torch.empty_like(u)
        lam_p = torch.empty((nrhs, self.n_p1), dtype=torch.float64, device=self.device)
        dJdmu = torch.empty(nrhs, dtype=torch.float64, device=self.device)
        o = _lib.default_opts(**opts)
        info = _lib.SolveInfo()
        check(self.lib.stokes_set_stream(self.ctx, _stream_handle()))
        status = check(self.lib.stokes_solve_adjoint(self.ctx, nrhs, ptr(u), ptr(dJdu), ptr(dJdp), ptr(lam_u),
                                                     ptr(lam_p), ptr(dJdf), ptr(dJdmu), ctypes.byref(o),
                                                     ctypes.byref(info)), "stokes_solve_adjoint")
        d = info.as_dict()
        d["status"] = status
        return lam_u, lam_p, dJdf, dJdmu, d

    def apply(self, op, x, precision=0, nrhs=1):
        """One assembled operator (see stokes_apply) on caller-layout tensors."""
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        nu, npr = nrhs * self.dim * self.n_p2, nrhs * self.n_p1
        out_len = {0: nu, 1: npr, 2: nu, 3: npr, 4: npr, 5: nu + npr, 6: npr, 7: npr, 8: npr, 9: nu, 10: nu}[op]
        y = torch.empty(out_len, dtype=torch.float64, device=self.device)
        check(self.lib.stokes_set_stream(self.ctx, _stream_handle()))
        check(self.lib.stokes_apply(self.ctx, int(op), int(precision), int(nrhs), ptr(x), ptr(y)), "stokes_apply")
        return y

    def residual(self, f, u, p, ubc=None):
        """True relative residual per right-hand side (numpy array)."""
        nrhs = self._nrhs(f)
        f, u, p = self._vel(f, nrhs), self._vel(u, nrhs), self._pres(p, nrhs)
        ubc = self._vel(ubc, nrhs) if ubc is not None else None
        out = (ctypes.c_double * nrhs)()
        check(self.lib.stokes_set_stream(self.ctx, _stream_handle()))
        check(self.lib.stokes_residual(self.ctx, nrhs, ptr(f), ptr(ubc), ptr(u), ptr(p), out), "stokes_residual")
        return np.array(out[:])


class StokesSolve(torch.autograd.Function):
    """u, p = StokesSolve.apply(f, mu, problem, opts): differentiable in f and mu.

    The backward pass is the adjoint Stokes solve of the library
    (stokes_solve_adjoint): dJ/df = M_V[I,:]^T lam_u and
    dJ/dmu = -lam_u^T L_V[I,:] u."""

    @staticmethod
    def forward(ctx, f, mu, problem, opts):
        mu_val = float(mu)
        if mu_val != problem.mu:
            problem.set_mu(mu_val)
        opts = dict(opts or {})
        method = opts.pop("method", "coupled")
        u, p, info = problem.solve(f, method=method, **opts)
        if info["status"] != 0:
            raise _lib.StokesError(info["status"], "forward solve did not converge")
        ctx.problem, ctx.opts = problem, opts
        ctx.mu_val = mu_val  # the operator of this solve, restored for the adjoint
        ctx.shape = f.shape
        ctx.mu_like = mu if torch.is_tensor(mu) else None
        ctx.save_for_backward(u)
        return u.view(f.shape), p.view(f.shape[:-2] + (problem.n_p1,)) if f.dim() == 3 else p.view(problem.n_p1)

    @staticmethod
    def backward(ctx, grad_u, grad_p):
        (u,) = ctx.saved_tensors
        prob = ctx.problem
        nrhs = u.shape[0]
        gu = torch.zeros_like(u) if grad_u is None else grad_u.reshape(u.shape)
        gp = None if grad_p is None else grad_p.reshape(nrhs, prob.n_p1)
        # the adjoint needs the forward solve's operator: another solve on the
        # same problem (or a set_mu call) may have changed mu since
        mu_now = prob.mu
        if mu_now != ctx.mu_val:
            prob.set_mu(ctx.mu_val)
        try:
            _, _, dJdf, dJdmu, info = prob.adjoint(u, gu, gp, **ctx.opts)
        finally:
            if mu_now != ctx.mu_val:
                prob.set_mu(mu_now)
        if info["status"] != 0:
            raise _lib.StokesError(info["status"], "adjoint solve did not converge")
        gmu = None
        if ctx.mu_like is not None:
            gmu = dJdmu.sum().to(device=ctx.mu_like.device, dtype=ctx.mu_like.dtype).reshape(ctx.mu_like.shape)
        return dJdf.view(ctx.shape), gmu, None, None
