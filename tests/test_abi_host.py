"""Host-side checks of the C-ABI library (no GPU needed).

* the library loads and exports every entry point declared in include/stokes.h;
* the host mesh is bit-identical to the oracle's independent construction;
* the host sparsity patterns equal the oracle's (structural, explicit zeros kept);
* arguments are validated before any HIP call.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import p3 as op3
from oracle import stokes as ostokes
from paper_2407_01783_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "stokes.h")).read()
    declared = set(re.findall(r"\b(stokes_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("dim,n,seed,jit", [(2, 1, 0, 0.0), (2, 5, 3, 0.1), (3, 2, 0, 0.0), (3, 4, 7, 0.1),
                                            (3, 6, 1, 0.2)])
def test_mesh_bit_exact_vs_oracle(lib, dim, n, seed, jit):
    pr = _lib.make_problem(dim, n, seed, jit, 1.0, 1.0)
    m = omesh.KuhnMesh(dim, n, seed=seed, jitter=jit)
    vc = np.empty((m.n_p1, dim))
    el = np.empty((m.n_e, dim + 1), dtype=np.int32)
    pc = np.empty((m.n_p2, dim))
    p2 = np.empty((m.n_e, m.n_loc), dtype=np.int32)
    assert lib.stokes_build_mesh_host(ctypes.byref(pr), _lib.ptr(vc), _lib.ptr(el), _lib.ptr(pc), _lib.ptr(p2)) == 0
    assert np.array_equal(vc.view(np.uint64), m.vcoords.view(np.uint64))
    assert np.array_equal(pc.view(np.uint64), m.p2coords.view(np.uint64))
    assert np.array_equal(el, m.elems)
    assert np.array_equal(p2, m.p2)


def _pattern(lib, pr, which):
    nr, nz = ctypes.c_int64(), ctypes.c_int64()
    assert lib.stokes_host_pattern(ctypes.byref(pr), which, ctypes.byref(nr), ctypes.byref(nz), None, None) == 0
    rp = np.empty(nr.value + 1, dtype=np.int32)
    cols = np.empty(nz.value, dtype=np.int32)
    assert lib.stokes_host_pattern(ctypes.byref(pr), which, ctypes.byref(nr), ctypes.byref(nz), _lib.ptr(rp),
                                   _lib.ptr(cols)) == 0
    return rp, cols


@pytest.mark.parametrize("dim,n,jit", [(2, 4, 0.1), (2, 4, 0.0), (3, 3, 0.1), (3, 3, 0.0)])
def test_patterns_bit_exact_vs_oracle(lib, dim, n, jit):
    # unjittered meshes have exact cancellations in alpha M + mu L; the
    # pattern stays structural
    pr = _lib.make_problem(dim, n, 2, jit, 1.0, 1.0)
    s = ostokes.StokesSystem(omesh.KuhnMesh(dim, n, seed=2, jitter=jit), 1.0, 1.0)
    ref = {0: s.mats.Ms, 1: s.A_II, 2: s.mats.B[0], 3: s.B_I[0], 4: s.mats.MQ}
    for which, A in ref.items():
        rp, cols = _pattern(lib, pr, which)
        assert np.array_equal(rp, A.indptr), which
        assert np.array_equal(cols, A.indices), which


@pytest.mark.parametrize("dim,n,seed,jit", [(2, 1, 0, 0.0), (2, 4, 3, 0.1), (3, 1, 0, 0.0), (3, 3, 7, 0.15)])
def test_p3_mesh_bit_exact_vs_oracle(lib, dim, n, seed, jit):
    # the Taylor-Hood P3/P2 numbering (STOKES_FLAG_P3): P3 node ids and
    # coordinates bit-identical to the oracle's independent construction
    pr = _lib.make_problem(dim, n, seed, jit, 1.0, 1.0, 0.0, _lib.FLAG_P3)
    m = op3.P3P2Mesh(dim, n, seed=seed, jitter=jit)
    vc = np.empty((m.base.n_p1, dim))
    el = np.empty((m.n_e, dim + 1), dtype=np.int32)
    pc = np.empty((m.n_vel, dim))
    p3ids = np.empty((m.n_e, m.n_loc), dtype=np.int32)
    assert lib.stokes_build_mesh_host(ctypes.byref(pr), _lib.ptr(vc), _lib.ptr(el), _lib.ptr(pc),
                                      _lib.ptr(p3ids)) == 0
    assert np.array_equal(vc.view(np.uint64), m.vcoords.view(np.uint64))
    assert np.array_equal(el, m.elems)
    assert np.array_equal(p3ids, m.vel)
    assert np.array_equal(pc.view(np.uint64), m.vel_coords.view(np.uint64))
    s = (ctypes.c_int64 * 10)()
    assert lib.stokes_problem_sizes(ctypes.byref(pr), s) == 0
    assert s[0] == m.n_vel and s[1] == m.n_q and s[2] == m.n_free_nodes and s[6] == m.n_e


@pytest.mark.parametrize("dim,n,jit", [(2, 3, 0.1), (3, 2, 0.1), (3, 2, 0.0)])
def test_p3_patterns_bit_exact_vs_oracle(lib, dim, n, jit):
    pr = _lib.make_problem(dim, n, 2, jit, 1.0, 1.0, 0.0, _lib.FLAG_P3)
    m = op3.P3P2Mesh(dim, n, seed=2, jitter=jit)
    s = ostokes.StokesSystem(m, 1.0, 1.0, mats=op3.assemble_p3p2(m))
    ref = {0: s.mats.Ms, 1: s.A_II, 2: s.mats.B[0], 3: s.B_I[0], 4: s.mats.MQ}
    for which, A in ref.items():
        rp, cols = _pattern(lib, pr, which)
        assert np.array_equal(rp, A.indptr), which
        assert np.array_equal(cols, A.indices), which


def test_problem_sizes(lib):
    for n in (2, 3, 5):
        pr = _lib.make_problem(3, n, 0, 0.1, 1.0, 1.0)
        s = (ctypes.c_int64 * 10)()
        assert lib.stokes_problem_sizes(ctypes.byref(pr), s) == 0
        assert s[0] == (2 * n + 1) ** 3 and s[1] == (n + 1) ** 3 and s[2] == (2 * n - 1) ** 3
        assert s[3] == 230 * n ** 3 - 690 * n ** 2 + 732 * n - 273
        assert s[4] == 65 * n ** 3 - 111 * n ** 2 + 69 * n - 15
        assert s[5] == 15 * n ** 3 + 21 * n ** 2 + 9 * n + 1
        assert s[6] == 6 * n ** 3 and s[7] == 3


@pytest.mark.parametrize("field,value", [("dim", 4), ("n", 0), ("mu", 0.0), ("mu", float("nan")),
                                         ("alpha", -1.0), ("gamma", -0.5), ("jitter", 0.3), ("flags", 4)])
def test_invalid_problem_rejected(lib, field, value):
    pr = _lib.make_problem(3, 4, 0, 0.1, 1.0, 1.0)
    setattr(pr, field, value)
    out = ctypes.c_void_p()
    st = lib.stokes_assemble(ctypes.byref(pr), None, ctypes.byref(out))
    assert st == -1
    assert out.value is None
    assert len(lib.stokes_last_error()) > 0
    s = (ctypes.c_int64 * 10)()
    assert lib.stokes_problem_sizes(ctypes.byref(pr), s) == -1


def test_null_arguments_rejected(lib):
    o = _lib.default_opts()
    assert lib.stokes_solve_coupled(None, 1, None, None, None, None, None, None, ctypes.byref(o), None) == -1
    assert lib.stokes_solve_schur(None, 1, None, None, None, None, None, None, ctypes.byref(o), None) == -1
    assert lib.stokes_solve_adjoint(None, 1, None, None, None, None, None, None, None, ctypes.byref(o), None) == -1
    assert lib.stokes_apply(None, 0, 0, 1, None, None) == -1
    assert lib.stokes_set_mu(None, 1.0) == -1
    pr = _lib.make_problem(3, 2, 0, 0.0, 1.0, 1.0)
    assert lib.stokes_assemble(ctypes.byref(pr), None, None) == -1
    lib.stokes_destroy(None)   # no-op


def test_default_opts(lib):
    o = _lib.default_opts()
    assert o.rtol == 1e-8 and o.restart == 30 and o.cheb_degree == 4 and o.precision == 0
