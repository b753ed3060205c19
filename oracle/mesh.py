"""Structured Kuhn mesh of the unit square/cube with P2/P1 Taylor-Hood numbering.

Test infrastructure only (see the package header).

The paper works on unstructured 2D meshes that are not distributed with it
(Sec. 3.1, "nonuniform triangular meshes"); the synthetic stand-in used here is
the unit square or unit cube cut into n^d cells, each split into d! simplices
(the Kuhn / Freudenthal split), with interior vertices moved by a seeded
uniform jitter.  All conventions below are readings, not the paper's:

* vertex (i, j[, k]) has id  i + (n+1) j [+ (n+1)^2 k]          (x fastest)
* cell (i, j[, k]) is visited x fastest; inside a cell the simplices follow
  the permutations pi of the axes in lexicographic order; the simplex of pi is
  (v0, v0 + e_pi0, v0 + e_pi0 + e_pi1, ..., v0 + (1,..,1)).
* local P2 nodes: vertices 0..d, then the edges (0,1),(0,2),(0,3),(1,2),(1,3),
  (2,3) in 3D, (0,1),(0,2),(1,2) in 2D.
* P2 node = point of the refined (2n+1)^d grid: vertex v -> 2v, edge (a,b) ->
  v_a + v_b (integer grid coordinates); id = I + (2n+1) J [+ (2n+1)^2 K].
* jitter: U = (mix(seed + (d*g + c + 1) * 0x9E3779B97F4A7C15) >> 11) * 2^-53
  with mix the SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014),
  arithmetic mod 2^64, g the vertex id and c the component; the shift is
  delta = (2U - 1) * jitter and x_c = (i_c + delta) / n, each step one IEEE
  double operation.  Boundary vertices do not move.  Edge nodes sit at
  (x_a + x_b) * 0.5.
"""

from itertools import permutations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    """SplitMix64 finaliser on uint64 arrays (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def jitter_unit(seed, counter):
    """U in [0, 1) from the counter-based SplitMix64 stream keyed by ``seed``."""
    counter = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter + np.uint64(1)) * GOLDEN_GAMMA
    return (splitmix64_mix(z) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def local_edges(dim):
    """Local edge list of a simplex in the reading's order."""
    nv = dim + 1
    return [(a, b) for a in range(nv) for b in range(a + 1, nv)]


class KuhnMesh:
    """Kuhn mesh + P2/P1 numbering of the unit square (dim 2) or cube (dim 3).

    Attributes
    ----------
    vcoords : (n_p1, dim) float64   jittered vertex coordinates (P1 nodes)
    vgrid   : (n_p1, dim) int64     integer grid position of every vertex
    elems   : (n_e, dim+1) int64    vertex ids of each simplex
    p2      : (n_e, n_loc) int64    P2 node ids of each simplex (local order)
    p2grid  : (n_p2, dim) int64     refined-grid position of every P2 node
    p2coords: (n_p2, dim) float64   P2 node coordinates
    """

    def __init__(self, dim, n, seed=0, jitter=0.0):
        if dim not in (2, 3) or n < 1:
            raise ValueError("dim must be 2 or 3 and n >= 1")
        self.dim, self.n, self.seed, self.jitter = dim, n, int(seed), float(jitter)
        nv1 = n + 1
        self.n_p1 = nv1 ** dim
        self.n_p2 = (2 * n + 1) ** dim

        # vertex grid, x fastest
        ids = np.arange(self.n_p1)
        vgrid = np.empty((self.n_p1, dim), dtype=np.int64)
        rem = ids.copy()
        for c in range(dim):
            vgrid[:, c] = rem % nv1
            rem //= nv1
        self.vgrid = vgrid

        # coordinates with jitter on interior vertices
        interior = np.all((vgrid > 0) & (vgrid < n), axis=1)
        vc = np.empty((self.n_p1, dim), dtype=np.float64)
        for c in range(dim):
            counter = np.uint64(dim) * ids.astype(np.uint64) + np.uint64(c)
            u = jitter_unit(self.seed, counter)
            delta = (2.0 * u - 1.0) * self.jitter
            shifted = np.where(interior, vgrid[:, c].astype(np.float64) + delta,
                               vgrid[:, c].astype(np.float64))
            vc[:, c] = shifted / float(n)
        self.vcoords = vc

        # simplices
        perms = list(permutations(range(dim)))  # lexicographic order
        ncell = n ** dim
        cell = np.arange(ncell)
        cgrid = np.empty((ncell, dim), dtype=np.int64)
        rem = cell.copy()
        for c in range(dim):
            cgrid[:, c] = rem % n
            rem //= n
        stride = np.array([nv1 ** c for c in range(dim)], dtype=np.int64)
        elems = np.empty((ncell, len(perms), dim + 1), dtype=np.int64)
        for q, pi in enumerate(perms):
            pos = cgrid.copy()
            elems[:, q, 0] = pos @ stride
            for s in range(dim):
                pos = pos.copy()
                pos[:, pi[s]] += 1
                elems[:, q, s + 1] = pos @ stride
        self.elems = elems.reshape(ncell * len(perms), dim + 1)
        self.n_e = self.elems.shape[0]

        # P2 nodes on the refined grid
        n2 = 2 * n + 1
        stride2 = np.array([n2 ** c for c in range(dim)], dtype=np.int64)
        edges = local_edges(dim)
        self.n_loc = dim + 1 + len(edges)
        p2 = np.empty((self.n_e, self.n_loc), dtype=np.int64)
        eg = vgrid[self.elems]  # (n_e, d+1, dim)
        for a in range(dim + 1):
            p2[:, a] = (2 * eg[:, a, :]) @ stride2
        for q, (a, b) in enumerate(edges):
            p2[:, dim + 1 + q] = (eg[:, a, :] + eg[:, b, :]) @ stride2
        self.p2 = p2

        rem = np.arange(self.n_p2)
        p2grid = np.empty((self.n_p2, dim), dtype=np.int64)
        for c in range(dim):
            p2grid[:, c] = rem % n2
            rem //= n2
        self.p2grid = p2grid

        # P2 coordinates: vertices copy, edge midpoints average
        p2c = np.full((self.n_p2, dim), np.nan)
        seen = np.zeros(self.n_p2, dtype=bool)
        for a in range(dim + 1):
            p2c[p2[:, a]] = vc[self.elems[:, a]]
            seen[p2[:, a]] = True
        for q, (a, b) in enumerate(edges):
            node = p2[:, dim + 1 + q]
            p2c[node] = (vc[self.elems[:, a]] + vc[self.elems[:, b]]) * 0.5
            seen[node] = True
        if not seen.all():
            raise AssertionError("P2 numbering is not onto the refined grid")
        self.p2coords = p2c

        # boundary flags (Dirichlet on the whole boundary, Sec. 3.1)
        self.p2_boundary = np.any((p2grid == 0) | (p2grid == 2 * n), axis=1)
        self.p2_interior = ~self.p2_boundary
        self.interior_nodes = np.nonzero(self.p2_interior)[0]
        self.n_free_nodes = self.interior_nodes.size

    def element_vertices(self):
        """(n_e, d+1, d) coordinates of each simplex's vertices."""
        return self.vcoords[self.elems]
