"""Seeded synthetic inputs for the generalized Stokes solve.

This module holds no part of the method: it only produces right-hand sides,
boundary data and random directions from seeds, as plain NumPy arrays in the
caller-facing layout ``[dim][n_p2]`` (component-major over every P2 node in the
natural numbering).  Node coordinates come in as arguments.

* ``fourier_forcing`` -- the smooth random forcing of the 3D workloads: a sum
  of 8 modes f_c(x) = sum_m a_{m,c} sin(pi k_m . x + phi_m) with k_m drawn from
  {1,2,3}^d, phi_m from [0, 2 pi) and a_{m,c} from [-1, 1], all drawn in that
  order from a SplitMix64 stream keyed by the seed (Steele, Lea & Flood 2014).
* ``manufactured_2d`` -- the divergence-free field of the paper's velocity
  test (Sec. 3.3.1, Eq. "divergence_free_velocity") with wave number pi
  instead of 16 pi, the pressure cos(pi x) cos(pi y), and the matching
  forcing f = alpha u - mu Laplacian(u) + grad p.
* ``fd_directions`` -- unit-RMS Gaussian directions for finite differences.
"""

import math

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


class SplitMix64:
    """Sequential SplitMix64 generator (Python ints, mod 2^64)."""

    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next_u64(self):
        self.state = (self.state + _GOLDEN) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self):
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * 2.0 ** -53


def fourier_modes(seed, dim, n_modes=8):
    """Mode parameters (k, phi, a) of the seeded Fourier forcing."""
    rng = SplitMix64(seed)
    ks, phis, amps = [], [], []
    for _ in range(n_modes):
        k = [1 + min(2, int(3.0 * rng.uniform())) for _ in range(dim)]
        phi = 2.0 * math.pi * rng.uniform()
        a = [2.0 * rng.uniform() - 1.0 for _ in range(dim)]
        ks.append(k)
        phis.append(phi)
        amps.append(a)
    return np.array(ks, dtype=np.float64), np.array(phis), np.array(amps)


def fourier_forcing(coords, seed, n_modes=8):
    """Nodal forcing (dim, n_nodes) at ``coords`` (n_nodes, dim)."""
    coords = np.asarray(coords, dtype=np.float64)
    dim = coords.shape[1]
    ks, phis, amps = fourier_modes(seed, dim, n_modes)
    f = np.zeros((dim, coords.shape[0]))
    for m in range(n_modes):
        s = np.sin(math.pi * (coords @ ks[m]) + phis[m])
        for c in range(dim):
            f[c] += amps[m, c] * s
    return f


def manufactured_2d(coords, mu, alpha):
    """u, p and f of the 2D manufactured solution at ``coords`` (n, 2).

    u = (sin pi x sin pi y, cos pi x cos pi y) is divergence free,
    p = cos pi x cos pi y has zero mean on the unit square, and
    f = alpha u - mu Laplacian(u) + grad p = (alpha + 2 pi^2 mu) u + grad p."""
    x, y = coords[:, 0], coords[:, 1]
    pi = math.pi
    u = np.stack([np.sin(pi * x) * np.sin(pi * y), np.cos(pi * x) * np.cos(pi * y)])
    p = np.cos(pi * x) * np.cos(pi * y)
    gp = np.stack([-pi * np.sin(pi * x) * np.cos(pi * y), -pi * np.cos(pi * x) * np.sin(pi * y)])
    f = (alpha + 2.0 * pi * pi * mu) * u + gp
    return u, p, f


def forcing_seed(mesh_seed, rhs_index=0):
    """Seed of the forcing of right-hand side ``rhs_index`` on a mesh seed."""
    return 1000 + int(mesh_seed) + 100 * int(rhs_index)


def target_seed(mesh_seed):
    """Seed of the forcing that defines the loss target u*."""
    return 9000 + int(mesh_seed)


def fd_directions(shape, count, seed):
    """``count`` Gaussian directions of ``shape`` scaled to unit RMS."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = rng.standard_normal(shape)
        out.append(v / np.sqrt(np.mean(v * v)))
    return out
