"""Seeded synthetic inputs for the REXII shallow-water workloads.

This module holds no part of the method's arithmetic: it only draws initial
states, depth fields and sample indices.  Both the HIP path's tests/benchmark
and the CPU oracle take their inputs from here.

Recipes (all grids are the periodic unit square, point (i, j) at
x = i/nx, y = j/ny, fields stored [c][j][i] with c in (eta, u, v)):

* ``gaussian_bumps``: eta = sum_b a_b exp(-d_b^2 / (2 sigma_b^2)) with d_b the
  periodic minimum-image distance to the centre c_b; centres uniform in
  [0,1)^2.  One bump: sigma = 0.05, a = 1.  Several bumps: sigma ~ U[0.02,
  0.08], a ~ N(0, 1).  Velocities zero unless ``velocity=True`` (then u and v
  are two further bump sums, amplitude scaled by 0.1).
* ``variable_depth``: H(x, y) = 1 + 0.3 sin(2 pi x) cos(2 pi y).
* ``sample_indices``: distinct flat indices of eta points.
* ``batched_instances``: grid sizes drawn from {128, 256, 512, 1024} and
  t*rho from U[lo, hi], one generator per instance seed.
"""
import numpy as np


def _bump_sum(nx, ny, rng, nbumps, sigma=None, amp=None):
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    out = np.zeros((ny, nx))
    for _ in range(nbumps):
        cx, cy = rng.random(2)
        s = sigma if sigma is not None else rng.uniform(0.02, 0.08)
        a = amp if amp is not None else rng.normal()
        ddx = (x - cx + 0.5) % 1.0 - 0.5
        ddy = (y - cy + 0.5) % 1.0 - 0.5
        out += a * np.exp(-(ddy[:, None] ** 2 + ddx[None, :] ** 2) / (2.0 * s * s))
    return out


def gaussian_bumps(nx, ny=None, nbumps=1, seed=1, velocity=False):
    """Initial state f[3][ny][nx] (float64) made of Gaussian bumps."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    f = np.zeros((3, ny, nx))
    if nbumps == 1:
        f[0] = _bump_sum(nx, ny, rng, 1, sigma=0.05, amp=1.0)
    else:
        f[0] = _bump_sum(nx, ny, rng, nbumps)
    if velocity:
        f[1] = 0.1 * _bump_sum(nx, ny, rng, max(1, nbumps))
        f[2] = 0.1 * _bump_sum(nx, ny, rng, max(1, nbumps))
    return f


def variable_depth(nx, ny=None, amp=0.3):
    """H(x, y) = 1 + amp sin(2 pi x) cos(2 pi y) on the grid, [ny][nx]."""
    ny = nx if ny is None else ny
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    return 1.0 + amp * np.cos(2 * np.pi * y)[:, None] * np.sin(2 * np.pi * x)[None, :]


def sample_indices(nx, ny, count, seed):
    """count distinct flat indices j*nx + i of eta points, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(nx * ny, size=count, replace=False)).astype(np.int64)


def batched_instances(count=64, seed0=300, sizes=(128, 256, 512, 1024),
                      trho_range=(50.0, 2000.0), nbumps=16):
    """List of dicts (D, trho, seed) for heterogeneous batches."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        D = int(rng.choice(sizes))
        trho = float(rng.uniform(*trho_range))
        out.append(dict(D=D, trho=trho, seed=seed0 + i, nbumps=nbumps))
    return out


# ----------------------------------------------------------------------------
# the paper's matrix test cases (Sec. 3.2): circulant matrices as stencils
# {offset d: coefficient c_d}, (A f)_j = sum_d c_d f_{(j + d) mod n}
# ----------------------------------------------------------------------------
def advection_stencil(n):
    """A_1: centred difference of d/dx, periodic on [0, 1] with step 1/n."""
    return {1: 0.5 * n, -1: -0.5 * n}


def schroedinger_stencil(n, length=2.0):
    """A_2: i times the second difference of d^2/dx^2, periodic on an
    interval of the given length with step length / n."""
    c = (n / length) ** 2
    return {-1: 1j * c, 0: -2j * c, 1: 1j * c}


def matrix_case_vector(n, start=0.0, length=1.0):
    """f_0 = (2 + cos(2 pi x))^{-1} at x = start + length j / n."""
    x = start + length * np.arange(n) / n
    return 1.0 / (2.0 + np.cos(2.0 * np.pi * x))


def random_vectors(n, count, seed):
    """count standard-normal vectors of length n, [count][n]."""
    return np.random.default_rng(seed).standard_normal((count, n))
