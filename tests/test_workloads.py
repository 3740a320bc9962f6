"""Pins of the finite-volume generator (the inputs both the library and the
oracle are checked on; the library's own FV assembly is compared with it
bit-exactly on the GPU): the textbook 5-/7-point stencil for constant kappa,
symmetry and harmonic face coefficients without convection, and the M-matrix
structure and row sums the boundary conditions fix with convection."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _dense(n, dim, kappa, vel=None):
    rp, ci, v = W.fv_matrix(n, dim, kappa, vel)
    N = n ** dim
    return sp.csr_matrix((v, ci, rp), shape=(N, N)).toarray()


def _coords(n, dim):
    idx = np.arange(n ** dim)
    return [(idx // n ** d) % n for d in range(dim)]   # x fastest


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_kappa_is_the_textbook_stencil(dim):
    """kappa = 1, no convection: an interior row is (2 dim, -1 x 2 dim) / h^2;
    a row without a Dirichlet face (faces y = 0, 1) sums to zero; each
    Dirichlet face adds 2 / h^2 to its row."""
    n = 6
    h = 1.0 / n
    A = _dense(n, dim, np.ones(n ** dim))
    c = _coords(n, dim)
    interior = np.all([(cd > 0) & (cd < n - 1) for cd in c], axis=0)
    for i in np.flatnonzero(interior)[:10]:
        row = A[i] * h * h
        assert row[i] == 2 * dim
        nb = [i + s * n ** d for d in range(dim) for s in (-1, 1)]
        assert np.all(row[nb] == -1.0)
        assert np.count_nonzero(row) == 2 * dim + 1
    dir_faces = (c[1] == 0).astype(int) + (c[1] == n - 1).astype(int)
    assert np.allclose(A.sum(axis=1) * h * h, 2.0 * dir_faces, rtol=0, atol=1e-12)


def test_diffusion_only_is_symmetric_with_harmonic_faces():
    """Without convection A is symmetric for any kappa, and the entry between
    two neighbouring cells is -2 kc km / ((kc + km) h^2)."""
    n = 12
    h = 1.0 / n
    kap = W.block_kappa(n, 2, 4, -3, 3, np.random.default_rng(3))
    A = _dense(n, 2, kap)
    assert np.array_equal(A, A.T)
    for i in (13, 50, 77):
        for m in (i + 1, i + n):
            ref = -2 * kap[i] * kap[m] / ((kap[i] + kap[m]) * h * h)
            assert np.isclose(A[i, m], ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", ["rotating", "constant"])
def test_convection_m_matrix_and_row_sums(case):
    """First-order upwind with face velocities of a divergence-free field:
    off-diagonals <= 0 < diagonal, and a row without a Dirichlet face sums to
    the inflow through its Neumann boundary faces divided by h (the interior
    faces' upwind terms and the outflow cancel by zero divergence; the inflow
    term is the one a zero boundary value drops): zero for the rotating field
    (no normal flow on the boundary), a_x / h on the column x = 0 for
    a = (1, 0.5)."""
    n = 16
    h = 1.0 / n
    kap = W.block_kappa(n, 2, 4, -2, 2, np.random.default_rng(4))
    vel = W.velocity_rotating(10.0) if case == "rotating" else W.velocity_const((1.0, 0.5))
    A = _dense(n, 2, kap, vel)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0) and np.all(np.diag(A) > 0)
    x, y = _coords(n, 2)
    free = (y > 0) & (y < n - 1)
    sums = A.sum(axis=1)[free]
    expect = np.zeros(n * n)
    if case == "constant":
        expect[x == 0] = 1.0 / h
    scale = np.abs(A).sum(axis=1)[free]
    assert np.all(np.abs(sums - expect[free]) <= 1e-12 * scale)


@pytest.mark.parametrize("dims", [(5, 3, 4), (13, 9, 21), (7, 1, 6)])
def test_grid7_pattern_and_dominance(dims):
    """The seven-point generator of the 3D wavefront tests: in natural order
    every off-diagonal entry sits at offset +-1 within a grid line, +-nx
    within a plane or +-nx*ny, every existing neighbour is present, the
    off-diagonals are negative and nonsymmetric, and each diagonal is 1.05
    times the row's off-diagonal magnitudes plus 0.01."""
    nx, ny, nz = dims
    rp, ci, v = W.grid7_matrix(nx, ny, nz, 3)
    n = nx * ny * nz
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    assert np.all(np.diff(rp) > 0) and A.has_sorted_indices
    for i in range(n):
        x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
        want = {i}
        if x > 0: want.add(i - 1)
        if x < nx - 1: want.add(i + 1)
        if y > 0: want.add(i - nx)
        if y < ny - 1: want.add(i + nx)
        if z > 0: want.add(i - nx * ny)
        if z < nz - 1: want.add(i + nx * ny)
        assert set(ci[rp[i]:rp[i + 1]]) == want
    D = A.diagonal()
    off = A - sp.diags(D)
    assert np.all(off.data <= 0)
    assert np.allclose(D, 1.05 * np.asarray(abs(off).sum(axis=1)).ravel() + 0.01, rtol=1e-15, atol=0)
    assert abs(off - off.T).max() > 0
