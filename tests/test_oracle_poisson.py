"""Pins of the oracle's pressure Poisson solve against independent constructions.

* dense brute force: the D*G matrix assembled cell by cell from the
  staggered-grid stencil definition (Sec. 2.1), solved with numpy.linalg with a
  zero-mean constraint row;
* residual of the solution measured with a sparse operator built here;
* the oracle's Thomas routine against scipy.linalg.solve_banded;
* scipy's real/complex FFT against an O(N^2) DFT.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse

from oracle.ibm_oracle import OGrid, poisson_solve, thomas


def _grid(nx, ny, nz, lx=2.0, lz=1.3, ylo=-1.0, yhi=0.7):
    return OGrid(nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y_lo=ylo, y_hi=yhi, nu=0.01, dt=0.01)


def _dg_dense(g: OGrid) -> np.ndarray:
    """D G for pressure on the full box, assembled entry by entry.

    Flux through an x (z) face between cells i-1, i: (phi_i - phi_{i-1})/dx, periodic.
    Flux through a y face j (1 <= j <= ny-2): (phi_j - phi_{j-1})/dy; the box-wall
    faces j = 0 and j = ny-1 carry no flux.  D sums outgoing minus incoming fluxes.
    """
    n = g.ny - 1
    N = n * g.nz * g.nx
    L = np.zeros((N, N))

    def idx(j, k, i):
        return (j * g.nz + (k % g.nz)) * g.nx + (i % g.nx)

    for j in range(n):
        for k in range(g.nz):
            for i in range(g.nx):
                r = idx(j, k, i)
                for di in (-1, 1):
                    L[r, idx(j, k, i + di)] += 1.0 / g.dx ** 2
                    L[r, r] -= 1.0 / g.dx ** 2
                for dk in (-1, 1):
                    L[r, idx(j, k + dk, i)] += 1.0 / g.dz ** 2
                    L[r, r] -= 1.0 / g.dz ** 2
                if j + 1 <= n - 1:
                    L[r, idx(j + 1, k, i)] += 1.0 / g.dy ** 2
                    L[r, r] -= 1.0 / g.dy ** 2
                if j - 1 >= 0:
                    L[r, idx(j - 1, k, i)] += 1.0 / g.dy ** 2
                    L[r, r] -= 1.0 / g.dy ** 2
    return L


def _dg_sparse(g: OGrid):
    n = g.ny - 1
    J, K, I = np.meshgrid(np.arange(n), np.arange(g.nz), np.arange(g.nx), indexing="ij")
    r = ((J * g.nz + K) * g.nx + I).ravel()
    rows, cols, vals = [], [], []

    def add(mask, jj, kk, ii, val):
        rr = r[mask.ravel()]
        cc = ((jj * g.nz + kk % g.nz) * g.nx + ii % g.nx).ravel()[mask.ravel()]
        rows.extend([rr, rr]); cols.extend([cc, rr])
        vals.extend([np.full(rr.size, val), np.full(rr.size, -val)])

    allm = np.ones(J.shape, bool)
    add(allm, J, K, I + 1, 1 / g.dx ** 2); add(allm, J, K, I - 1, 1 / g.dx ** 2)
    add(allm, J, K + 1, I, 1 / g.dz ** 2); add(allm, J, K - 1, I, 1 / g.dz ** 2)
    add(J + 1 <= n - 1, np.minimum(J + 1, n - 1), K, I, 1 / g.dy ** 2)
    add(J - 1 >= 0, np.maximum(J - 1, 0), K, I, 1 / g.dy ** 2)
    N = n * g.nz * g.nx
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(N, N))


@pytest.mark.parametrize("shape", [(4, 5, 4), (6, 9, 6), (10, 7, 5), (5, 9, 3), (20, 5, 10), (160, 5, 4), (8, 3, 6)])
def test_poisson_matches_dense_bruteforce(shape):
    nx, ny, nz = shape
    g = _grid(nx, ny, nz)
    rng = np.random.default_rng(11)
    rhs = rng.standard_normal(g.shape)
    phi, mean_removed = poisson_solve(g, rhs)
    L = _dg_dense(g)
    N = L.shape[0]
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = L
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    sol = np.linalg.solve(M, np.concatenate([rhs.ravel(), [0.0]]))
    ref = sol[:N].reshape(g.shape)
    assert abs(mean_removed - rhs.mean()) < 1e-14
    err = np.abs(phi - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err
    assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()


@pytest.mark.parametrize("shape", [(32, 33, 16), (48, 17, 30), (64, 9, 10)])
def test_poisson_residual_sparse(shape):
    g = _grid(*shape)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(g.shape)
    phi, m = poisson_solve(g, rhs)
    L = _dg_sparse(g)
    res = (L @ phi.ravel()) - (rhs.ravel() - rhs.mean())
    assert np.abs(res).max() / np.abs(rhs).max() < 1e-13


def test_poisson_exact_mode():
    """A single discrete eigenmode is reproduced: cos in y (Neumann), Fourier in x, z."""
    g = _grid(12, 9, 10)
    n = g.ny - 1
    J, K, I = np.meshgrid(np.arange(n), np.arange(g.nz), np.arange(g.nx), indexing="ij")
    mx, mz, my = 2, 3, 1
    phi = np.cos(np.pi * my * (J + 0.5) / n) * np.cos(2 * np.pi * mx * I / g.nx) * np.sin(2 * np.pi * mz * K / g.nz)
    eig = -(4 / g.dx ** 2) * np.sin(np.pi * mx / g.nx) ** 2 - (4 / g.dz ** 2) * np.sin(np.pi * mz / g.nz) ** 2 \
        - (4 / g.dy ** 2) * np.sin(np.pi * my / (2 * n)) ** 2
    out, _ = poisson_solve(g, eig * phi)
    assert np.abs(out - phi).max() < 1e-12


def test_thomas_vs_solve_banded():
    rng = np.random.default_rng(3)
    n, m = 37, 5
    lower = rng.uniform(0.5, 1.0, (n, m)); lower[0] = 0
    upper = rng.uniform(0.5, 1.0, (n, m)); upper[-1] = 0
    diag = -(lower + upper) - rng.uniform(0.1, 1.0, (n, m))
    rhs = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    x = thomas(lower, diag, upper, rhs)
    for c in range(m):
        ab = np.zeros((3, n), dtype=np.complex128)
        ab[0, 1:] = upper[:-1, c]
        ab[1] = diag[:, c]
        ab[2, :-1] = lower[1:, c]
        ref = scipy.linalg.solve_banded((1, 1), ab, rhs[:, c])
        assert np.abs(x[:, c] - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [6, 15, 20, 32])
def test_fft_vs_direct_dft(n):
    import scipy.fft
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    W = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    assert np.abs(scipy.fft.rfft(x) - (W @ x)[: n // 2 + 1]).max() < 1e-12
    z = x + 1j * rng.standard_normal(n)
    assert np.abs(scipy.fft.fft(z) - W @ z).max() < 1e-12
