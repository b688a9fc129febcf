"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method: it only draws random numbers
and shapes them into fields in the natural layouts

    gauge  U[mu][t][z][y][x][3][3]   (mu = 0..3 <-> x, y, z, t)
    5D     psi[s][t][z][y][x][4][3]

The recipe (the paper's thermalised ensembles are not available):
  * links U = exp(i eps H), H = (A + A^dag)/2 - tr(.)/3 with A_ij having
    independent N(0,1) real and imaginary parts; the exponential is taken
    through numpy's Hermitian eigendecomposition;
  * sources: independent N(0,1) real and imaginary parts per component;
  * every draw comes from numpy.random.default_rng(seed).
"""
import numpy as np


def _rng(seed):
    return np.random.default_rng(int(seed))


def random_hermitian_traceless(rng, n):
    """n random traceless Hermitian 3x3 matrices (Gaussian entries)."""
    A = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[:, None, None] * np.eye(3)[None]
    return H


def expi_hermitian(H, eps):
    """exp(i eps H) for a stack of Hermitian matrices via eigh (unitary, det 1 when traceless)."""
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", V, ph, np.conj(V))


def random_links(dims, eps, seed):
    """SU(3) gauge field U = exp(i eps H), shape (4, T, Z, Y, X, 3, 3)."""
    X, Y, Z, T = dims
    rng = _rng(seed)
    n = 4 * X * Y * Z * T
    H = random_hermitian_traceless(rng, n)
    U = expi_hermitian(H, eps)
    return U.reshape(4, T, Z, Y, X, 3, 3)


def unit_links(dims):
    X, Y, Z, T = dims
    U = np.zeros((4, T, Z, Y, X, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_gauge_transform(dims, seed, eps=1.0):
    """Random SU(3) matrix per 4D site, shape (T, Z, Y, X, 3, 3)."""
    X, Y, Z, T = dims
    rng = _rng(seed)
    H = random_hermitian_traceless(rng, X * Y * Z * T)
    return expi_hermitian(H, eps).reshape(T, Z, Y, X, 3, 3)


def gaussian_spinor(dims, Ls, seed):
    """Gaussian complex 5D spinor, shape (Ls, T, Z, Y, X, 4, 3)."""
    X, Y, Z, T = dims
    rng = _rng(seed)
    shape = (Ls, T, Z, Y, X, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def parity_array(dims):
    """4D checkerboard parity (x+y+z+t) mod 2, shape (T, Z, Y, X)."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return (x + y + z + t) & 1


def gaussian_spinor_parity(dims, Ls, seed, parity):
    """Gaussian 5D spinor supported on one 4D parity (zero elsewhere)."""
    psi = gaussian_spinor(dims, Ls, seed)
    mask = parity_array(dims) == parity
    psi[:, ~mask] = 0
    return psi


def random_su3_algebra(n, seed):
    """n random real 8-vectors (coefficients of the generators)."""
    return _rng(seed).standard_normal((n, 8))


def random_momenta(dims, seed):
    """Gaussian momenta P = i H on every link, H Hermitian traceless distributed as
    sum_a p_a lambda_a / 2 with independent p_a ~ N(0, 1) (Gell-Mann matrices lambda_a): the
    off-diagonal entries (x + i y) / 2, x, y ~ N(0, 1); the diagonal (p3 / 2 + p8 / (2 sqrt 3),
    -p3 / 2 + p8 / (2 sqrt 3), -p8 / sqrt 3).  Shape [4][T][Z][Y][X][3][3]."""
    X, Y, Z, T = dims
    rng = _rng(seed)
    n = 4 * X * Y * Z * T
    H = np.zeros((n, 3, 3), np.complex128)
    for (i, j) in ((0, 1), (0, 2), (1, 2)):
        v = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / 2
        H[:, i, j] = v
        H[:, j, i] = np.conj(v)
    p3, p8 = rng.standard_normal(n), rng.standard_normal(n)
    H[:, 0, 0] = p3 / 2 + p8 / (2 * np.sqrt(3))
    H[:, 1, 1] = -p3 / 2 + p8 / (2 * np.sqrt(3))
    H[:, 2, 2] = -p8 / np.sqrt(3)
    return (1j * H).reshape((4, T, Z, Y, X, 3, 3))


def sample_links(dims, count, seed):
    """Seeded choice of (mu, t, z, y, x, a) link/generator coordinates."""
    X, Y, Z, T = dims
    rng = _rng(seed)
    mu = rng.integers(0, 4, count)
    t = rng.integers(0, T, count)
    z = rng.integers(0, Z, count)
    y = rng.integers(0, Y, count)
    x = rng.integers(0, X, count)
    a = rng.integers(0, 8, count)
    return list(zip(mu.tolist(), t.tolist(), z.tolist(), y.tolist(), x.tolist(), a.tolist()))


# Seeds used across the suite and the benchmark (links 1000 + cfg, sources 2000 + 10 cfg + rhs)
def link_seed(cfg):
    return 1000 + int(cfg)


def source_seed(cfg, rhs=0):
    return 2000 + 10 * int(cfg) + int(rhs)
