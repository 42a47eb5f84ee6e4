"""Seeded gauge fields, spinor fields and sources (numpy, complex128).

Recipe for the interacting fields (stand-ins for the paper's CLS ensembles):
for every link (x, mu) draw eight iid N(0,1) numbers h_a, form the traceless
Hermitian ``H = sum_a h_a lambda_a / 2`` with the Gell-Mann matrices, take
``U = exp(i eps H)`` through an FP64 eigendecomposition, and project back to
SU(3): normalise row 0, Gram-Schmidt row 1 against it, and set
``row 2 = conj(row 0 x row 1)``.  The numbers come from numpy's PCG64 with the
given seed, drawn one timeslice at a time in site order.
"""
import numpy as np

GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1] = -1j
GELL_MANN[1][1, 0] = 1j
GELL_MANN[2][0, 0], GELL_MANN[2][1, 1] = 1, -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2] = -1j
GELL_MANN[4][2, 0] = 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2] = -1j
GELL_MANN[6][2, 1] = 1j
GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)


def volume(dims):
    T, L1, L2, L3 = dims
    return T * L1 * L2 * L3


def free_gauge(dims):
    """All links equal to the identity."""
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U.reshape(tuple(dims) + (4, 3, 3))


def project_su3(U):
    """Project a stack of 3x3 matrices onto SU(3) (rows 0, 1 Gram-Schmidt)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    r0 = U[..., 0, :]
    r0 /= np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 -= np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 /= np.linalg.norm(r1, axis=-1, keepdims=True)
    U[..., 0, :] = r0
    U[..., 1, :] = r1
    U[..., 2, :] = np.conj(np.cross(r0, r1))
    return U


def _exp_i_eps_h(h, eps):
    H = np.einsum("na,aij->nij", h, GELL_MANN * 0.5)
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(Q, 1, 2))


def gauge_su3(dims, eps, seed):
    """Synthetic SU(3) field ``U = P_SU3[exp(i eps H)]``, H Gaussian per link."""
    T, L1, L2, L3 = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    per_slice = L1 * L2 * L3 * 4
    out = np.empty((T, per_slice, 3, 3), dtype=np.complex128)
    for t in range(T):
        h = rng.standard_normal((per_slice, 8))
        out[t] = project_su3(_exp_i_eps_h(h, eps))
    return out.reshape(tuple(dims) + (4, 3, 3))


def random_su3(n, rng):
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, then projected)."""
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    return project_su3(Q)


def gauge_transform(dims, seed):
    """A random SU(3) matrix g(x) per site, shape dims + (3, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return random_su3(volume(dims), rng).reshape(tuple(dims) + (3, 3))


def random_spinor(dims, seed, nrhs=None):
    """Complex Gaussian spinor field(s), shape ([nrhs,] T, L1, L2, L3, 4, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(dims) + (4, 3)
    if nrhs is not None:
        shape = (nrhs,) + shape
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def point_source(dims, site, spin, colour):
    """Unit point source at ``site`` = (x0, x1, x2, x3) in one spin-colour component."""
    eta = np.zeros(tuple(dims) + (4, 3), dtype=np.complex128)
    eta[tuple(site) + (spin, colour)] = 1.0
    return eta


def point_sources_12(dims, site, ncols=12):
    """The first ``ncols`` spin-colour point sources (column c = 3*spin + colour)."""
    eta = np.zeros((ncols,) + tuple(dims) + (4, 3), dtype=np.complex128)
    for c in range(ncols):
        eta[(c,) + tuple(site) + (c // 3, c % 3)] = 1.0
    return eta


def sf_boundary_link(phi, L):
    """An abelian boundary link of the Schroedinger functional:
    diag(exp(i phi_a / L)), phi a triple summing to zero (SU(3))."""
    phi = np.asarray(phi, dtype=np.float64)
    return np.diag(np.exp(1j * phi / L))


def gauge_su3_sf(dims, eps, seed, phi=(0.0, 0.0, 0.0), phi_prime=(0.0, 0.0, 0.0), interior_free=False):
    """Links of a Schroedinger-functional lattice whose interior has
    dims = (T, L1, L2, L3): an array of T + 2 timeslices (index 0 the boundary
    x0 = 0, T + 1 the boundary x0 = T + 1).  All links are drawn as in
    gauge_su3 (or are unit links with interior_free), then the spatial links of
    the two boundary timeslices are set to the constant abelian fields of phi
    and phi_prime (direction k: diag(exp(i phi_a / L_k)))."""
    T, L1, L2, L3 = dims
    ext = (T + 2, L1, L2, L3)
    U = free_gauge(ext) if interior_free else gauge_su3(ext, eps, seed)
    for k, L in enumerate((L1, L2, L3), start=1):
        U[0, :, :, :, k] = sf_boundary_link(phi, L)
        U[T + 1, :, :, :, k] = sf_boundary_link(phi_prime, L)
    return U
