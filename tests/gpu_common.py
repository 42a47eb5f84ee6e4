"""Shared helpers of the GPU parity tests (oracle side and the binding)."""
import sys

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lattice(dims, bc_t=-1):
    import paper_1006_4028_amd as dp
    return dp.Lattice(dims, bc_t=bc_t)


def rel_err(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def parity_mask(dims):
    x = np.indices(dims)
    return (x.sum(axis=0) % 2)  # 0 even, 1 odd


def oracle_hop(oracle, U, C, M, psi, alpha, bc_t=-1, dagger=False):
    """The hopping part of D' (or of D'^+) from the oracle: D'psi - (4 + M + C) psi
    (the clover term is Hermitian, so it is the same diagonal for the adjoint).
    alpha: a time profile, or a tuple of four per-direction profiles (beta)."""
    if isinstance(alpha, tuple):
        full = oracle.apply_beta(U, C, M, psi, alpha, bc_t=bc_t, dagger=dagger)
    else:
        full = oracle.apply(U, C, M, psi, alpha=alpha, bc_t=bc_t, dagger=dagger)
    diag = (4.0 + M) * psi
    if C is not None:
        diag = diag + np.einsum("...ij,...j->...i", C, psi.reshape(psi.shape[:4] + (12,))).reshape(psi.shape)
    return full - diag


def oracle_schur(oracle, U, C, M, psi, alpha, bc_t=-1, dagger=False):
    """A_ee psi_e - H_eo A_oo^-1 H_oe psi_e on the even sites (odd part zero),
    from the oracle's operator and a per-site LAPACK solve for A_oo^-1."""
    dims = U.shape[:4]
    par = parity_mask(dims)[..., None, None]
    pe = psi * (par == 0)
    h = oracle_hop(oracle, U, C, M, pe, alpha, bc_t, dagger) * (par == 1)
    A = (4.0 + M) * np.eye(12) + (C if C is not None else 0.0)
    A = np.broadcast_to(A, tuple(dims) + (12, 12))
    t = np.linalg.solve(A, h.reshape(tuple(dims) + (12, 1)))[..., 0].reshape(psi.shape) * (par == 1)
    u = oracle_hop(oracle, U, C, M, t, alpha, bc_t, dagger) * (par == 0)
    Ae = np.einsum("...ij,...j->...i", A, pe.reshape(tuple(dims) + (12,))).reshape(psi.shape)
    return (Ae - u) * (par == 0)
