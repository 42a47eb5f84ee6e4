"""Closed forms used to pin the oracle (and, for the free field, the GPU path).

Free Wilson propagator in momentum space.  With all links equal to one the
operator D + M of the oracle is diagonal in momentum space: for psi(x) =
exp(i p.x) the derivatives give nabla_mu -> exp(i p_mu) - 1 and
nabla*_mu -> 1 - exp(-i p_mu), hence

    D + M -> m(p) + i sum_mu gamma_mu sin p_mu,   m(p) = M + sum_mu (1 - cos p_mu)

and the propagator of a unit point source at the origin is

    S(x) = V^-1 sum_p exp(i p.x) [m(p) - i sum_mu gamma_mu sin p_mu]
                                  / [m(p)^2 + sum_mu sin^2 p_mu]  (x) 1_colour

with p_k = 2 pi n_k / L_k in space and p_0 = pi (2 n_0 + 1) / T for
antiperiodic time (2 pi n_0 / T for periodic).  The sum over p is a library
inverse FFT.  The gamma matrices here are written out independently of the
oracle (chiral basis, gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]]).
"""
import numpy as np

_s = [np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
      np.array([[1, 0], [0, -1]], dtype=complex)]
_Z = np.zeros((2, 2))
_I = np.eye(2)
GAMMA = [np.block([[_Z, -_I], [-_I, _Z]]).astype(complex)] + \
        [np.block([[_Z, -1j * s], [1j * s, _Z]]) for s in _s]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def momenta(dims, bc_t=-1):
    T = dims[0]
    n0 = np.arange(T)
    p0 = np.pi * (2 * n0 + 1) / T if bc_t == -1 else 2 * np.pi * n0 / T
    ps = [p0] + [2 * np.pi * np.arange(L) / L for L in dims[1:]]
    return np.meshgrid(*ps, indexing="ij")


def free_propagator_spin(dims, M, bc_t=-1):
    """Spin part of the free propagator from the origin: array [T,L1,L2,L3,4,4]
    (row = sink spin, column = source spin).  Colour is a unit matrix."""
    P = momenta(dims, bc_t)
    m = M + sum(1 - np.cos(p) for p in P)
    den = m ** 2 + sum(np.sin(p) ** 2 for p in P)
    Sp = m[..., None, None] * np.eye(4)
    for mu in range(4):
        Sp = Sp - 1j * np.sin(P[mu])[..., None, None] * GAMMA[mu]
    Sp = Sp / den[..., None, None]
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3))
    if bc_t == -1:
        T = dims[0]
        Sx = Sx * np.exp(1j * np.pi * np.arange(T) / T)[:, None, None, None, None, None]
    return Sx


def free_propagator_columns(dims, M, bc_t=-1, ncols=12):
    """Columns c = 3*spin_src + colour_src as spinor fields [ncols, T,L1,L2,L3,4,3]."""
    Ss = free_propagator_spin(dims, M, bc_t)
    out = np.zeros((ncols,) + tuple(dims) + (4, 3), dtype=np.complex128)
    for c in range(ncols):
        s, a = divmod(c, 3)
        out[c, ..., :, a] = Ss[..., :, s]
    return out


def free_cpp(dims, M, bc_t=-1):
    """C_PP(t) = -sum_x tr[S^+ S] for all 12 columns (colour trace gives 3)."""
    Ss = free_propagator_spin(dims, M, bc_t)
    return -3.0 * np.sum(np.abs(Ss) ** 2, axis=(1, 2, 3, 4, 5))


def free_energy_zero_momentum(M):
    """Pole of the zero-spatial-momentum free propagator: exp(E) = 1 + M."""
    return np.log1p(M)
