"""Distance profiles alpha(x0) as plain tables (one positive number per timeslice).

Convention of these tables: the preconditioned propagator is ``S' = alpha * S``
and the physical one is restored as ``S = S' / alpha``.  The paper writes its
field redefinition with the reciprocal function (``S = alpha_p S'``, eq.
redeft); its own prose on restoration (introduction) uses this table's
convention.  So ``alpha = 1 / alpha_p``.

``t = (x0 - x0_src) mod T`` is the distance from the source timeslice.
"""
import numpy as np


def _dist(T, x0_src):
    return (np.arange(T) - x0_src) % T


def alpha_exp(T, alpha0, x0_src=0):
    """alpha(x0) = exp(alpha0 * t): the exponential profile (paper, end of the
    heavy-quark section, used there for Schroedinger-functional runs)."""
    return np.exp(alpha0 * _dist(T, x0_src).astype(np.float64))


def alpha_exp_sym(T, alpha0, x0_src=0):
    """alpha(x0) = exp(alpha0 * min(t, T - t)): periodic exponential profile."""
    t = _dist(T, x0_src).astype(np.float64)
    return np.exp(alpha0 * np.minimum(t, T - t))


def alpha_cosh_paper(T, alpha0, x0_src=0):
    """The paper's periodic-time profile alpha_p = cosh[alpha0 (y0 - L0/2)]
    (eq. pbcalpha), returned in this module's convention: 1 / alpha_p."""
    t = _dist(T, x0_src).astype(np.float64)
    return 1.0 / np.cosh(alpha0 * (t - T / 2.0))


def beta_cosh_paper(dims, alpha0):
    """The light-quark factorisation beta(y) = prod_mu 1/cosh[alpha0 (y_mu - L_mu/2)]
    (eq. betaa), returned in this module's convention (S' = beta S) as its four
    per-direction profiles: cosh[alpha0 (y_mu - L_mu/2)] for mu = 0..3."""
    return tuple(np.cosh(alpha0 * (np.arange(L, dtype=np.float64) - L / 2.0)) for L in dims)


def alpha_table(kind, T, alpha0, x0_src=0):
    kinds = {"exp": alpha_exp, "exp_sym": alpha_exp_sym, "cosh": alpha_cosh_paper}
    if kind not in kinds:
        raise ValueError(f"unknown alpha profile {kind!r}")
    return kinds[kind](T, alpha0, x0_src)
