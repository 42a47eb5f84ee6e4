"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

Thin ctypes wrapper around ``oracle/liborc.so`` (built from ``orc.c`` by
``oracle.build.build()``).  All arrays are numpy complex128 in the host
layouts ``U[T,L1,L2,L3,4,3,3]``, ``psi[T,L1,L2,L3,4,3]`` and
``C[T,L1,L2,L3,12,12]``.  ``alpha`` is a table of T positive numbers in the
convention ``S' = alpha S`` (the reciprocal of the function the paper
factorises in eq. redeft).  ``beta`` (light-quark section, eqs. redefa and
betaa) is a tuple of four per-direction profiles ``(alpha_0[T], alpha_1[L1],
alpha_2[L2], alpha_3[L3])`` with ``beta(y) = prod_mu alpha_mu(y_mu)``; a
``None`` entry is a profile of ones.

The pins that make this oracle trustworthy live in ``tests/test_oracle_*.py``
(closed-form free propagator, dense LU, similarity, gamma5-hermiticity, gauge
covariance, an analytic clover field).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ENOCONV, ORC_EBREAK = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    pass


def _lib():
    global _LIB
    if _LIB is None:
        # ORC_LIB names another build of orc.c (the sanitizer test uses it)
        path = os.environ.get("ORC_LIB") or os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_clover.argtypes = [ip, dp, ctypes.c_double, dp]
        lib.orc_apply.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp, dp]
        lib.orc_apply_modified.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp,
                                           ctypes.c_double, ctypes.c_double, dp, dp]
        lib.orc_solve.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp,
                                  ctypes.c_double, ctypes.c_int, dp, dp, dp]
        lib.orc_apply_beta.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp, dp]
        lib.orc_apply_modified4.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp, dp, dp]
        lib.orc_solve_beta.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp,
                                       ctypes.c_double, ctypes.c_int, dp, dp, dp]
        lib.orc_solve_sap.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ip, dp, ctypes.c_double,
                                      ctypes.c_int, dp, dp, dp]
        lib.orc_sap_apply.argtypes = [ip, ctypes.c_int, dp, dp, ctypes.c_double, dp, ip, dp, dp]
        lib.orc_cpp.argtypes = [ip, ctypes.c_int, dp, ctypes.c_int, dp]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_get_threads.restype = ctypes.c_int
        lib.orc_gamma.argtypes = [ctypes.c_int, dp]
        _LIB = lib
    return _LIB


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(f"{what} failed with code {rc}")


def set_threads(n):
    _lib().orc_set_threads(int(n))


def get_threads():
    return int(_lib().orc_get_threads())


def gamma(mu):
    out = np.zeros((4, 4), dtype=np.complex128)
    _lib().orc_gamma(int(mu), _ptr(out))
    return out


def clover(U, csw):
    """Dense 12x12 clover term c_sw (i/4) sum sigma F per site."""
    U = _c128(U)
    dims = U.shape[:4]
    C = np.zeros(tuple(dims) + (12, 12), dtype=np.complex128)
    _check(_lib().orc_clover(_dims(dims), _ptr(U), float(csw), _ptr(C)), "orc_clover")
    return C


def apply(U, C, M, psi, alpha=None, bc_t=-1, dagger=False):
    """alpha (D+M) alpha^-1 psi (or its adjoint); alpha None means no preconditioning."""
    U = _c128(U)
    psi = _c128(psi)
    dims = U.shape[:4]
    out = np.zeros_like(psi)
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    Cc = None if C is None else _c128(C)
    _check(_lib().orc_apply(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(a),
                            int(bool(dagger)), _ptr(psi), _ptr(out)), "orc_apply")
    return out


def apply_modified(U, C, M, psi, alpha, alpha_T=1.0, alpha_m1=1.0, bc_t=-1):
    """D'+M through the paper's modified time derivatives and boundary rule."""
    U = _c128(U)
    psi = _c128(psi)
    dims = U.shape[:4]
    out = np.zeros_like(psi)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    Cc = None if C is None else _c128(C)
    _check(_lib().orc_apply_modified(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(a),
                                     float(alpha_T), float(alpha_m1), _ptr(psi), _ptr(out)),
           "orc_apply_modified")
    return out


def _profiles(dims, beta):
    """The four profiles of beta concatenated (T + L1 + L2 + L3 values)."""
    assert len(beta) == 4
    parts = [np.ones(dims[mu]) if b is None else np.asarray(b, dtype=np.float64) for mu, b in enumerate(beta)]
    for mu, b in enumerate(parts):
        assert b.shape == (dims[mu],)
    return np.ascontiguousarray(np.concatenate(parts))


def beta_field(dims, beta):
    """beta(y) = prod_mu alpha_mu(y_mu) on the lattice, shape dims."""
    out = np.ones(tuple(dims))
    for mu, b in enumerate(beta):
        if b is not None:
            shape = [1, 1, 1, 1]
            shape[mu] = dims[mu]
            out = out * np.asarray(b, dtype=np.float64).reshape(shape)
    return out


def apply_beta(U, C, M, psi, beta, bc_t=-1, dagger=False):
    """beta (D+M) beta^-1 psi (or its adjoint), beta(y) = prod_mu alpha_mu(y_mu)."""
    U = _c128(U)
    psi = _c128(psi)
    dims = U.shape[:4]
    out = np.zeros_like(psi)
    prof = _profiles(dims, beta)
    Cc = None if C is None else _c128(C)
    _check(_lib().orc_apply_beta(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(prof),
                                 int(bool(dagger)), _ptr(psi), _ptr(out)), "orc_apply_beta")
    return out


def apply_modified4(U, C, M, psi, beta, ext, bc_t=-1):
    """D'+M through the modified covariant derivatives in every direction, the
    boundary rule continued with ext = [alpha_mu(L_mu), alpha_mu(-1)] per mu."""
    U = _c128(U)
    psi = _c128(psi)
    dims = U.shape[:4]
    out = np.zeros_like(psi)
    prof = _profiles(dims, beta)
    e = np.ascontiguousarray(ext, dtype=np.float64)
    assert e.shape == (8,)
    Cc = None if C is None else _c128(C)
    _check(_lib().orc_apply_modified4(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(prof),
                                      _ptr(e), _ptr(psi), _ptr(out)), "orc_apply_modified4")
    return out


def solve(U, C, M, eta, alpha=None, r=1e-13, solver="bicgstab", maxit=100000, bc_t=-1,
          return_prec=False, allow_unconverged=False, beta=None):
    """Solve (D+M) S = eta via the alpha- (or beta-) preconditioned system.

    Returns ``(S, info)`` (or ``(S, S', info)``) with info = dict(iters,
    relres_prec, relres).
    """
    U = _c128(U)
    eta = _c128(eta)
    dims = U.shape[:4]
    S = np.zeros_like(eta)
    Sp = np.zeros_like(eta) if return_prec else None
    info = np.zeros(3)
    Cc = None if C is None else _c128(C)
    sid = {"bicgstab": 0, "cgnr": 1}[solver]
    if beta is not None:
        assert alpha is None
        prof = _profiles(dims, beta)
        rc = _lib().orc_solve_beta(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(prof), sid,
                                   _ptr(eta), float(r), int(maxit), _ptr(S), _ptr(Sp), _ptr(info))
    else:
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
        rc = _lib().orc_solve(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(a), sid,
                              _ptr(eta), float(r), int(maxit), _ptr(S), _ptr(Sp), _ptr(info))
    if rc != ORC_OK and not (allow_unconverged and rc == ORC_ENOCONV):
        raise OracleError(f"orc_solve failed with code {rc} after {int(info[0])} iterations")
    d = dict(iters=int(info[0]), relres_prec=float(info[1]), relres=float(info[2]), code=rc)
    return (S, Sp, d) if return_prec else (S, d)


def _sap_par(block, ncy, nmr, nkv):
    return (ctypes.c_int * 7)(*[int(b) for b in block], int(ncy), int(nmr), int(nkv))


def solve_sap(U, C, M, eta, block, beta=None, ncy=5, nmr=4, nkv=16, r=1e-13, maxit=10000, bc_t=-1,
              return_prec=False, allow_unconverged=False):
    """Solve (D+M) S = eta with SAP+GCR (Schwarz blocks of extents `block`)
    on the beta-preconditioned system.  Returns (S, info) or (S, S', info)."""
    U = _c128(U)
    eta = _c128(eta)
    dims = U.shape[:4]
    S = np.zeros_like(eta)
    Sp = np.zeros_like(eta) if return_prec else None
    info = np.zeros(3)
    prof = None if beta is None else _profiles(dims, beta)
    Cc = None if C is None else _c128(C)
    rc = _lib().orc_solve_sap(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(prof),
                              _sap_par(block, ncy, nmr, nkv), _ptr(eta), float(r), int(maxit), _ptr(S), _ptr(Sp),
                              _ptr(info))
    if rc != ORC_OK and not (allow_unconverged and rc == ORC_ENOCONV):
        raise OracleError(f"orc_solve_sap failed with code {rc} after {int(info[0])} iterations")
    d = dict(iters=int(info[0]), relres_prec=float(info[1]), code=rc)
    return (S, Sp, d) if return_prec else (S, d)


def sap_apply(U, C, M, r, block, beta=None, ncy=5, nmr=4, bc_t=-1):
    """One application of the SAP preconditioner to r."""
    U = _c128(U)
    r = _c128(r)
    dims = U.shape[:4]
    out = np.zeros_like(r)
    prof = None if beta is None else _profiles(dims, beta)
    Cc = None if C is None else _c128(C)
    _check(_lib().orc_sap_apply(_dims(dims), int(bc_t), _ptr(U), _ptr(Cc), float(M), _ptr(prof),
                                _sap_par(block, ncy, nmr, 1), _ptr(r), _ptr(out)), "orc_sap_apply")
    return out


def cpp(S, x0_src=0):
    """C_PP(t) = -sum_x sum_cols |S|^2 per timeslice, t = (x0 - x0_src) mod T.
    S: ([ncols,] T, L1, L2, L3, 4, 3)."""
    S = _c128(S)
    if S.ndim == 6:
        S = S[None]
    dims = S.shape[1:5]
    out = np.zeros(dims[0])
    _check(_lib().orc_cpp(_dims(dims), S.shape[0], _ptr(S), int(x0_src), _ptr(out)), "orc_cpp")
    return out


def sf_clover(U_ext, csw, ct_tilde=1.0):
    """Clover term of the interior of a Schroedinger-functional lattice (the
    closing remark of the heavy-quark section names the formulation).  U_ext
    holds T + 2 timeslices: the boundary x0 = 0, the interior, the boundary
    x0 = T + 1.  The clover leaves of an interior site stay within the padded
    lattice (they reach at most one timeslice beyond the interior), so the
    clover of the padded lattice, restricted to the interior, is the
    interior's clover with the boundary links in its leaves; (ct_tilde - 1)
    is added on the first and last interior timeslices (the fermion boundary
    counterterm).  Returns C[T, L1, L2, L3, 12, 12]."""
    C = clover(U_ext, csw)[1:-1].copy()
    eye = np.eye(12, dtype=np.complex128)
    C[0] += (ct_tilde - 1.0) * eye
    C[-1] += (ct_tilde - 1.0) * eye
    return C


def sf_apply(U_ext, csw, M, psi, alpha=None, ct_tilde=1.0, dagger=False):
    """The Schroedinger-functional operator on the interior field psi: the
    Dirichlet-boundary operator with the interior links, the clover term of
    sf_clover and the boundary counterterm (alpha as in apply)."""
    U = np.ascontiguousarray(np.asarray(U_ext)[1:-1])
    return apply(U, sf_clover(U_ext, csw, ct_tilde), M, psi, alpha=alpha, bc_t=0, dagger=dagger)
