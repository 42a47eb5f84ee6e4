"""The operator kernels the solves run, at the 24^3 x 48 workload size with 12
right-hand sides (one launch, every slot active), column by column against
the oracle by the largest element error.

* FP32: the shared-tile kernels (links and clover staged in LDS, one slot per
  wave), with one mass for all slots (the odd-site kernel stages the common
  A_oo^-1 in LDS as well) and with a mass and a time profile per slot (each
  slot its own A_oo^-1, as in a served batch);
* FP16 storage with per-site scales (slab kernels) and FP64;
* the even-odd Schur operator and its adjoint (the solver's operator), and
  the full operator (the clover-diagonal kernel on both parities).

Reference: the oracle's D' (eq. linsysprec with the modified time
derivatives) on the full lattice; the Schur operator from it as
[D'(psi_e - A_oo^-1 [D' psi_e]_odd)]_even, with A_oo^-1 from a LAPACK inverse
of the oracle's 12x12 clover plus 4 + M at every odd site.
Bound: max |GPU - ref| <= tol max |ref| per column, tol = 1e-12 (FP64),
1e-6 (FP32), 2e-3 (FP16).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log, parity_mask

pytestmark = pytest.mark.gpu

NRHS = 12
TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3}
MASSES = (0.5, 0.05, 0.2)


class Workload:
    def __init__(self):
        cfg = synth.config("su3_24c48")
        self.dims = dims = cfg["dims"]
        self.T = dims[0]
        self.csw = cfg["csw"]
        log("building the 24^3x48 field, clover and A_oo^-1 (oracle, LAPACK)")
        self.U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
        self.C = oracle.clover(self.U, self.csw)
        par = parity_mask(dims)
        self.even = (par == 0)[..., None, None]
        self.odd_idx = np.nonzero(par.ravel() == 1)[0]
        Co = self.C.reshape(-1, 12, 12)[self.odd_idx]
        self.ainv = {M: np.linalg.inv(Co + (4.0 + M) * np.eye(12)) for M in MASSES}
        del Co
        self.psi = synth.random_spinor(dims, 2448, nrhs=NRHS)
        self.alpha = synth.alpha_table(cfg["profile"], self.T, 0.4)
        # per-slot profiles of a served batch: the symmetric exponential from
        # the slot's source timeslice
        self.alphas = np.stack([synth.alpha_exp_sym(self.T, (0.0, 0.1, 0.4)[k % 3], (7 * k) % self.T)
                                for k in range(NRHS)])
        self.slot_masses = np.array([MASSES[k % len(MASSES)] for k in range(NRHS)])
        self._cache = {}

    def schur_ref(self, k, M, alpha, dagger):
        key = ("schur", k, M, None if alpha is None else alpha.tobytes(), dagger)
        if key not in self._cache:
            pe = self.psi[k] * self.even
            h = oracle.apply(self.U, self.C, M, pe, alpha=alpha, dagger=dagger).reshape(-1, 12)[self.odd_idx]
            chi = np.zeros((int(np.prod(self.dims)), 12), dtype=np.complex128)
            chi[self.odd_idx] = -np.matmul(self.ainv[M], h[..., None])[..., 0]
            x = pe + chi.reshape(pe.shape)
            self._cache[key] = oracle.apply(self.U, self.C, M, x, alpha=alpha, dagger=dagger) * self.even
        return self._cache[key]

    def full_ref(self, k, M, alpha, dagger):
        key = ("full", k, M, alpha.tobytes(), dagger)
        if key not in self._cache:
            self._cache[key] = oracle.apply(self.U, self.C, M, self.psi[k], alpha=alpha, dagger=dagger)
        return self._cache[key]


_W = None


def workload():
    global _W
    if _W is None:
        _W = Workload()
    return _W


def run(W, precision, schur, dagger, per_slot):
    import torch
    with lattice(W.dims) as L:
        L.set_gauge(W.U)
        L.set_clover(W.csw)
        L.set_mass(0.5)
        L.set_alpha(W.alpha)
        x = torch.from_numpy(W.psi.reshape(NRHS, -1)).cuda()
        y = torch.empty_like(x)
        if per_slot:
            L.apply_dev(x, y, precond=True, dagger=dagger, schur=schur, precision=precision,
                        masses=W.slot_masses, alphas=W.alphas)
        else:
            L.apply_dev(x, y, precond=True, dagger=dagger, schur=schur, precision=precision)
        torch.cuda.synchronize()
        out = y.cpu().numpy().reshape(W.psi.shape)
        del x, y
    return out


def check(W, got, precision, schur, dagger, per_slot):
    worst = 0.0
    for k in range(NRHS):
        M = W.slot_masses[k] if per_slot else 0.5
        a = W.alphas[k] if per_slot else W.alpha
        ref = W.schur_ref(k, M, a, dagger) if schur else W.full_ref(k, M, a, dagger)
        e = float(np.abs(got[k] - ref).max() / np.abs(ref).max())
        worst = max(worst, e)
        assert e <= TOL[precision], (k, e)
    log(f"  {precision} schur={schur} dagger={dagger} per_slot={per_slot}: worst column max-element err {worst:.2e}")


@pytest.mark.parametrize("precision", ["f32", "f16", "f64"])
@pytest.mark.parametrize("dagger", [False, True])
def test_24c48_schur_12rhs_one_mass(precision, dagger):
    log(f"test_24c48_schur_12rhs_one_mass {precision} dagger={dagger}")
    W = workload()
    check(W, run(W, precision, True, dagger, False), precision, True, dagger, False)


@pytest.mark.parametrize("precision", ["f32", "f16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_24c48_schur_12rhs_mass_and_profile_per_slot(precision, dagger):
    log(f"test_24c48_schur_12rhs_mass_and_profile_per_slot {precision} dagger={dagger}")
    W = workload()
    check(W, run(W, precision, True, dagger, True), precision, True, dagger, True)


@pytest.mark.parametrize("precision", ["f32", "f16", "f64"])
def test_24c48_full_operator_12rhs(precision):
    log(f"test_24c48_full_operator_12rhs {precision}")
    W = workload()
    check(W, run(W, precision, False, False, False), precision, False, False, False)
