"""The paper's demonstration on the free field (Figs. 1 and 2, heavy-quark
section): with a loose global residue r = 1e-6, the unpreconditioned
correlator of a heavy quark (M = 0.5) is wrong at far timeslices, where
|C_PP| approaches r^2, while the distance-preconditioned solve at the
same residue, restored by eq. backcorrection, agrees with the exact one at
every timeslice.  The exact correlator is the momentum-space closed form.
No printed values exist for these figures (the lattice size is not stated);
this is the qualitative claim on an 8^3 x 48 lattice."""
import numpy as np
import pytest

import synth
from closed_form import free_cpp
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_loose_residue_far_timeslices(precision):
    dims, M, r = (48, 8, 8, 8), 0.5, 1e-6
    log(f"test_loose_residue_far_timeslices {precision}")
    exact = free_cpp(dims, M)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    with lattice(dims) as L:
        L.set_mass(M)
        L.set_alpha(np.ones(dims[0]))
        _, c_plain, _ = L.solve(eta, r=r, precision=precision, ncols_group=12, want_S=False)
        L.set_alpha(synth.alpha_cosh_paper(dims[0], 0.4))
        _, c_prec, _ = L.solve(eta, r=r, precision=precision, ncols_group=12, want_S=False)
    e_plain = np.abs(c_plain[0] / exact - 1)
    e_prec = np.abs(c_prec[0] / exact - 1)
    t = np.arange(dims[0])
    far = np.abs(exact) < 100 * r ** 2  # where |S| ~ sqrt|C| approaches the residue
    log("  t    |C_exact|    err(alpha0=0)  err(alpha0=0.4)")
    for k in range(0, dims[0], 4):
        log(f"  {k:2d}  {abs(exact[k]):.3e}  {e_plain[k]:.3e}      {e_prec[k]:.3e}")
    assert far.any()
    # unpreconditioned: fine near the source, wrong by percents where |C| nears r^2
    assert e_plain[t < 6].max() < 1e-3
    assert e_plain[far].max() > 1e-2
    # preconditioned at the same residue: right everywhere, by orders of magnitude more
    assert e_prec.max() < 1e-4
    assert e_prec[far].max() < 1e-3 * e_plain[far].max()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_schroedinger_functional_boundary_loose_residue(precision):
    """The closing remark of the heavy-quark section: with Schroedinger-
    functional (Dirichlet) time boundaries the correlator decays over the
    whole time extent, so far timeslices need tiny residues; the paper used
    the exponential profile there.  Free field, 4^3 x 32, M = 0.5, source on
    the first timeslice, r = 1e-6: without the profile the far timeslices are
    wrong by percents, with alpha = exp(0.4 t) (the paper's exp(-alpha0 x0) in
    this convention) every timeslice agrees with the oracle's solve at 1e-13."""
    import oracle
    dims, M, r = (32, 4, 4, 4), 0.5, 1e-6
    log(f"test_schroedinger_functional_boundary_loose_residue {precision}")
    U = synth.free_gauge(dims)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    exact = oracle.cpp(np.stack([oracle.solve(U, None, M, eta[c], r=1e-13, bc_t=0)[0] for c in range(12)]))
    with lattice(dims, bc_t=0) as L:
        L.set_mass(M)
        L.set_alpha(np.ones(dims[0]))
        _, c_plain, _ = L.solve(eta, r=r, precision=precision, ncols_group=12, want_S=False)
        L.set_alpha(synth.alpha_exp(dims[0], 0.4))
        _, c_prec, _ = L.solve(eta, r=r, precision=precision, ncols_group=12, want_S=False)
    e_plain = np.abs(c_plain[0] / exact - 1)
    e_prec = np.abs(c_prec[0] / exact - 1)
    for k in range(0, dims[0], 4):
        log(f"  {k:2d}  {abs(exact[k]):.3e}  {e_plain[k]:.3e}  {e_prec[k]:.3e}")
    assert np.all(np.diff(-exact) < 0)  # decays over the whole extent
    assert e_plain[-4:].max() > 1e-2
    assert e_prec.max() < 1e-4
