"""Pin the link directions and the clover leaves of the oracle.

* gauge covariance: U_mu(x) -> g(x) U_mu(x) g(x+mu)^+ maps D+M to G (D+M) G^+
  and leaves C_PP invariant; a link used at the wrong site or undaggered fails;
* a constant abelian field (colour-diagonal, flux quantised on the torus)
  has every plaquette equal to exp(i phi), so Fhat_mu_nu = i sin(phi) exactly
  and the clover term is c_sw (i/4) sum sigma_mu_nu Fhat_mu_nu in closed form;
  a leaf with the wrong orientation or a wrong link in it fails.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import GAMMA, GAMMA5


def transform(U, g):
    dims = U.shape[:4]
    Up = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=mu)  # g(x + mu)
        Up[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(g_fwd, -1, -2))
    return Up


@pytest.mark.parametrize("bc_t", [-1, 1])
def test_operator_gauge_covariance(bc_t):
    dims = (4, 4, 2, 4)
    U = synth.gauge_su3(dims, 0.8, seed=21)
    g = synth.gauge_transform(dims, seed=22)
    Ug = transform(U, g)
    C, Cg = oracle.clover(U, 1.6), oracle.clover(Ug, 1.6)
    # clover: C'(x) = g(x) C(x) g(x)^+ on each spin block
    G12 = np.einsum("st,...ab->...satb", np.eye(4), g).reshape(tuple(dims) + (12, 12))
    np.testing.assert_allclose(Cg, G12 @ C @ np.conj(np.swapaxes(G12, -1, -2)), atol=1e-13)
    psi = synth.random_spinor(dims, 23)
    alpha = synth.alpha_exp(dims[0], 0.4)
    lhs = oracle.apply(Ug, Cg, 0.2, np.einsum("...ab,...sb->...sa", g, psi), alpha=alpha, bc_t=bc_t)
    rhs = np.einsum("...ab,...sb->...sa", g, oracle.apply(U, C, 0.2, psi, alpha=alpha, bc_t=bc_t))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_cpp_gauge_invariance():
    dims = (8, 4, 4, 4)
    U = synth.gauge_su3(dims, 0.5, seed=31)
    g = synth.gauge_transform(dims, seed=32)
    Ug = transform(U, g)
    C, Cg = oracle.clover(U, 1.6), oracle.clover(Ug, 1.6)
    alpha = synth.alpha_exp(dims[0], 0.3)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=12)
    # the transformed source is g(0) applied to the colour index at the origin
    g0 = g[0, 0, 0, 0]
    S = np.stack([oracle.solve(U, C, 0.5, eta[c], alpha=alpha, r=1e-13)[0] for c in range(12)])
    etag = np.einsum("ab,csb->csa", g0, eta[:, 0, 0, 0, 0])
    Sg = []
    for c in range(12):
        e = np.zeros_like(eta[c])
        e[0, 0, 0, 0] = etag[c]
        Sg.append(oracle.solve(Ug, Cg, 0.5, e, alpha=alpha, r=1e-13)[0])
    np.testing.assert_allclose(oracle.cpp(np.stack(Sg)), oracle.cpp(S), rtol=1e-11)


def abelian_field(dims, quanta):
    """Colour-diagonal links with uniform plaquette angle phi^c_mu_nu =
    2 pi n^c_mu_nu / (L_mu L_nu) in every (mu<nu) plane; quanta[(mu,nu)] =
    (n^0, n^1, n^2) with sum zero so that det U = 1."""
    x = np.indices(dims)
    U = np.zeros(tuple(dims) + (4, 3, 3), dtype=np.complex128)
    for rho in range(4):
        for c in range(3):
            ph = np.zeros(dims)
            for (mu, nu), n in quanta.items():
                phi = 2 * np.pi * n[c] / (dims[mu] * dims[nu])
                if rho == mu:      # gradient along x_nu in U_mu
                    ph -= phi * x[nu]
                elif rho == nu:    # twist in U_nu on the last x_nu slice, growing with x_mu
                    ph += phi * dims[nu] * x[mu] * (x[nu] == dims[nu] - 1)
            U[..., rho, c, c] = np.exp(1j * ph)
    return U


def test_clover_constant_abelian_field():
    dims = (4, 6, 4, 2)
    quanta = {(0, 1): (1, 2, -3), (0, 2): (2, -1, -1), (0, 3): (0, 1, -1),
              (1, 2): (-1, 0, 1), (1, 3): (3, -2, -1), (2, 3): (1, 1, -2)}
    U = abelian_field(dims, quanta)
    csw = 1.7
    C = oracle.clover(U, csw).reshape(-1, 12, 12)
    expect = np.zeros((12, 12), dtype=np.complex128)
    for (mu, nu), n in quanta.items():
        phi = 2 * np.pi * np.array(n) / (dims[mu] * dims[nu])
        F = np.diag(1j * np.sin(phi))
        sig = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
        # the (mu,nu) and (nu,mu) terms are equal: sigma and F both flip sign
        expect += 2 * csw * 0.25j * np.kron(sig, F)
    np.testing.assert_allclose(C, np.broadcast_to(expect, C.shape), atol=1e-13)


def test_gamma_matrices_clifford():
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        np.testing.assert_allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            np.testing.assert_allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4), atol=1e-15)
    np.testing.assert_allclose(g[0] @ g[1] @ g[2] @ g[3], np.diag([1, 1, -1, -1]), atol=1e-15)
    np.testing.assert_allclose(GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)
