"""Pins for the oracle's matrix exponential, lattice paths and observables
(plaquette, Wilson action, topological charge, unitarity norm) against
library routines, the theta-term density written out literally, closed-form
configurations and gauge invariance."""
import math

import numpy as np
import pytest
import scipy.linalg

from tests import latutil as lu


def test_expm_matches_scipy(orc):
    rng = np.random.default_rng(1)
    for scale in (1e-3, 0.1, 0.7, 2.0, 4.0):
        for _ in range(10):
            A = scale * (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
            ref = scipy.linalg.expm(A)
            got = orc.expm(A)
            assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_expm_group_properties(orc):
    rng = np.random.default_rng(2)
    for _ in range(20):
        H = lu.lie(rng.normal(size=8))  # Hermitian traceless
        U = orc.expm(1j * H)
        np.testing.assert_allclose(U @ U.conj().T, np.eye(3), atol=1e-14)
        X = lu.lie(rng.normal(size=8) + 1j * rng.normal(size=8))  # traceless
        assert abs(np.linalg.det(orc.expm(1j * X)) - 1) < 1e-13


def test_gell_mann_basis():
    """Tr(lambda_a lambda_b) = 2 delta_ab and sum_a Tr(lambda_a M) lambda_a = 2 TL(M):
    the normalisation that gives the factor 16 of the one-link cooling rate."""
    G = np.einsum("aij,bji->ab", lu.LAMBDA, lu.LAMBDA)
    np.testing.assert_allclose(G, 2 * np.eye(8), atol=1e-15)
    rng = np.random.default_rng(3)
    M = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    S = sum(np.trace(lu.LAMBDA[a] @ M) * lu.LAMBDA[a] for a in range(8))
    np.testing.assert_allclose(S, 2 * (M - np.trace(M) / 3 * np.eye(3)), atol=1e-14)


def test_path_conventions(orc):
    """Forward hops multiply U_mu(x); backward hops multiply U_mu(x-mu)^{-1}."""
    rng = np.random.default_rng(4)
    dims = (2, 4, 2, 4)
    U = lu.random_links(rng, dims)
    for x in [(0, 0, 0, 0), (1, 3, 1, 2)]:
        s = lu.site(dims, x)
        for dirs in ([1, 2, -1, -2], [-3, 4, 3, -4], [2, 2, 1, -2, -2, -1], [-1]):
            np.testing.assert_allclose(orc.path(dims, U, s, dirs), lu.walk(U, dims, x, dirs),
                                       atol=1e-13)


def test_cold_start(orc):
    dims = (4, 4, 4, 4)
    U = orc.cold_links(dims)
    assert orc.plaquette(dims, U) == 1.0
    assert orc.topological_charge(dims, U) == 0.0
    assert orc.distance(dims, U) == 0.0
    assert orc.wilson_action(dims, U, 6.0) == 0.0


def test_initial_configuration(orc):
    """U = exp(i lambda_a (x_a + i y_a)) from Philox stream tag 1."""
    dims = (4, 4, 4, 4)
    seed = 1
    U = orc.init_links(dims, seed, 0.3, 0.05)
    dmax, tmin = orc.link_stats(dims, U)
    assert dmax < 1e-13 and tmin >= 1.0
    assert orc.distance(dims, U) > 0
    # rebuild two links from the raw draws
    for s, mu in [(0, 0), (37, 2), (255, 3)]:
        x = np.zeros(8)
        y = np.zeros(8)
        for j in range(8):
            n = orc.normal_pair(seed, 4 * s + mu, 0, j, 1)
            tgt, sig = (x, 0.3) if j < 4 else (y, 0.05)
            tgt[2 * (j & 3):2 * (j & 3) + 2] = sig * n
        ref = scipy.linalg.expm(1j * lu.lie(x + 1j * y))
        np.testing.assert_allclose(lu.to_c(U[s, mu]), ref, atol=1e-13)
    # sample moments of the generator coefficients: log(U) recovers x + i y
    xs = []
    for s in range(0, 256, 3):
        Z = scipy.linalg.logm(lu.to_c(U[s, 0])) / 1j
        xs.append([np.real(np.trace(lu.LAMBDA[a] @ Z)) / 2 for a in range(8)])
    assert 0.2 < np.std(xs) < 0.4


def test_unitarity_norm_and_distance(orc):
    rng = np.random.default_rng(5)
    dims = (2, 2, 4, 2)
    U = lu.random_links(rng, dims)
    Uc = lu.to_c(U)
    ref = np.sum(np.abs(Uc) ** 2)
    assert abs(orc.unitarity_norm(dims, U) - ref) < 1e-12 * ref
    assert orc.distance(dims, U) > 0
    # (1/3) Tr U U^dagger >= 1 on SL(3,C), equality on SU(3)
    _, tmin = orc.link_stats(dims, U)
    assert tmin >= 1.0
    S = lu.from_c(lu.random_su3(rng, n=lu.volume(dims) * 4)).reshape(U.shape)
    assert abs(orc.distance(dims, S)) < 1e-14


def test_plaquette_and_action_brute_force(orc):
    rng = np.random.default_rng(6)
    dims = (2, 4, 2, 2)
    U = lu.random_links(rng, dims)
    V = lu.volume(dims)
    tp = 0j
    sw = 0j
    for s in range(V):
        x = lu.coords(dims, s)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                P = lu.walk(U, dims, x, [mu + 1, nu + 1, -(mu + 1), -(nu + 1)])
                tp += np.trace(P)
                sw += 1 - (np.trace(P) + np.trace(np.linalg.inv(P))) / 6
    p = orc.plaquette(dims, U)
    assert abs(p - tp / (18 * V)) < 1e-13
    beta = 5.7
    assert abs(orc.wilson_action(dims, U, beta) - beta * sw) < 1e-11 * abs(beta * sw)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 2, 2, 3)])
def test_topological_charge_literal_definition(orc, dims):
    """The clover form of the oracle equals the signed-index sum over
    eps~_{mu nu rho sigma} Tr[U_{mu nu} U_{rho sigma}] written out term by term."""
    rng = np.random.default_rng(8)
    U = lu.random_links(rng, dims, 0.5, 0.3)
    V = lu.volume(dims)
    lit = sum(lu.q_density_literal(U, dims, lu.coords(dims, s)) for s in range(V))
    q = orc.topological_charge(dims, U)
    assert abs(q - lit) < 1e-12 * max(1.0, abs(lit))
    assert abs(lit) > 1e-4  # non-trivial


@pytest.mark.parametrize("dims,n12,n34", [((4, 4, 4, 4), 1, 1), ((4, 4, 4, 4), 2, -1),
                                          ((6, 4, 4, 6), 1, 2)])
def test_abelian_flux_closed_form(orc, dims, n12, n34):
    U, th12, th34 = lu.abelian_flux(dims, n12, n34)
    V = lu.volume(dims)
    q = orc.topological_charge(dims, U)
    q_ref = V / (2 * math.pi ** 2) * math.sin(th12) * math.sin(th34)
    assert abs(q - q_ref) < 1e-12 * abs(q_ref)
    p = orc.plaquette(dims, U)
    p_ref = (4 + (1 + 2 * math.cos(th12)) / 3 + (1 + 2 * math.cos(th34)) / 3) / 6
    assert abs(p - p_ref) < 1e-14
    if (dims, n12, n34) == ((4, 4, 4, 4), 1, 1):
        assert abs(q.real - 1.89928) < 5e-6  # 1.89928... on 4^4, n = (1, 1)


def test_topological_charge_reflection(orc):
    """Q flips sign under the reflection x0 -> -x0 (an odd permutation of the
    epsilon tensor): U'_0(x) = U_0(Rx - 0)^{-1}, U'_i(x) = U_i(Rx)."""
    rng = np.random.default_rng(9)
    dims = (4, 2, 2, 2)
    U = lu.random_links(rng, dims, 0.6, 0.2)
    V = lu.volume(dims)
    Uc = lu.to_c(U)
    R = np.empty_like(Uc)
    for s in range(V):
        x = lu.coords(dims, s)
        rx = [(-x[0]) % dims[0]] + x[1:]
        rxm = [(-x[0] - 1) % dims[0]] + x[1:]
        R[s, 0] = np.linalg.inv(Uc[lu.site(dims, rxm), 0])
        for i in (1, 2, 3):
            R[s, i] = Uc[lu.site(dims, rx), i]
    q = orc.topological_charge(dims, U)
    qr = orc.topological_charge(dims, lu.from_c(R))
    assert abs(q) > 1e-3
    assert abs(q + qr) < 1e-12 * abs(q)
    # the Wilson action (symmetric in U_{mu nu} and its inverse) is reflection invariant
    s0 = orc.wilson_action(dims, U, 6.0)
    assert abs(s0 - orc.wilson_action(dims, lu.from_c(R), 6.0)) < 1e-12 * abs(s0)


def test_gauge_invariance(orc):
    """P, S_W and Q are invariant under SL(3,C) gauge transformations; the
    unitarity norm is invariant under SU(3) ones only."""
    rng = np.random.default_rng(10)
    dims = (4, 2, 2, 4)
    V = lu.volume(dims)
    U = lu.random_links(rng, dims, 0.5, 0.2)
    p0, q0 = orc.plaquette(dims, U), orc.topological_charge(dims, U)
    s0 = orc.wilson_action(dims, U, 6.0)
    un0 = orc.unitarity_norm(dims, U)
    W = U.copy()
    orc.gauge_transform(dims, W, lu.random_sl3c(rng, 0.5, 0.3, n=V))
    assert abs(orc.plaquette(dims, W) - p0) < 1e-13
    assert abs(orc.topological_charge(dims, W) - q0) < 1e-12 * max(1, abs(q0))
    assert abs(orc.wilson_action(dims, W, 6.0) - s0) < 1e-11 * abs(s0)
    assert abs(orc.unitarity_norm(dims, W) - un0) > 1e-3 * un0
    Y = U.copy()
    orc.gauge_transform(dims, Y, lu.random_su3(rng, n=V))
    assert abs(orc.unitarity_norm(dims, Y) - un0) < 1e-12 * un0
