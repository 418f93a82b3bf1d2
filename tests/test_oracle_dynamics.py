"""Pins for the oracle's drift, Langevin update and gauge cooling: central
finite differences of the action, the topological charge and the unitarity
norm, the one-link cooling rate of the paper, closed forms and invariants."""
import numpy as np
import pytest
import scipy.linalg

from tests import latutil as lu


def _replace(U, s, mu, M):
    W = U.copy()
    W[s, mu] = lu.from_c(M)
    return W


def _fd_lie_derivative(fun, U, s, mu, h=1e-3):
    """D_a f = d/dt f(exp(i t lambda_a) U_{s,mu}) at t = 0 for a = 1..8,
    by the 4-point central stencil (error O(h^4))."""
    U0 = lu.to_c(U[s, mu])
    out = np.zeros(8, dtype=np.complex128)
    for a in range(8):
        vals = {}
        for k in (-2, -1, 1, 2):
            vals[k] = fun(_replace(U, s, mu, scipy.linalg.expm(1j * k * h * lu.LAMBDA[a]) @ U0))
        out[a] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
    return out


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 3, 3, 3), (4, 2, 2, 2)])
def test_wilson_drift_is_minus_gradient_of_action(orc, dims):
    rng = np.random.default_rng(11)
    U = lu.random_links(rng, dims, 0.5, 0.2)
    beta = 5.7
    K = orc.drift(dims, U, beta, 0.0)
    V = lu.volume(dims)
    for s, mu in [(0, 0), (V - 1, 3), (V // 2, 1), (5 % V, 2)]:
        DS = _fd_lie_derivative(lambda W: orc.wilson_action(dims, W, beta), U, s, mu)
        Kfd = lu.lie(-DS)
        Kor = lu.to_c(K[s, mu])
        assert np.max(np.abs(Kor - Kfd)) < 1e-8 * np.max(np.abs(Kor))
        # the drift is traceless
        assert abs(np.trace(Kor)) < 1e-13 * np.max(np.abs(Kor))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 3, 3, 3), (2, 4, 2, 2)])
def test_theta_drift_is_gradient_of_topological_charge(orc, dims):
    """K_a = -D_a(-i theta Q) = i theta D_a Q for beta = 0."""
    rng = np.random.default_rng(12)
    U = lu.random_links(rng, dims, 0.6, 0.3)
    V = lu.volume(dims)
    for theta in (1.0, 0.7 - 0.4j):
        K = orc.drift(dims, U, 0.0, theta)
        for s, mu in [(0, 0), (V - 1, 3), (V // 3, 1), (7 % V, 2)]:
            DQ = _fd_lie_derivative(lambda W: orc.topological_charge(dims, W), U, s, mu)
            Kfd = lu.lie(1j * theta * DQ)
            Kor = lu.to_c(K[s, mu])
            assert np.max(np.abs(Kor)) > 1e-6
            assert np.max(np.abs(Kor - Kfd)) < 1e-7 * np.max(np.abs(Kor))


def test_full_drift_is_linear_in_beta_and_theta(orc):
    rng = np.random.default_rng(13)
    dims = (2, 2, 4, 2)
    U = lu.random_links(rng, dims)
    Kw = orc.drift(dims, U, 6.0, 0.0)
    Kt = orc.drift(dims, U, 0.0, 2.0)
    K = orc.drift(dims, U, 6.0, 2.0)
    np.testing.assert_allclose(K, Kw + Kt, atol=1e-12)


def test_drift_closed_forms(orc):
    dims = (4, 4, 4, 4)
    # cold start: no force
    assert np.max(np.abs(orc.drift(dims, orc.cold_links(dims), 6.0, 1.0))) == 0.0
    # uniform abelian flux: every loop pair cancels, Wilson and theta drift vanish
    U, _, _ = lu.abelian_flux(dims, 1, 1)
    assert np.max(np.abs(orc.drift(dims, U, 6.0, 1.0))) < 1e-13


def test_drift_hermiticity(orc):
    """On SU(3) links the action is real for theta = 0 and for imaginary
    theta, so the drift coefficients K_a are real (Khat Hermitian); a real
    theta makes the action complex and the drift non-Hermitian."""
    rng = np.random.default_rng(14)
    dims = (2, 2, 2, 4)
    U = lu.from_c(lu.random_su3(rng, n=lu.volume(dims) * 4)).reshape(-1, 4, 18)
    for theta, herm in ((0.0, True), (1.5j, True), (1.5, False)):
        K = lu.to_c(orc.drift(dims, U, 6.0, theta))
        dev = np.max(np.abs(K - np.conj(np.swapaxes(K, -1, -2))))
        if herm:
            assert dev < 1e-12
        else:
            assert dev > 1e-6


def test_update_from_cold_start_is_pure_noise(orc):
    """With zero drift one step gives U = exp(i sqrt(eps) eta_a lambda_a) exactly."""
    dims = (2, 2, 2, 2)
    U = orc.cold_links(dims)
    eps, seed, step = 1e-2, 99, 7
    eps_n, kmax, _ = orc.langevin_step(dims, U, 6.0, 0.0, seed, step, eps)
    assert eps_n == eps and kmax == 0.0
    for s in range(lu.volume(dims)):
        for mu in range(4):
            eta = orc.cl_noise(seed, s, mu, step)
            ref = scipy.linalg.expm(1j * np.sqrt(eps) * lu.lie(eta))
            np.testing.assert_allclose(lu.to_c(U[s, mu]), ref, atol=1e-14)


def test_update_formula(orc):
    """U' = exp(i(eps K + sqrt(eps) eta)) U det(.)^{-1/3} for a given drift."""
    rng = np.random.default_rng(15)
    dims = (2, 2, 2, 2)
    U = lu.random_links(rng, dims)
    K = lu.from_c(lu.lie(rng.normal(size=(8,)) + 1j * rng.normal(size=(8,)))[None, None]
                  * np.ones((lu.volume(dims), 4, 1, 1)))
    W = U.copy()
    orc.langevin_update(dims, W, np.ascontiguousarray(K), 3e-3, 5, 1)
    for s, mu in [(0, 0), (9, 3)]:
        eta = orc.cl_noise(5, s, mu, 1)
        X = 3e-3 * lu.to_c(K[s, mu]) + np.sqrt(3e-3) * lu.lie(eta)
        R = scipy.linalg.expm(1j * X) @ lu.to_c(U[s, mu])
        R = R * np.linalg.det(R) ** (-1 / 3)
        np.testing.assert_allclose(lu.to_c(W[s, mu]), R, atol=1e-13)
    dmax, tmin = orc.link_stats(dims, W)
    assert dmax < 1e-14 and tmin >= 1.0


def test_real_langevin_stays_unitary(orc):
    """theta = 0 (and imaginary theta) from an SU(3) start is real Langevin:
    links stay in SU(3) and the unitarity distance stays at rounding level."""
    rng = np.random.default_rng(16)
    dims = (2, 2, 2, 2)
    for theta in (0.0, 1.0j):
        U = lu.from_c(lu.random_su3(rng, n=lu.volume(dims) * 4)).reshape(-1, 4, 18)
        for n in range(10):
            orc.langevin_step(dims, U, 6.0, theta, 3, n, 1e-2)
        assert abs(orc.distance(dims, U)) < 1e-13
    U = lu.from_c(lu.random_su3(rng, n=lu.volume(dims) * 4)).reshape(-1, 4, 18)
    for n in range(10):
        orc.langevin_step(dims, U, 6.0, 2.0, 3, n, 1e-2)
    assert orc.distance(dims, U) > 1e-8


def test_adaptive_step_size(orc):
    dims = (4, 4, 4, 4)
    U = orc.init_links(dims, 2)
    eps0 = 1e-2
    bound = 0.0
    for n in range(4):
        eps, kmax, bound = orc.langevin_step(dims, U, 6.0, 0.0, 2, n, eps0, adaptive=True,
                                             bound=bound)
        if n == 0:
            assert eps == eps0 and abs(bound - eps0 * kmax) < 1e-15 * bound
        assert eps <= eps0
        assert eps * kmax <= bound * (1 + 1e-15)
        K = orc.drift(dims, U, 6.0, 0.0)  # drift of the next step
    # an explicit bound caps the step
    U2 = orc.init_links(dims, 2)
    eps, kmax, b = orc.langevin_step(dims, U2, 6.0, 0.0, 2, 0, eps0, adaptive=True,
                                     drift_bound=1e-3)
    assert b == 1e-3 and abs(eps - min(eps0, 1e-3 / kmax)) < 1e-18


def _transform_one_site(U, dims, s, Om):
    W = lu.to_c(U).copy()
    x = lu.coords(dims, s)
    Oi = np.linalg.inv(Om)
    for mu in range(4):
        W[s, mu] = Om @ W[s, mu]
        xb = list(x)
        xb[mu] -= 1
        b = lu.site(dims, xb)
        W[b, mu] = W[b, mu] @ Oi
    return lu.from_c(W)


def test_cooling_gradient_is_gradient_of_unitarity_norm(orc):
    """f_ax = d/d delta of sum Tr U U^dagger under Omega_x = exp(delta lambda_a)."""
    rng = np.random.default_rng(17)
    dims = (2, 2, 2, 2)
    U = lu.random_links(rng, dims, 0.5, 0.3)
    h = 1e-3
    for s in (0, 5, 15):
        f = orc.cool_gradient(dims, U, s)
        fd = np.zeros(8)
        for a in range(8):
            v = {k: orc.unitarity_norm(dims, _transform_one_site(
                U, dims, s, scipy.linalg.expm(k * h * lu.LAMBDA[a]))) for k in (-2, -1, 1, 2)}
            fd[a] = (8 * (v[1] - v[-1]) - (v[2] - v[-2])) / (12 * h)
        assert np.max(np.abs(f - fd)) < 1e-8 * np.max(np.abs(f))


def test_one_link_cooling_rate(orc):
    """Paper's one-link rate: f_a f_a = 16 Tr(U U^dagger [U, U^dagger]), and to
    first order in eps a half-sweep lowers the norm by eps alpha sum f^2
    (d_dot = -alpha f^2 / N for the one-link model)."""
    rng = np.random.default_rng(18)
    dims = (2, 2, 2, 2)
    Uc = np.tile(np.eye(3, dtype=np.complex128), (lu.volume(dims), 4, 1, 1))
    M = lu.random_sl3c(rng, 0.6, 0.4)
    x0 = lu.site(dims, (0, 0, 0, 0))
    x1 = lu.site(dims, (1, 0, 0, 0))
    Uc[x0, 0] = M
    Uc[x1, 0] = M  # on L0 = 2 the backward link at x0 is U_0(x1)
    U = lu.from_c(Uc)
    f = orc.cool_gradient(dims, U, x0)
    rhs = 16 * np.trace(M @ M.conj().T @ (M @ M.conj().T - M.conj().T @ M))
    assert abs(np.sum(f ** 2) - rhs.real) < 1e-12 * abs(rhs) and abs(rhs.imag) < 1e-12 * abs(rhs)
    # first-order lattice rate over the even half-sweep
    U2 = lu.random_links(rng, dims, 0.5, 0.3)
    un0 = orc.unitarity_norm(dims, U2)
    fsum = sum(np.sum(orc.cool_gradient(dims, U2, s) ** 2)
               for s in range(lu.volume(dims)) if sum(lu.coords(dims, s)) % 2 == 0)
    rates = []
    for ea in (1e-5, 2e-5):
        W = U2.copy()
        orc.cool_halfsweep(dims, W, 0, ea)
        rates.append((orc.unitarity_norm(dims, W) - un0) / ea)
    rate0 = 2 * rates[0] - rates[1]  # Richardson: remove the O(eps) term
    assert abs(rate0 + fsum) < 1e-5 * fsum


def test_cooling_preserves_gauge_invariants_and_det(orc):
    rng = np.random.default_rng(19)
    dims = (4, 2, 2, 4)
    U = lu.random_links(rng, dims, 0.5, 0.3)
    p0, q0 = orc.plaquette(dims, U), orc.topological_charge(dims, U)
    un, al = orc.gauge_cool(dims, U, 20, 0.01, 1.0, 0)
    assert abs(orc.plaquette(dims, U) - p0) < 1e-13
    assert abs(orc.topological_charge(dims, U) - q0) < 1e-12 * max(1, abs(q0))
    assert np.all(np.diff(un) <= 0)  # "not possible to cool too much": monotone
    dmax, tmin = orc.link_stats(dims, U)
    assert dmax < 1e-13 and tmin >= 1.0
    np.testing.assert_array_equal(al, 1.0)


def test_cooling_returns_gauge_rotated_su3_to_unitarity(orc):
    """A configuration gauge-equivalent to SU(3) cools towards d = 0 while the
    distance of a generic SL(3,C) configuration stays finite."""
    rng = np.random.default_rng(20)
    dims = (2, 2, 2, 2)
    V = lu.volume(dims)
    S = lu.from_c(lu.random_su3(rng, n=V * 4)).reshape(-1, 4, 18)
    orc.gauge_transform(dims, S, lu.random_sl3c(rng, 0.0, 0.3, n=V))
    d0 = orc.distance(dims, S)
    un, _ = orc.gauge_cool(dims, S, 400, 0.05, 1.0, 1)
    d1 = orc.distance(dims, S)
    assert d0 > 0.05 and d1 < 1e-6 * d0
    G = lu.random_links(rng, dims, 0.5, 0.3)
    un, _ = orc.gauge_cool(dims, G, 400, 0.05, 1.0, 1)
    assert orc.distance(dims, G) > 1e-3


def test_adaptive_alpha_modes(orc):
    rng = np.random.default_rng(21)
    dims = (2, 2, 2, 2)
    V = lu.volume(dims)
    U = lu.random_links(rng, dims, 0.5, 0.3)
    W = U.copy()
    un, al = orc.gauge_cool(dims, W, 3, 1e-3, 2.0, 1)
    np.testing.assert_allclose(al, 2.0 / (un[:3] / (4 * V)), rtol=1e-15)
    W = U.copy()
    f = np.array([orc.cool_gradient(dims, W, s) for s in range(V)])
    un, al = orc.gauge_cool(dims, W, 1, 1e-3, 2.0, 2)
    np.testing.assert_allclose(al[0], 2.0 / np.mean(np.abs(f)), rtol=1e-13)
    # odd extents cannot be checkerboarded
    with pytest.raises(RuntimeError):
        orc.gauge_cool((3, 2, 2, 2), lu.random_links(rng, (3, 2, 2, 2)), 1, 1e-3)


def test_run_resume_is_bitwise(orc):
    dims = (4, 4, 4, 4)
    a = orc.init_links(dims, 1)
    b = a.copy()
    oa, ba = orc.run(dims, a, 5.7, 0.5, 1, 4, 1e-2, True, 3, 1e-2, 1.0, 1)
    ob1, bb = orc.run(dims, b, 5.7, 0.5, 1, 2, 1e-2, True, 3, 1e-2, 1.0, 1)
    ob2, bb = orc.run(dims, b, 5.7, 0.5, 1, 2, 1e-2, True, 3, 1e-2, 1.0, 1, step0=2, bound=bb)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(oa, np.concatenate([ob1, ob2]))
    assert np.all(oa[:, 1] <= oa[:, 0])  # cooling lowers d


def test_sampled_drift_equals_full_drift(orc):
    """The per-link entry point (clover matrices evaluated on demand) gives the
    same drift as the whole-lattice one."""
    rng = np.random.default_rng(22)
    dims = (4, 2, 4, 2)
    U = lu.random_links(rng, dims)
    for theta in (0.0, 0.7 + 0.2j):
        K = orc.drift(dims, U, 5.0, theta).reshape(-1, 18)
        sel = np.arange(0, 4 * lu.volume(dims), 3)
        np.testing.assert_array_equal(orc.drift_links(dims, U, 5.0, theta, sel), K[sel])


@pytest.mark.timeout(60)
def test_expm_of_non_finite_matrix_terminates(orc):
    """A runaway configuration can hand the exponential an infinite entry: the
    scaling loop must stay bounded and the result be non-finite (regression:
    halving an infinite norm never reached the threshold)."""
    A = np.zeros((3, 3), complex)
    A[0, 1] = np.inf
    assert not np.all(np.isfinite(orc.expm(A)))
    A[0, 1] = np.nan
    assert not np.all(np.isfinite(orc.expm(A)))
    # finite inputs of any size still give the exact exponential
    X = 40.0 * lu.lie(np.random.default_rng(3).normal(size=8))
    assert np.allclose(orc.expm(1j * X), scipy.linalg.expm(1j * X), rtol=1e-9, atol=1e-9)
