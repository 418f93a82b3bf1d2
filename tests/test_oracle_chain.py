"""Pins of the SU(2) Polyakov-chain oracle against what the paper and the
mathematics fix: scipy's matrix exponential, finite-difference gradients of the
action and of the unitarity norm, the one-link gauge-cooling solution of the
section on the one-link model (rate equation and its fixed points), gauge
invariance of the Polyakov loop, and the exactly solvable equilibrium
<Tr P / 2> = I_2(beta) / I_1(beta) of the chain (section on the SU(2)
Polyakov chain: the model reduces to one link)."""
import numpy as np
import pytest
import scipy.linalg
import scipy.special

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]


def c2(a):
    return np.asarray(a)[..., 0::2] + 1j * np.asarray(a)[..., 1::2]


def to_m(links):
    return c2(links).reshape(links.shape[:-1] + (2, 2))


def from_m(m):
    m = np.asarray(m, complex)
    out = np.zeros(m.shape[:-2] + (8,))
    out[..., 0::2] = m.real.reshape(m.shape[:-2] + (4,))
    out[..., 1::2] = m.imag.reshape(m.shape[:-2] + (4,))
    return out


def sl2c(rng, re=0.4, im=0.2, n=None):
    shape = () if n is None else (n,)
    c = rng.normal(0, re, shape + (3,)) + 1j * rng.normal(0, im, shape + (3,))
    return np.array([scipy.linalg.expm(1j * sum(ci[a] * SIG[a] for a in range(3))) for ci in c.reshape(-1, 3)]
                    ).reshape(shape + (2, 2))


def action(links, beta):
    P = np.eye(2, dtype=complex)
    for U in to_m(links):
        P = P @ U
    return -0.5 * beta * np.trace(P)


def test_expm_matches_scipy(orc):
    rng = np.random.default_rng(1)
    for scale in (0.1, 1.0, 6.0):
        A = scale * (rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)))
        assert np.allclose(orc.chain_expm(A), scipy.linalg.expm(A), rtol=1e-12, atol=1e-12 * np.exp(2 * scale))
    A = 1j * sum(c * s for c, s in zip(rng.normal(size=3) + 0.3j * rng.normal(size=3), SIG))
    assert abs(np.linalg.det(orc.chain_expm(A)) - 1) < 1e-14


def test_noise_moments_and_streams(orc):
    eta = np.array([orc.chain_noise(5, c, k, 3) for c in range(40) for k in range(500)])
    assert abs(eta.mean()) < 0.02
    cov = eta.T @ eta / len(eta)
    assert np.allclose(cov, 2 * np.eye(3), atol=0.06)
    # different chains, steps and links draw different words; the same call repeats
    assert not np.allclose(orc.chain_noise(5, 0, 7, 3), orc.chain_noise(5, 1, 7, 3))
    assert not np.allclose(orc.chain_noise(5, 0, 7, 3), orc.chain_noise(5, 0, 7, 4))
    assert np.array_equal(orc.chain_noise(5, 2, 9, 1), orc.chain_noise(5, 2, 9, 1))


@pytest.mark.parametrize("n", [1, 2, 5])
def test_drift_is_minus_gradient_of_action(orc, n):
    """K_a(k) = -d/dt S(e^{i t sigma_a} U_k) (holomorphic: real-t central differences)."""
    rng = np.random.default_rng(n)
    links = from_m(sl2c(rng, n=n))
    beta = 1.3 - 0.7j
    K = to_m(orc.chain_drift(links, beta))
    h = 1e-5
    for k in range(n):
        Kfd = np.zeros((2, 2), complex)
        for a in range(3):
            lp, lm = links.copy(), links.copy()
            lp[k] = from_m(scipy.linalg.expm(1j * h * SIG[a]) @ to_m(links)[k])
            lm[k] = from_m(scipy.linalg.expm(-1j * h * SIG[a]) @ to_m(links)[k])
            Ka = -(action(lp, beta) - action(lm, beta)) / (2 * h)
            Kfd += Ka * SIG[a]
        assert np.allclose(K[k], Kfd, atol=1e-8 * max(1, np.abs(K[k]).max())), (k, K[k], Kfd)


def test_drift_closed_forms(orc):
    rng = np.random.default_rng(3)
    U = sl2c(rng)
    K = to_m(orc.chain_drift(from_m(U[None]), 0.9 + 0.2j))[0]
    assert np.allclose(K, 1j * (0.9 + 0.2j) * (U - 0.5 * np.trace(U) * np.eye(2)), atol=1e-14)
    # real beta on SU(2) links: K_a real, so Khat Hermitian (real Langevin)
    links = from_m(sl2c(rng, 0.8, 0.0, n=4))
    K = to_m(orc.chain_drift(links, 2.0))
    assert np.allclose(K, np.conj(np.swapaxes(K, -1, -2)), atol=1e-14)


def test_update_from_identity_is_pure_noise(orc):
    links = from_m(np.broadcast_to(np.eye(2), (3, 2, 2)).copy())
    K = np.zeros((3, 8))
    eps = 0.01
    orc.chain_update(links, K, eps, 9, 4, 2)
    for k in range(3):
        eta = orc.chain_noise(9, 4, k, 2)
        ref = scipy.linalg.expm(1j * np.sqrt(eps) * sum(eta[a] * SIG[a] for a in range(3)))
        assert np.allclose(to_m(links)[k], ref, atol=1e-14)


def test_real_langevin_stays_unitary(orc):
    links = from_m(sl2c(np.random.default_rng(4), 0.7, 0.0, n=6))
    rc, obs, _ = orc.chain_run(links, 2.0, 5, 0, 200, 1e-2, False, 0, 1e-2)
    assert rc == 0 and np.max(np.abs(obs[:, 2])) < 1e-13
    m = to_m(links)
    assert np.allclose(np.linalg.det(m), 1, atol=1e-14)


def test_cooling_gradient_is_gradient_of_unitarity_norm(orc):
    """f_ak = d/d delta UN under U_k -> Omega U_k, U_{k-1} -> U_{k-1} Omega^-1, Omega = exp(delta sigma_a)."""
    rng = np.random.default_rng(6)
    for n in (1, 3):
        links = from_m(sl2c(rng, n=n))
        f = orc.chain_gradient(links)
        h = 1e-6
        for k in range(n):
            for a in range(3):
                vals = []
                for s in (+1, -1):
                    m = to_m(links).copy()
                    O = scipy.linalg.expm(s * h * SIG[a])
                    m[k] = O @ m[k]
                    m[(k - 1) % n] = m[(k - 1) % n] @ np.linalg.inv(O)
                    vals.append(np.sum(np.abs(m) ** 2))
                assert abs((vals[0] - vals[1]) / (2 * h) - f[k, a]) < 1e-6 * max(1, abs(f[k, a]))


def test_one_link_cooling_rate(orc):
    """One-link model: with Pauli generators (Tr sigma sigma = 2 delta) the
    paper's rate equation, written for sigma/2, reads
    d' = -32 alpha (d^2 + 2(1 - |c|^2) d + c^2 + c*^2 - 2|c|^2),
    c = Tr U / 2; and f^2 = 16 Tr(U U^dag [U, U^dag]) (eq. (eqgc))."""
    rng = np.random.default_rng(7)
    for _ in range(4):
        U = sl2c(rng, 0.6, 0.4)
        c = 0.5 * np.trace(U)
        d = 0.5 * np.trace(U @ U.conj().T).real - 1
        Ud = U.conj().T
        f = orc.chain_gradient(from_m(U[None]))[0]
        assert abs((f ** 2).sum() - 16 * np.trace(U @ Ud @ (U @ Ud - Ud @ U)).real) < 1e-10 * (f ** 2).sum()
        rate = -32 * (d * d + 2 * (1 - abs(c) ** 2) * d + (c * c + np.conj(c) ** 2).real - 2 * abs(c) ** 2)
        eps = 1e-7
        links = from_m(U[None])
        orc.chain_cool_step(links, eps)
        d1 = orc.chain_measure(links, 1.0)[1]
        assert abs((d1 - d) / eps - rate) < 1e-4 * abs(rate)


def test_one_link_cooling_fixed_points(orc):
    """Real c (gauge equivalent to SU(2)): d -> 0 at the rate 64 alpha (1 - c^2)
    (the paper's 16 alpha (1 - c^2) for sigma/2); complex c: d -> |c|^2 - 1 +
    sqrt(1 - c^2 - c*^2 + |c|^4) > 0.  c itself is invariant."""
    rng = np.random.default_rng(8)
    V = sl2c(rng, 0.9, 0.0)
    O = sl2c(rng, 0.3, 0.5)
    U = O @ V @ np.linalg.inv(O)
    c = 0.5 * np.trace(U)
    assert abs(c.imag) < 1e-12
    links = from_m(U[None])
    ea = 2e-3
    for _ in range(200):
        orc.chain_cool_step(links, ea)
    d_a = orc.chain_measure(links, 1.0)[1]
    for _ in range(100):
        orc.chain_cool_step(links, ea)
    d_b = orc.chain_measure(links, 1.0)[1]
    rate = -np.log(d_b / d_a) / (100 * ea)
    assert abs(rate - 64 * (1 - c.real ** 2)) < 0.02 * 64 * (1 - c.real ** 2)
    assert abs(0.5 * np.trace(to_m(links)[0]) - c) < 1e-12
    U = sl2c(rng, 0.7, 0.4)
    c = 0.5 * np.trace(U)
    dinf = abs(c) ** 2 - 1 + np.sqrt((1 - c * c - np.conj(c) ** 2 + abs(c) ** 4).real)
    links = from_m(U[None])
    for _ in range(20000):
        orc.chain_cool_step(links, 5e-3)
    assert abs(orc.chain_measure(links, 1.0)[1] - dinf) < 1e-9 and dinf > 1e-3


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_chain_cooling_keeps_loop_and_reduces_distance(orc, mode):
    """A gauge-transformed unitary chain: cooling keeps L = Tr P / 2 and det,
    and brings d towards 0 (section on the chain model)."""
    rng = np.random.default_rng(9)
    n = 8
    V = sl2c(rng, 0.8, 0.0, n=n)
    O = sl2c(rng, 0.3, 0.3, n=n)
    U = np.array([O[k] @ V[k] @ np.linalg.inv(O[(k + 1) % n]) for k in range(n)])
    links = from_m(U)
    L0, d0, _ = orc.chain_measure(links, 1.0)
    rc, un, al = orc.chain_cool(links, 400, 1e-2, 1.0, mode)
    L1, d1, _ = orc.chain_measure(links, 1.0)
    assert rc == 0 and abs(L1 - L0) < 1e-12 and d1 < 0.2 * d0
    assert np.allclose(np.linalg.det(to_m(links)), 1, atol=1e-13)
    if mode == 1:
        assert np.allclose(al, 1.0 / (un[:-1] / n))


@pytest.mark.timeout(300)
def test_real_beta_equilibrium_is_the_bessel_ratio(orc):
    """Real beta: CL is real Langevin on SU(2), whose equilibrium is the
    one-link model: <Tr P / 2> = I_2(beta) / I_1(beta)."""
    beta = 2.0
    n, chains, steps, therm = 3, 48, 3000, 500
    means = []
    for c in range(chains):
        links = orc.chain_init(n, c, 21, 0.3, 0.0)
        rc, obs, _ = orc.chain_run(links, beta, 21, c, steps, 5e-3, False, 0, 5e-3)
        assert rc == 0
        means.append(obs[therm:, 0].mean())
    m, err = np.mean(means), np.std(means) / np.sqrt(chains)
    exact = scipy.special.iv(2, beta) / scipy.special.iv(1, beta)
    # O(eps) step bias is well below the statistical error at eps = 5e-3
    assert abs(m - exact) < 4 * err + 0.01, (m, err, exact)


@pytest.mark.timeout(120)
def test_chain_cooling_power_law(orc):
    """Section on the chain model (figure of adaptive variants on a long
    chain): cooling a gauge-rotated unitary chain with fixed alpha, d(t) decays
    asymptotically like t^(-3/2).  (Linearised, cooling diffuses the gauge
    field; for independent Omega_k the non-unitarity is its lattice gradient,
    so d ~ sum_k k^2 exp(-c k^2 t) ~ t^(-3/2).)  16 chains of 100 links,
    eps_c alpha = 1e-2, slope of log <d> between 300 and 3000 steps."""
    from tests.chainutil import gauge_rotated_chains
    links = gauge_rotated_chains(16, 100, 40)
    d = np.zeros(2)
    for c in range(16):
        lk = links[c].copy()
        L0 = orc.chain_measure(lk, 1.0)[0]
        orc.chain_cool(lk, 300, 1e-2, 1.0, 0)
        d[0] += orc.chain_measure(lk, 1.0)[1]
        orc.chain_cool(lk, 2700, 1e-2, 1.0, 0)
        L1, d1, _ = orc.chain_measure(lk, 1.0)
        d[1] += d1
        assert abs(L1 - L0) < 1e-11
    slope = np.log(d[1] / d[0]) / np.log(10.0)
    assert abs(slope + 1.5) < 0.2, slope
