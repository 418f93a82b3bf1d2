"""GPU parity of the SU(2) Polyakov-chain workload (cl_chain_*) against the
FP64 oracle: start, drift (scans up to 1024 links), single CL steps with
identical Philox words (fixed and adaptive step, D_0/D_1/D_2 cooling),
cooling alone, trajectories, independence of chains, runaway handling, and
the exactly solvable equilibrium <Tr P / 2> = I_2(beta) / I_1(beta) for real
beta.  All calls go through the C ABI.

Tolerances: FP64 everywhere.  The drift is the same product of n 2x2
matrices associated differently (a prefix and a suffix scan on the GPU, a
left-to-right product in the oracle), so its rounding grows with n like
n * 1e-16 relative for near-unitary links; 1e-12 covers n <= 1024 with a
margin of ten.  Exponentials differ in method (closed 2x2 series on the GPU,
Taylor with scaling and squaring in the oracle), both at rounding level."""
import numpy as np
import pytest
import scipy.linalg
import scipy.special

pytestmark = pytest.mark.gpu

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]


@pytest.fixture(scope="module")
def cl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_1056_amd as cl
    return cl


def say(*a):
    print(*a, flush=True)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def sl2c_links(rng, shape, re=0.4, im=0.2):
    c = rng.normal(0, re, shape + (3,)) + 1j * rng.normal(0, im, shape + (3,))
    m = np.array([scipy.linalg.expm(1j * sum(ci[a] * SIG[a] for a in range(3))) for ci in c.reshape(-1, 3)])
    out = np.zeros(shape + (8,))
    out[..., 0::2] = m.real.reshape(shape + (4,))
    out[..., 1::2] = m.imag.reshape(shape + (4,))
    return out


def test_init_matches_oracle(cl, orc):
    say("chain init")
    ch = cl.Chain(37, 3, 1.0, seed=11)
    ch.init(0.3, 0.05)
    U = ch.get_links()
    for c in range(3):
        assert relerr(U[c], orc.chain_init(37, c, 11, 0.3, 0.05)) < 1e-14, c
    ch.close()


def test_init_of_many_chains(cl, orc):
    """More chains than a grid's second dimension holds (70000 chains of 3
    links): the start of sampled chains equals the oracle's."""
    say("chain init, 70000 chains")
    ch = cl.Chain(3, 70000, 1.0, seed=13)
    ch.init(0.3, 0.05)
    U = ch.get_links()
    for c in (0, 65534, 65535, 65536, 69999):
        assert relerr(U[c], orc.chain_init(3, c, 13, 0.3, 0.05)) < 1e-14, c
    m = ch.measure()
    assert all(x["status"] == 0 and x["step"] == 0 for x in m[65530:65540])
    ch.close()


# (two links per thread up to 512 links, four above)
@pytest.mark.parametrize("n", [1, 2, 5, 64, 257, 512, 513, 1000, 1024])
def test_drift_matches_oracle(cl, orc, n):
    say("chain drift", n)
    rng = np.random.default_rng(n)
    links = sl2c_links(rng, (2, n))
    beta = 1.7 - 0.6j
    ch = cl.Chain(n, 2, beta, seed=1)
    ch.set_links(links)
    K, kmax = ch.drift()
    for c in range(2):
        ref = orc.chain_drift(links[c], beta)
        assert relerr(K[c], ref) < 1e-12, (n, c, relerr(K[c], ref))
        Kc = orc.chain_to_complex(ref)
        kref = np.sqrt(np.max(0.5 * np.sum(np.abs(Kc) ** 2, axis=(1, 2))))
        assert abs(kmax[c] - kref) < 1e-12 * kref
    ch.close()


@pytest.mark.parametrize("adaptive", [False, True])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_step_matches_oracle(cl, orc, adaptive, mode):
    """One CL step + 3 cooling steps from identical links and Philox words."""
    say("chain step", adaptive, mode)
    n, nc, beta, seed = 9, 3, 2.0 + 0.8j, 5
    links = sl2c_links(np.random.default_rng(3 + mode), (nc, n))
    ch = cl.Chain(n, nc, beta, seed=seed, obs_cap=4)
    ch.set_links(links)
    ch.run(1, 1e-2, adaptive, 3, 1e-2, 1.0, mode, record=True)
    U = ch.get_links()
    rec = ch.record(1)
    for c in range(nc):
        ref = links[c].copy()
        rc, obs, _ = orc.chain_run(ref, beta, seed, c, 1, 1e-2, adaptive, 3, 1e-2, 1.0, mode)
        assert rc == 0
        assert relerr(U[c], ref) < 1e-12, (c, relerr(U[c], ref))
        assert np.allclose(rec[0, c], obs[0], rtol=1e-12, atol=1e-13), (c, rec[0, c], obs[0])
    ch.close()


@pytest.mark.parametrize("n", [16, 512, 513])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_cooling_matches_oracle(cl, orc, mode, n):
    say("chain cooling", mode, n)
    nc = 2
    links = sl2c_links(np.random.default_rng(20 + mode + n), (nc, n), 0.5, 0.4)
    ch = cl.Chain(n, nc, 1.0)
    ch.set_links(links)
    ch.cool(25, 1e-2, 1.0, mode)
    U = ch.get_links()
    m = ch.measure()
    for c in range(nc):
        ref = links[c].copy()
        rc, un, _ = orc.chain_cool(ref, 25, 1e-2, 1.0, mode)
        assert rc == 0 and relerr(U[c], ref) < 1e-12, (c, relerr(U[c], ref))
        L, d, _ = orc.chain_measure(ref, 1.0)
        # L is a product of n links: its rounding error scales with |L|
        assert abs(m[c]["L"] - L) < 1e-12 * max(1.0, abs(L)), (c, m[c]["L"], L)
        assert abs(m[c]["d"] - d) < 1e-12 * max(1.0, abs(d)), (c, m[c]["d"], d)
    ch.close()


def test_trajectory_matches_oracle(cl, orc):
    """20 steps with adaptive step and D_1 cooling: per-step record and final
    links (rounding differences stay at the 1e-12 level over 20 steps)."""
    say("chain trajectory")
    n, nc, beta, seed = 12, 2, 1.5 + 1.0j, 8
    ch = cl.Chain(n, nc, beta, seed=seed, obs_cap=20)
    ch.init(0.3, 0.05)
    links = ch.get_links()
    ch.run(20, 5e-3, True, 5, 5e-3, 1.0, 1, record=True)
    rec = ch.record(20)
    U = ch.get_links()
    for c in range(nc):
        ref = links[c].copy()
        rc, obs, _ = orc.chain_run(ref, beta, seed, c, 20, 5e-3, True, 5, 5e-3, 1.0, 1)
        assert rc == 0
        assert relerr(U[c], ref) < 1e-11
        assert np.allclose(rec[:, c], obs, rtol=1e-10, atol=1e-12)
    m = ch.measure()
    assert all(x["step"] == 20 and x["status"] == 0 and x["n_sum"] == 20 for x in m)
    # the running means are Langevin-time averages: sum eps_n L_n / sum eps_n
    for c in range(nc):
        w = rec[:, c, 3]
        assert abs(m[c]["t_sum"] - w.sum()) < 1e-15 * 20
        ref = np.sum(w * (rec[:, c, 0] + 1j * rec[:, c, 1])) / w.sum()
        assert abs(m[c]["mean_L"] - ref) < 1e-13
        assert abs(m[c]["mean_d"] - np.sum(w * rec[:, c, 2]) / w.sum()) < 1e-13
    ch.close()


def test_chains_are_independent_and_resumable(cl):
    """A chain's result does not depend on the others, and two calls of 5
    steps equal one call of 10 (the step counter and the bound carry over)."""
    say("chain independence")
    n = 33
    rng = np.random.default_rng(4)
    links = sl2c_links(rng, (3, n))
    a = cl.Chain(n, 3, 2.0 + 0.5j, seed=2)
    a.set_links(links)
    a.run(10, 1e-2, True, 2, 1e-2, 1.0, 1)
    b = cl.Chain(n, 3, 2.0 + 0.5j, seed=2)
    other = links.copy()
    other[1] = sl2c_links(rng, (1, n))[0]
    b.set_links(other)
    b.run(5, 1e-2, True, 2, 1e-2, 1.0, 1)
    b.run(5, 1e-2, True, 2, 1e-2, 1.0, 1)
    Ua, Ub = a.get_links(), b.get_links()
    assert np.array_equal(Ua[0], Ub[0]) and np.array_equal(Ua[2], Ub[2])
    assert not np.allclose(Ua[1], Ub[1])
    a.close()
    b.close()


@pytest.mark.parametrize("n", [4, 100, 300])
def test_chain_does_not_depend_on_batch(cl, n):
    """Short chains share a workgroup (T threads each, 64 / T or 256 / T per
    workgroup): a chain's result equals, bit for bit, that of the same chain
    run in a batch of another size."""
    say("chain batch independence", n)
    nc = 70
    links = sl2c_links(np.random.default_rng(30 + n), (nc, n), 0.3, 0.01)
    out = []
    for m in (nc, 3):
        ch = cl.Chain(n, m, 1.5 + 0.7j, seed=4, obs_cap=3)
        ch.set_links(links[:m])
        ch.run(3, 1e-2, True, 4, 1e-2, 1.0, 2, record=True)
        out.append((ch.get_links(), ch.record(3), ch.measure()))
        ch.close()
    assert np.array_equal(out[0][0][:3], out[1][0])
    assert np.array_equal(out[0][1][:, :3], out[1][1])
    assert all(x["status"] == 0 for x in out[0][2])
    assert [x["mean_L"] for x in out[0][2][:3]] == [x["mean_L"] for x in out[1][2]]


def test_many_workgroups_of_short_chains_match_oracle(cl, orc):
    """n = 4 (one thread per chain, 64 chains per workgroup) over three
    workgroups, the last one partly filled."""
    say("chain short, 3 workgroups")
    n, nc, beta, seed = 4, 130, 2.0 - 0.4j, 12
    links = sl2c_links(np.random.default_rng(13), (nc, n))
    ch = cl.Chain(n, nc, beta, seed=seed, obs_cap=2)
    ch.set_links(links)
    ch.run(2, 1e-2, True, 3, 1e-2, 1.0, 1, record=True)
    U = ch.get_links()
    rec = ch.record(2)
    for c in (0, 63, 64, 127, 128, 129):
        ref = links[c].copy()
        rc, obs, _ = orc.chain_run(ref, beta, seed, c, 2, 1e-2, True, 3, 1e-2, 1.0, 1)
        assert rc == 0 and relerr(U[c], ref) < 1e-12, (c, relerr(U[c], ref))
        assert np.allclose(rec[:, c], obs, rtol=1e-12, atol=1e-13)
    ch.close()


def test_runaway_chain_is_frozen_alone(cl):
    say("chain runaway")
    n = 6
    links = sl2c_links(np.random.default_rng(5), (3, n))
    links[1, 2, 3] = np.nan
    ch = cl.Chain(n, 3, 1.0, seed=3)
    ch.set_links(links)
    ch.run(4, 1e-2, True, 2, 1e-2, 1.0, 2)
    m = ch.measure()
    U = ch.get_links()
    assert m[1]["status"] == 1 and m[1]["step"] == 0
    assert np.array_equal(U[1][~np.isnan(links[1])], links[1][~np.isnan(links[1])])
    assert m[0]["status"] == 0 and m[2]["status"] == 0 and m[0]["step"] == 4
    ch.close()


def test_real_beta_equilibrium_is_the_bessel_ratio(cl):
    """Real beta is real Langevin on SU(2): the ensemble and time average of
    Tr P / 2 is I_2(beta) / I_1(beta) (the chain reduces to one link)."""
    say("chain equilibrium, real beta")
    beta, n, nc = 2.0, 4, 512
    ch = cl.Chain(n, nc, beta, seed=9)
    ch.init(0.3, 0.0)
    ch.run(600, 5e-3)                 # thermalisation
    ch.run(3000, 5e-3)
    m = ch.measure()
    means = np.array([x["mean_L"].real for x in m])
    exact = scipy.special.iv(2, beta) / scipy.special.iv(1, beta)
    err = means.std() / np.sqrt(nc)
    # the O(eps) step bias at eps = 5e-3 is below 0.005 here
    assert abs(means.mean() - exact) < 4 * err + 0.005, (means.mean(), err, exact)
    assert max(abs(x["mean_L"].imag) for x in m) < 1e-12
    ch.close()


def test_complex_beta_cooled_cl_converges_to_exact(cl):
    """Complex beta = 2 + i, 10 links, adaptive step with 10 D_2 cooling steps
    per update: the Langevin-time average of S = -beta Tr P / 2, linearly
    extrapolated to eps = 0 from eps0 = 1e-3 and 5e-4 (the step-size bias is
    O(eps)), equals the exact one-link value -beta I_2(beta) / I_1(beta)
    (section on the SU(2) Polyakov chain and its reduction to one link)."""
    say("chain complex beta convergence")
    beta = 2.0 + 1.0j
    exact = -beta * scipy.special.iv(2, beta) / scipy.special.iv(1, beta)
    est = []
    for eps, seed in ((1e-3, 17), (5e-4, 18)):
        ch = cl.Chain(10, 1024, beta, seed=seed)
        ch.init(0.3, 0.0)
        ch.run(int(2.5 / eps), eps, True, 10, eps, 1.0, 2)
        ch.run(int(10.0 / eps), eps, True, 10, eps, 1.0, 2)
        m = ch.measure()
        ch.close()
        assert all(x["status"] == 0 for x in m)
        S = np.array([-beta * x["mean_L"] for x in m])
        est.append((S.mean(), S.real.std() / np.sqrt(len(S)), S.imag.std() / np.sqrt(len(S))))
    (s1, r1, i1), (s2, r2, i2) = est
    s0 = 2 * s2 - s1
    er, ei = np.hypot(2 * r2, r1), np.hypot(2 * i2, i1)
    assert abs(s0.real - exact.real) < 4 * er + 0.01, (s0, er, exact)
    assert abs(s0.imag - exact.imag) < 4 * ei + 0.01, (s0, ei, exact)


def test_cooling_of_gauge_rotated_chains_follows_the_paper(cl):
    """Section on the chain model, its cooling exercise (gauge-rotated unitary
    chains): with fixed alpha (D_0) d decays like t^(-3/2) on a chain of 1000
    links, a chain of 2 links cools to d = 0 exponentially (the slowing down
    sets in for longer chains), D_2 is far ahead of D_0 early on, and L is
    conserved throughout.  64 chains per case."""
    say("chain cooling d(t)")
    from tests.chainutil import gauge_rotated_chains

    def d_at(n, eps, mode, ts):
        links = gauge_rotated_chains(64, n, 3)
        ch = cl.Chain(n, 64, 1.0)
        ch.set_links(links)
        L0 = np.array([x["L"] for x in ch.measure()])
        out, t = [], 0
        for T in ts:
            ch.cool(T - t, eps, 1.0, mode)
            t = T
            m = ch.measure()
            assert all(x["status"] == 0 for x in m)
            out.append(np.mean([x["d"] for x in m]))
        assert np.max(np.abs(np.array([x["L"] for x in m]) - L0)) < 1e-10
        ch.close()
        return np.array(out)

    d0 = d_at(1000, 1e-2, 0, (1000, 10000))
    slope = np.log(d0[1] / d0[0]) / np.log(10.0)
    assert abs(slope + 1.5) < 0.1, (slope, d0)
    assert d_at(2, 1e-2, 0, (3000,))[0] < 1e-9
    early0 = d_at(1000, 1e-3, 0, (300,))[0]
    early2 = d_at(1000, 1e-3, 2, (300,))[0]
    assert early2 < early0 / 10, (early0, early2)
