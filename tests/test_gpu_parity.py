"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Per-step parity: one operation applied to identical input links must agree
to 1e-12 relative (max |dU| / max |U|) in FP64; drift, links, observables and
the control scalars (eps_n, alpha_ad, unitarity norm) are compared element by
element.  Whole trajectories are compared over the short 4^4 workload."""
import numpy as np
import pytest

from tests import latutil as lu
from tests.golden import fixture as gf

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def cl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_1056_amd as cl
    return cl


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8), (2, 2, 2, 2)])
def test_init_matches_oracle(cl, orc, dims):
    say("init", dims)
    lat = cl.Lattice(dims, 6.0, 0.0, cl.CL_FP64, seed=11)
    lat.init(True, 0.3, 0.05)
    U = lat.get_links()
    ref = orc.init_links(dims, 11, 0.3, 0.05)
    assert relerr(U, ref) < 1e-14
    assert abs(lat.unitarity_norm() - orc.distance(dims, ref)) < 1e-14
    lat.init(False)
    assert np.array_equal(lat.get_links(), orc.cold_links(dims))
    lat.close()


def test_set_get_roundtrip(cl):
    rng = np.random.default_rng(1)
    dims = (4, 2, 6, 4)
    U = lu.random_links(rng, dims)
    lat = cl.Lattice(dims, 6.0)
    lat.set_links(U)
    assert np.array_equal(lat.get_links(), U)
    lat.close()


@pytest.mark.parametrize("dims,theta", [((4, 4, 4, 4), 0.0), ((4, 4, 4, 4), 1.0), ((2, 4, 2, 6), 0.7 - 0.4j),
                                        ((2, 2, 2, 2), 2.0), ((6, 4, 4, 2), 1.0j)])
def test_drift_matches_oracle(cl, orc, dims, theta):
    say("drift", dims, theta)
    rng = np.random.default_rng(2)
    U = lu.random_links(rng, dims, 0.5, 0.2)
    lat = cl.Lattice(dims, 5.7, theta, cl.CL_FP64, seed=3)
    lat.set_links(U)
    K = lat.compute_drift()
    ref = orc.drift(dims, U, 5.7, theta)
    assert relerr(K, ref) < TOL
    if theta != 0:
        # the theta part alone, well above rounding of the Wilson part
        Kt = K - orc.drift(dims, U, 5.7, 0.0)
        Kt_ref = ref - orc.drift(dims, U, 5.7, 0.0)
        assert relerr(Kt, Kt_ref) < 1e-10
    lat.close()


@pytest.mark.parametrize("adaptive,theta", [(False, 0.0), (True, 0.0), (True, 1.0), (False, 2.0 + 0.5j)])
def test_langevin_step_matches_oracle(cl, orc, adaptive, theta):
    say("step", adaptive, theta)
    dims = (4, 4, 4, 4)
    U = orc.init_links(dims, 5, 0.3, 0.05)
    lat = cl.Lattice(dims, 6.0, theta, cl.CL_FP64, seed=5)
    lat.set_links(U)
    W = U.copy()
    bound = 0.0
    for n in range(3):
        eps = lat.langevin_step(1e-2, adaptive=adaptive)
        e_ref, k_ref, bound = orc.langevin_step(dims, W, 6.0, theta, 5, n, 1e-2, adaptive, bound=bound)
        assert abs(eps - e_ref) <= 1e-13 * e_ref
        obs = lat.measure()
        assert abs(obs["kmax"] - k_ref) <= 1e-12 * k_ref
        assert relerr(lat.get_links(), W) < TOL
        assert abs(obs["d_pre"] - orc.distance(dims, W)) < 1e-13
        # re-sync the input so every step is compared from identical links
        lat.set_links(W)
    lat.close()


@pytest.mark.parametrize("c3", [1.0 + 3e-5 - 4e-5j, 1.3 * np.exp(0.9j)])
def test_update_renormalises_any_determinant(cl, orc, c3):
    """Links whose determinant is c3 != 1 before the step: the update must
    still land on det U = 1 by the principal cube root, whether |det - 1| is
    inside the range of the kernel's short series (first case) or far
    outside it (second)."""
    say("renorm", c3)
    dims = (4, 4, 2, 4)
    U = orc.init_links(dims, 7, 0.3, 0.05)
    U = np.ascontiguousarray((U.view(np.complex128) * complex(c3) ** (1.0 / 3.0)).view(np.float64))
    lat = cl.Lattice(dims, 6.0, 0.5, cl.CL_FP64, seed=7)
    lat.set_links(U)
    W = U.copy()
    lat.langevin_step(1e-2, adaptive=False)
    orc.langevin_step(dims, W, 6.0, 0.5, 7, 0, 1e-2, False)
    got = lat.get_links()
    assert relerr(got, W) < TOL
    assert np.max(np.abs(np.linalg.det(got.view(np.complex128).reshape(-1, 3, 3)) - 1.0)) < 1e-13
    lat.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_gauge_cool_matches_oracle(cl, orc, mode):
    say("cool mode", mode)
    dims = (4, 4, 2, 6)
    rng = np.random.default_rng(4)
    U = lu.random_links(rng, dims, 0.5, 0.3)
    lat = cl.Lattice(dims, 6.0, 0.0, cl.CL_FP64)
    lat.set_links(U)
    d = lat.gauge_cool(7, 0.01, 1.0, mode)
    W = U.copy()
    un, al = orc.gauge_cool(dims, W, 7, 0.01, 1.0, mode)
    assert relerr(lat.get_links(), W) < TOL
    V = lu.volume(dims)
    assert abs(d - (un[-1] / (12 * V) - 1)) < 1e-13
    hu, ha = lat.cool_history()
    np.testing.assert_allclose(hu, un, rtol=1e-13)
    np.testing.assert_allclose(ha, al, rtol=1e-12)
    lat.close()


@pytest.mark.parametrize("theta", [0.0, 1.0, 0.3 + 0.8j])
def test_measure_matches_oracle(cl, orc, theta):
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(5)
    U = lu.random_links(rng, dims, 0.5, 0.2)
    lat = cl.Lattice(dims, 5.9, theta, cl.CL_FP64)
    lat.set_links(U)
    o = lat.measure()
    assert abs(o["plaq"] - orc.plaquette(dims, U)) < 1e-13
    q = orc.topological_charge(dims, U)
    assert abs(o["q"] - q) < 1e-12 * max(1, abs(q))
    s_ref = orc.wilson_action(dims, U, 5.9) - 1j * complex(theta) * q
    assert abs(o["action"] - s_ref) < 1e-12 * abs(s_ref)
    assert abs(o["d"] - orc.distance(dims, U)) < 1e-14
    lat.close()


def test_abelian_flux_on_gpu(cl):
    """Closed form: uniform abelian flux gives Q = V sin th12 sin th34 / (2 pi^2)."""
    dims = (4, 4, 4, 4)
    U, th12, th34 = lu.abelian_flux(dims, 1, 1)
    lat = cl.Lattice(dims, 6.0, 1.0)
    lat.set_links(U)
    o = lat.measure()
    assert abs(o["q"] - 256 / (2 * np.pi ** 2) * np.sin(th12) * np.sin(th34)) < 1e-12
    assert np.max(np.abs(lat.compute_drift())) < 1e-13
    lat.close()


def test_config1_trajectory(cl, orc):
    """4^4, beta 5.7, theta 0, seed 1, 20 steps eps 1e-3, 5 cooling steps alpha 1 (D0)
    after each: per-step d, plaquette and final links against the oracle."""
    dims, beta, seed = (4, 4, 4, 4), 5.7, 1
    lat = cl.Lattice(dims, beta, 0.0, cl.CL_FP64, seed)
    lat.init(True, 0.3, 0.05)
    W = orc.init_links(dims, seed, 0.3, 0.05)
    obs_ref, _ = orc.run(dims, W, beta, 0.0, seed, 20, 1e-3, False, 5, 1e-3, 1.0, 0)
    worst = 0.0
    for n in range(20):
        lat.langevin_step(1e-3, adaptive=False, sync=False)
        lat.gauge_cool(5, 1e-3, 1.0, 0, sync=False)
        o = lat.measure()
        assert abs(o["d_pre"] - obs_ref[n, 0]) < 1e-12
        assert abs(o["d"] - obs_ref[n, 1]) < 1e-12
        assert abs(o["plaq"] - complex(obs_ref[n, 2], obs_ref[n, 3])) < 1e-12
        worst = max(worst, abs(o["plaq"] - complex(obs_ref[n, 2], obs_ref[n, 3])))
    err = relerr(lat.get_links(), W)
    say(f"config1: final link rel err {err:.3e}, worst plaquette diff {worst:.3e}")
    assert err < 1e-11
    lat.close()


def test_config1_against_stored_values(cl):
    """The same 4^4 workload through the captured multi-step path
    (cl_run_steps), against the values tests/golden/ stores for it (written
    by the oracle), read from the device record of every step."""
    g = gf.read()
    lat = cl.Lattice(gf.DIMS, gf.BETA, gf.THETA, cl.CL_FP64, gf.SEED)
    lat.init(True, gf.SIGMA_X, gf.SIGMA_Y)
    lat.record_enable(True)
    lat.run_steps(gf.N_STEPS, gf.EPS, False, gf.N_COOL, gf.EPS_C, gf.ALPHA, gf.MODE)
    rec = lat.record_read(1, gf.N_STEPS)
    # record columns 1-4: d before and after the cooling steps, plaquette re and im
    worst = float(np.max(np.abs(rec[:, 1:5] - g["steps"][:, 1:5])))
    Uc = lu.to_c(lat.get_links())
    link_err = max(abs(Uc[s, mu, i, j] - z) for s, mu, i, j, z in g["links"])
    norm_err = abs(np.sum(np.abs(Uc) ** 2) - g["norm2"]) / g["norm2"]
    say(f"config1 stored: worst per-step diff {worst:.3e}, sampled link diff {link_err:.3e}, norm {norm_err:.3e}")
    assert worst < 1e-12
    assert link_err < 1e-11
    assert norm_err < 1e-12
    lat.close()
