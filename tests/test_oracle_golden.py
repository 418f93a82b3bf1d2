"""The stored 4^4 workload of tests/golden/ (written by the oracle: the paper
prints no numerical example): the oracle still reproduces it, and the stored
values are consistent with what the paper fixes about them."""
import numpy as np

from tests.golden import fixture as gf


def test_oracle_reproduces_stored_values(orc):
    g = gf.read()
    U = orc.init_links(gf.DIMS, gf.SEED, gf.SIGMA_X, gf.SIGMA_Y)
    obs, _ = orc.run(gf.DIMS, U, gf.BETA, gf.THETA, gf.SEED, gf.N_STEPS, gf.EPS, False, gf.N_COOL,
                     gf.EPS_C, gf.ALPHA, gf.MODE)
    assert g["steps"].shape == (gf.N_STEPS, 5)
    np.testing.assert_array_equal(g["steps"][:, 0], np.arange(gf.N_STEPS))
    np.testing.assert_allclose(obs[:, :4], g["steps"][:, 1:], rtol=1e-13, atol=1e-16)
    Uc = orc.to_complex(U)
    assert abs(np.sum(np.abs(Uc) ** 2) - g["norm2"]) <= 1e-13 * g["norm2"]
    for s, mu, i, j, z in g["links"]:
        assert abs(Uc[s, mu, i, j] - z) <= 1e-13


def test_stored_values_are_consistent():
    g = gf.read()
    st = g["steps"]
    V = int(np.prod(gf.DIMS))
    # eq. (d): d = (1/3) Tr(U U^dagger) - 1 averaged over links, so the stored
    # norm of the final links fixes the last d
    assert abs(g["norm2"] / (3 * 4 * V) - 1.0 - st[-1, 2]) < 1e-14
    # d >= 0 on SL(3,C), and cooling at small alpha_gf lowers it
    assert np.all(st[:, 1:3] > 0.0)
    assert np.all(st[:, 2] < st[:, 1])
