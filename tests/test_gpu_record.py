"""The per-step record of cl_run_steps against the oracle stepped by hand.

Each CL step's entry (d before and after cooling, plaquette, Q, action, eps,
Kmax, alpha_ad) is measured on the device without host synchronisation and
read back afterwards; the oracle runs the same steps one call at a time and
measures after each.  Whole short trajectories: the paper's results are
series in Langevin time (the running <Q_L>, the distance d along the
trajectory)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_1056_amd as cl
    return cl


def say(*a):
    print(*a, flush=True)


def oracle_series(orc, dims, W, beta, theta, seed, n_steps, eps0, adaptive, n_cool, eps_c, alpha, mode):
    """Per-step (12-field) series of the oracle, in place on W."""
    V = int(np.prod(dims))
    out = np.zeros((n_steps, 12))
    bound = 0.0
    th = complex(theta)
    for n in range(n_steps):
        eps, kmax, bound = orc.langevin_step(dims, W, beta, theta, seed, n, eps0, adaptive, bound=bound)
        d_pre = orc.distance(dims, W)
        un, al = orc.gauge_cool(dims, W, n_cool, eps_c, alpha, mode)
        P = orc.plaquette(dims, W)
        Q = orc.topological_charge(dims, W)
        S = orc.wilson_action(dims, W, beta) - 1j * th * Q
        d = un[-1] / (12.0 * V) - 1.0 if n_cool > 0 else orc.distance(dims, W)
        out[n] = [n + 1, d_pre, d, P.real, P.imag, Q.real, Q.imag, S.real, S.imag, eps, kmax,
                  al[-1] if n_cool > 0 else np.nan]
    return out


CASES = [
    # 4^4 workload: beta 5.7, theta 0, seed 1, 20 steps, fixed eps 1e-3, 5 D_0 cooling steps
    dict(dims=(4, 4, 4, 4), beta=5.7, theta=0.0, seed=1, n=20, eps0=1e-3, adaptive=False, nc=5, eps_c=1e-3,
         mode=0, calls=(20,)),
    # 8^4 workload: beta 6, seed 2, adaptive eps0 1e-2, 10 D_1 steps; four steps in three calls
    dict(dims=(8, 8, 8, 8), beta=6.0, theta=0.0, seed=2, n=4, eps0=1e-2, adaptive=True, nc=10, eps_c=1e-2,
         mode=1, calls=(1, 2, 1)),
    # theta term (the FP64 measurement reads the clover field of the next step's drift), D_2,
    # a graph block of eight steps and one more
    dict(dims=(4, 4, 2, 6), beta=6.0, theta=1.0, seed=3, n=9, eps0=5e-3, adaptive=True, nc=3, eps_c=5e-3,
         mode=2, calls=(9,)),
    # complex theta
    dict(dims=(2, 4, 4, 4), beta=5.9, theta=0.6 - 0.8j, seed=5, n=3, eps0=5e-3, adaptive=True, nc=2, eps_c=5e-3,
         mode=1, calls=(3,)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{'x'.join(map(str, c['dims']))}_th{c['theta']}" for c in CASES])
def test_record_matches_oracle_series(cl, orc, case):
    c = case
    say("record", c["dims"], c["theta"])
    lat = cl.Lattice(c["dims"], c["beta"], c["theta"], cl.CL_FP64, seed=c["seed"])
    lat.init(True, 0.3, 0.05)
    W = lat.get_links()
    lat.record_enable(True)
    for k in c["calls"]:
        lat.run_steps(k, c["eps0"], c["adaptive"], c["nc"], c["eps_c"], 1.0, c["mode"])
    got = lat.record_read(1, c["n"])
    ref = oracle_series(orc, c["dims"], W, c["beta"], c["theta"], c["seed"], c["n"], c["eps0"], c["adaptive"],
                        c["nc"], c["eps_c"], 1.0, c["mode"])
    assert np.array_equal(got[:, 0], np.arange(1, c["n"] + 1))
    # P, Q and S per unit volume are O(1); d, eps, Kmax, alpha relative
    scale = np.maximum(np.abs(ref), 1.0)
    scale[:, [1, 2, 9, 10, 11]] = np.abs(ref[:, [1, 2, 9, 10, 11]])
    scale[:, [7, 8]] = np.maximum(np.abs(ref[:, [7, 8]]), float(np.prod(c["dims"])))
    err = np.abs(got - ref) / scale
    worst = float(np.nanmax(err[:, 1:]))
    say(f"  worst relative error over {c['n']} steps: {worst:.2e}")
    assert worst < 1e-12, np.nanmax(err, axis=0)
    # the entry of the last step equals a synchronous measurement of the final links
    o = lat.measure()
    assert abs(got[-1, 3] + 1j * got[-1, 4] - o["plaq"]) < 1e-14
    assert abs(got[-1, 5] + 1j * got[-1, 6] - o["q"]) < 1e-12
    lat.close()


def test_record_after_a_measurement(cl, orc):
    """FP64 with a theta term records inside the step (the clover kernel's
    plaquette traces and link norms, a charge pass over its field): after a
    cl_measure the clover field is already valid, and the recorded step must
    still rebuild it with its record partials.  Two calls, a measurement
    before each."""
    dims, beta, theta, seed = (4, 2, 4, 6), 5.8, 1.3, 9
    lat = cl.Lattice(dims, beta, theta, cl.CL_FP64, seed=seed)
    lat.init(True, 0.3, 0.05)
    W = lat.get_links()
    lat.record_enable(True)
    lat.measure()
    lat.run_steps(3, 5e-3, True, 4, 5e-3, 1.0, cl.CL_ALPHA_UNORM)
    lat.measure()
    lat.run_steps(2, 5e-3, True, 4, 5e-3, 1.0, cl.CL_ALPHA_UNORM)
    got = lat.record_read(1, 5)
    ref = oracle_series(orc, dims, W, beta, theta, seed, 5, 5e-3, True, 4, 5e-3, 1.0, 1)
    scale = np.maximum(np.abs(ref), 1.0)
    scale[:, [1, 2, 9, 10, 11]] = np.abs(ref[:, [1, 2, 9, 10, 11]])
    scale[:, [7, 8]] = np.maximum(np.abs(ref[:, [7, 8]]), float(np.prod(dims)))
    worst = float(np.nanmax(np.abs(got - ref)[:, 1:] / scale[:, 1:]))
    say(f"record after measurements: worst relative error {worst:.2e}")
    assert worst < 1e-12
    lat.close()


def test_record_mixed_against_fp64(cl):
    """Mixed precision records in FP64 from its FP32 links: its series stays
    within the mixed tolerances of the FP64 series (same start, same noise)."""
    dims = (8, 8, 8, 8)
    mx = cl.Lattice(dims, 6.0, 1.0, cl.CL_MIXED, seed=4)
    mx.init(True, 0.3, 0.05)
    U = mx.get_links()
    fp = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=4)
    fp.set_links(U)
    recs = []
    for lat in (mx, fp):
        lat.record_enable(True)
        lat.run_steps(3, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
        recs.append(lat.record_read(1, 3))
        lat.close()
    a, b = recs
    err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    say("mixed vs FP64 record, d / P / Q error per step:", err[:, [2, 3, 5]].tolist())
    # the first step starts from identical links: the per-step bound; later
    # steps start from links that already differ (reported, not gated)
    for col in (2, 3, 4, 5, 6):
        assert err[0, col] < 1e-6, col


def test_record_range_errors(cl):
    lat = cl.Lattice((4, 4, 4, 4), 6.0, 0.0, cl.CL_FP64, seed=1)
    lat.init(True)
    lat.record_enable(True)
    lat.run_steps(2, 1e-3, False, 1, 1e-3)
    assert lat.record_read(1, 2).shape == (2, 12)
    for first, n in ((0, 1), (2, 2), (3, 1)):
        with pytest.raises(cl.ClError) as e:
            lat.record_read(first, n)
        assert e.value.status == cl.CL_EINVAL
    # recording off: no new entries, the counter still advances
    lat.record_enable(False)
    lat.run_steps(1, 1e-3, False, 1, 1e-3)
    with pytest.raises(cl.ClError):
        lat.record_read(3, 1)
    lat.close()
