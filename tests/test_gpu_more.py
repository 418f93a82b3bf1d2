"""GPU tests beyond single-operation parity: graph replay vs eager launches,
the mixed-precision path's tolerances, the 16^4 production size, larger
lattices on sampled links, error and runaway handling, determinism and
checkpoint/resume.  All calls go through the C ABI."""
import ctypes

import numpy as np
import pytest

from tests import latutil as lu

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n_steps", [2, 11])
def test_graph_replay_matches_eager(cl, n_steps):
    """cl_run_steps replays captured graphs (blocks of 8 steps, then single
    steps); it must give exactly what individual launches give, replay after
    replay."""
    dims = (4, 4, 4, 8)
    a = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=9)
    b = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=9)
    a.init(True)
    b.init(True)
    for rep in range(3):
        a.run_steps(n_steps, 1e-2, True, 3, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
        ma = a.measure()  # eager work and a synchronisation between replays
        for _ in range(n_steps):
            b.langevin_step(1e-2, adaptive=True, sync=False)
            b.gauge_cool(3, 1e-2, 1.0, cl.CL_ALPHA_UNORM, sync=False)
        mb = b.measure()
        assert np.array_equal(a.get_links(), b.get_links()), rep
        assert ma == mb
    a.close()
    b.close()


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_mixed_precision_step_tolerance(cl, orc, theta):
    """Mixed path (FP32 links, drift, cooling; FP64 det renormalisation,
    reductions and control) against the FP64 oracle from the same links and
    noise: link error <= 1e-5 relative, observables within 1e-6."""
    dims = (8, 8, 8, 8)
    U = orc.init_links(dims, 4, 0.3, 0.05)
    lat = cl.Lattice(dims, 6.0, theta, cl.CL_MIXED, seed=4)
    lat.set_links(U)
    Uin = lat.get_links()  # the FP32-rounded input both sides start from
    W = Uin.copy()
    bound = 0.0
    worst = 0.0
    for n in range(2):
        eps = lat.langevin_step(1e-2, adaptive=True)
        e_ref, _, bound = orc.langevin_step(dims, W, 6.0, theta, 4, n, 1e-2, True, bound=bound)
        assert abs(eps - e_ref) <= 1e-5 * e_ref
        lat.gauge_cool(10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
        orc.gauge_cool(dims, W, 10, 1e-2, 1.0, 1)
        got = lat.get_links()
        err = relerr(got, W)
        worst = max(worst, err)
        assert err <= 1e-5
        o = lat.measure()
        assert abs(o["plaq"] - orc.plaquette(dims, W)) <= 1e-6
        q = orc.topological_charge(dims, W)
        assert abs(o["q"] - q) <= 1e-6 * max(1, abs(q))
        assert abs(o["d"] - orc.distance(dims, W)) <= 1e-6
        lat.set_links(W)  # restart the next step from identical (rounded) links
        W = lat.get_links()
    say(f"mixed theta={theta}: worst per-step link error {worst:.2e}")
    lat.close()


@pytest.mark.parametrize("theta", [1.0, 0.6 - 0.8j])
def test_mixed_drift_tolerance(cl, orc, theta):
    """The FP32 drift (real and complex theta: the walk scales the charge
    insertions by a real factor in the first case) against the oracle."""
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(7)
    U = lu.random_links(rng, dims, 0.5, 0.2)
    lat = cl.Lattice(dims, 6.0, theta, cl.CL_MIXED)
    lat.set_links(U)
    Ur = lat.get_links()
    K = lat.compute_drift()
    err = relerr(K, orc.drift(dims, Ur, 6.0, theta))
    say(f"mixed drift theta={theta}: rel err {err:.2e}")
    assert err < 1e-5
    lat.close()


@pytest.mark.slow
def test_production_size_16x4_full_step(cl, orc):
    """The benchmark's workload and launch configuration: 16^4, beta 6, theta 1,
    adaptive eps, 10 D_1 cooling steps; one full step compared link by link."""
    dims = (16, 16, 16, 16)
    lat = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=3)
    lat.init(True, 0.3, 0.05)
    U0 = lat.get_links()
    lat.run_steps(1, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    got = lat.get_links()
    o = lat.measure()
    W = U0.copy()
    obs, bound = orc.run(dims, W, 6.0, 1.0, 3, 1, 1e-2, True, 10, 1e-2, 1.0, 1)
    err = relerr(got, W)
    say(f"16^4 full step: link rel err {err:.2e}")
    assert err < 1e-12
    assert abs(o["plaq"] - complex(obs[0, 2], obs[0, 3])) < 1e-12
    assert abs(o["q"] - complex(obs[0, 4], obs[0, 5])) < 1e-11
    assert abs(o["d"] - obs[0, 1]) < 1e-13
    assert abs(o["eps"] - obs[0, 6]) < 1e-14
    lat.close()


@pytest.mark.slow
def test_production_size_16x4_full_step_mixed(cl, orc):
    """The mixed-precision leg of the benchmark in its launch configuration
    (16^4, beta 6, theta 1, adaptive eps, 10 D_1 cooling steps, the captured
    step graph) against the FP64 oracle from the same FP32-rounded links:
    links within 1e-5 relative, observables within 1e-6."""
    dims = (16, 16, 16, 16)
    lat = cl.Lattice(dims, 6.0, 1.0, cl.CL_MIXED, seed=3)
    lat.init(True, 0.3, 0.05)
    U0 = lat.get_links()
    lat.run_steps(1, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    got = lat.get_links()
    o = lat.measure()
    W = U0.copy()
    obs, _ = orc.run(dims, W, 6.0, 1.0, 3, 1, 1e-2, True, 10, 1e-2, 1.0, 1)
    err = relerr(got, W)
    q = complex(obs[0, 4], obs[0, 5])
    say(f"16^4 mixed full step: link rel err {err:.2e}, |dP| {abs(o['plaq'] - complex(obs[0, 2], obs[0, 3])):.2e}, "
        f"|dQ| {abs(o['q'] - q):.2e} (|Q| {abs(q):.2f}), |dd| {abs(o['d'] - obs[0, 1]):.2e}")
    assert err <= 1e-5
    assert abs(o["plaq"] - complex(obs[0, 2], obs[0, 3])) <= 1e-6
    assert abs(o["q"] - q) <= 1e-6 * max(1.0, abs(q))
    assert abs(o["d"] - obs[0, 1]) <= 1e-6
    assert abs(o["eps"] - obs[0, 6]) <= 1e-5 * obs[0, 6]
    lat.close()


@pytest.mark.slow
@pytest.mark.parametrize("dims,precs", [((24, 24, 24, 24), (1, 0)), ((32, 32, 32, 32), (1,)),
                                        ((46, 46, 46, 46), (0,)), ((56, 56, 56, 56), (1,))])
def test_large_lattice_sampled_drift(cl, orc, dims, precs):
    """24^4, 32^4 and the largest lattices the buffer resources address (46^4
    FP64, 56^4 mixed): the drift of sampled links (the first and the last
    among them) against the oracle, which evaluates each sampled link on its
    own."""
    rng = np.random.default_rng(8)
    V = lu.volume(dims)
    sel = np.sort(rng.choice(4 * V, size=48, replace=False))
    sel = np.concatenate([sel, [0, 4 * V - 1]])
    for prec in precs:
        lat = cl.Lattice(dims, 6.0, 1.0, prec, seed=4)
        lat.init(True, 0.3, 0.05)
        U = lat.get_links()
        K = lat.compute_drift().reshape(-1, 18)[sel]
        ref = orc.drift_links(dims, U, 6.0, 1.0, sel)
        tol = 1e-12 if prec == cl.CL_FP64 else 1e-5
        err = relerr(K, ref)
        say(f"{dims} prec={prec}: sampled drift rel err {err:.2e}")
        assert err < tol
        if dims[0] >= 46:
            # a full step with cooling at the largest size (the prefetching
            # cooling kernels at their largest chunk count): finite, advanced,
            # and the cooling lowers the distance
            lat.run_steps(1, 1e-2, True, 2, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
            o = lat.measure()
            assert o["step"] == 1 and np.isfinite(o["d"]) and 0 < o["d"] <= o["d_pre"], o
        lat.close()


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(24, 24, 24, 24), (32, 32, 32, 32)])
def test_large_lattice_mixed_against_fp64_step(cl, dims):
    """24^4 and 32^4, theta 1, seed 4: one CL step (adaptive eps) and 10 D_1
    cooling steps on the mixed and the FP64 path from identical links and the
    same Philox words.  Per-step link error <= 1e-5 relative; plaquette, Q and
    d within 1e-6 of max(1, |value|).  The FP64 path is the one pinned to the
    oracle at smaller sizes and on sampled links here.  The observable error
    is split into the part the FP32 links carry (the mixed links measured on
    an FP64 lattice against the FP64 run) and the part the mixed measurement
    adds (the mixed lattice's own measurement against that FP64 measurement of
    the same links)."""
    mx = cl.Lattice(dims, 6.0, 1.0, cl.CL_MIXED, seed=4)
    mx.init(True, 0.3, 0.05)
    U = mx.get_links()  # FP32-representable: both paths start from these
    fp = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=4)
    fp.set_links(U)
    del U
    for lat in (mx, fp):
        lat.run_steps(1, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    a, b = mx.measure(), fp.measure()
    Um = mx.get_links()
    err = relerr(Um, fp.get_links())
    say(f"{dims}: mixed vs FP64 one step, link rel err {err:.2e}, eps {a['eps']:.6e} / {b['eps']:.6e}")
    assert err <= 1e-5
    assert abs(a["eps"] - b["eps"]) <= 1e-5 * b["eps"]
    fp.set_links(Um)  # the mixed links, measured in FP64
    del Um
    c = fp.measure()
    for k in ("plaq", "q", "d"):
        links_part = abs(c[k] - b[k]) / max(1.0, abs(b[k]))
        meas_part = abs(a[k] - c[k]) / max(1.0, abs(b[k]))
        say(f"  {k}: total {abs(a[k] - b[k]) / max(1.0, abs(b[k])):.2e} = links {links_part:.2e} "
            f"+ measurement {meas_part:.2e}")
        assert abs(a[k] - b[k]) <= 1e-6 * max(1.0, abs(b[k])), (k, a[k], b[k])
        # the mixed lattice measures in FP64 from its FP32 links
        assert meas_part <= 1e-12, k
    mx.close()
    fp.close()


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(24, 24, 24, 24), (32, 32, 32, 32)])
def test_large_lattice_full_step_against_oracle(cl, orc, dims):
    """The mixed-precision workload's sizes, 24^4 and 32^4 (theta 1, seed 4,
    adaptive eps, 10 D_1 cooling steps), one whole step in the captured launch
    configuration against the oracle stepping the same links: the FP64 path
    at 1e-12, the mixed path at its stated bounds (links 1e-5 relative; P, Q
    and d within 1e-6 of max(1, |value|))."""
    mx = cl.Lattice(dims, 6.0, 1.0, cl.CL_MIXED, seed=4)
    mx.init(True, 0.3, 0.05)
    W = mx.get_links()  # FP32-representable: every side starts from these
    fp = cl.Lattice(dims, 6.0, 1.0, cl.CL_FP64, seed=4)
    fp.set_links(W)
    for lat in (mx, fp):
        lat.run_steps(1, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    a, b = mx.measure(), fp.measure()
    obs, _ = orc.run(dims, W, 6.0, 1.0, 4, 1, 1e-2, True, 10, 1e-2, 1.0, 1)
    ref = {"plaq": complex(obs[0, 2], obs[0, 3]), "q": complex(obs[0, 4], obs[0, 5]), "d": obs[0, 1],
           "eps": obs[0, 6]}
    ef = relerr(fp.get_links(), W)
    em = relerr(mx.get_links(), W)
    say(f"{dims}: FP64 link rel err {ef:.2e}, mixed {em:.2e}; |Q| {abs(ref['q']):.2f}")
    assert ef < 1e-12
    assert em <= 1e-5
    assert abs(b["eps"] - ref["eps"]) <= 1e-13 * ref["eps"]
    assert abs(a["eps"] - ref["eps"]) <= 1e-5 * ref["eps"]
    for k in ("plaq", "q", "d"):
        scale = max(1.0, abs(ref[k]))
        say(f"  {k}: FP64 {abs(b[k] - ref[k]) / scale:.2e}, mixed {abs(a[k] - ref[k]) / scale:.2e}")
        assert abs(b[k] - ref[k]) <= 1e-11 * scale, k
        assert abs(a[k] - ref[k]) <= 1e-6 * scale, k
    mx.close()
    fp.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_minimum_and_ragged_lattices(cl, orc, prec):
    """2^4 (every neighbour wraps) and extents with a ragged last block (a
    cooling chunk of 64 sites with idle lanes in its LDS exchange), FP64 at
    1e-12 and mixed precision at its per-step 1e-5."""
    for dims in [(2, 2, 2, 2), (2, 6, 4, 10), (6, 2, 2, 2), (4, 2, 6, 6)]:
        say("ragged", dims, prec)
        lat = cl.Lattice(dims, 5.5, 0.8, prec, seed=2)
        lat.init(True)
        U = lat.get_links()
        lat.langevin_step(5e-3)
        lat.gauge_cool(3, 5e-3, 1.0, cl.CL_ALPHA_GRAD)
        W = U.copy()
        orc.langevin_step(dims, W, 5.5, 0.8, 2, 0, 5e-3)
        orc.gauge_cool(dims, W, 3, 5e-3, 1.0, 2)
        assert relerr(lat.get_links(), W) < (1e-12 if prec == 0 else 1e-5), dims
        lat.close()


def test_zero_step_and_zero_cooling_calls(cl, orc):
    """Degenerate calls: zero CL steps and zero cooling steps change nothing;
    CL steps without cooling, replayed from the captured graphs (a block of
    eight steps and one more: the norm is then finalized every step, and with
    the theta term in FP64 the record is taken inside the step), follow the
    oracle at 1e-12."""
    dims, beta, theta, seed = (4, 4, 4, 6), 5.9, 0.7, 6
    lat = cl.Lattice(dims, beta, theta, cl.CL_FP64, seed)
    lat.init(True, 0.3, 0.05)
    U0 = lat.get_links()
    o0 = lat.measure()
    lat.run_steps(0, 1e-2, True, 5, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    d = lat.gauge_cool(0, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    assert np.array_equal(lat.get_links(), U0)
    o1 = lat.measure()
    assert o1["step"] == o0["step"] == 0
    assert o1["plaq"] == o0["plaq"] and o1["q"] == o0["q"]
    assert abs(d - o0["d"]) <= 1e-12 * o0["d"]
    lat.record_enable(True)
    lat.run_steps(9, 1e-2, True, 0, 1e-2, 1.0, cl.CL_ALPHA_FIXED)
    rec = lat.record_read(1, 9)
    W = U0.copy()
    obs, _ = orc.run(dims, W, beta, theta, seed, 9, 1e-2, True, 0, 1e-2, 1.0, 0)
    err = relerr(lat.get_links(), W)
    say(f"9 CL steps without cooling: link rel err {err:.2e}")
    assert err < 1e-12
    assert np.array_equal(rec[:, 0], np.arange(1, 10))
    # record columns against the oracle's: d before and after the (empty)
    # cooling, P re/im, Q re/im, eps, K_max
    for rc, oc in ((1, 0), (2, 1), (3, 2), (4, 3), (5, 4), (6, 5), (9, 6), (10, 7)):
        ref = obs[:, oc]
        scale = np.abs(ref) if rc in (1, 2, 9, 10) else np.maximum(np.abs(ref), 1.0)
        assert np.all(np.abs(rec[:, rc] - ref) <= 1e-12 * scale), (rc, rec[:, rc], ref)
    # without cooling d before and after it are one value, formed here by two
    # different reductions (the update's norm partials, the record's own sum)
    assert np.all(np.abs(rec[:, 1] - rec[:, 2]) <= 1e-13 * rec[:, 2])
    lat.close()


def test_errors(cl):
    with pytest.raises(cl.ClError) as e:
        cl.Lattice((3, 4, 4, 4), 6.0)
    assert e.value.status == cl.CL_EINVAL
    import torch
    desc = cl.make_desc((4, 4, 4, 4), 6.0)
    need = cl.cl_lattice_bytes(desc)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    h = ctypes.c_void_p()
    st = cl.lib.cl_lattice_create(ctypes.byref(desc), ctypes.c_void_p(buf.data_ptr()), need - 256, None,
                                  ctypes.byref(h))
    assert st == cl.CL_ENOMEM
    lat = cl.Lattice((4, 4, 4, 4), 6.0)
    with pytest.raises(cl.ClError) as e:
        lat.set_links(np.zeros(10))
    assert e.value.status == cl.CL_EINVAL
    with pytest.raises(cl.ClError):
        lat.langevin_step(-1.0)
    with pytest.raises(cl.ClError):
        lat.gauge_cool(100, 1e-2)
    lat.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_cooling_overflow_is_flagged_and_ends(cl, orc, prec):
    """Fixed-alpha cooling with a large eps_c alpha on a strongly gauge-rotated
    start overflows the links: the call must end promptly with CL_ENONFINITE
    (regression: an infinite norm once turned the Hermitian exponential's
    scaling count into 2^31 squarings), and the same start cools under D_1."""
    dims = (4, 4, 4, 4)
    U = orc.cold_links(dims)
    orc.gauge_transform(dims, U, lu.random_sl3c(np.random.default_rng(5), 0.6, 0.4, n=lu.volume(dims)))
    say("cooling overflow", dims, prec)
    lat = cl.Lattice(dims, 6.0, 0.0, prec)
    lat.set_links(U)
    with pytest.raises(cl.ClError) as e:
        for _ in range(10):
            lat.gauge_cool(20, 0.5, 1.0, cl.CL_ALPHA_FIXED)
    assert e.value.status == cl.CL_ENONFINITE
    lat.close()
    lat = cl.Lattice(dims, 6.0, 0.0, prec)
    lat.set_links(U)
    d0 = lat.unitarity_norm()
    d = lat.gauge_cool(60, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    assert np.isfinite(d) and d < 1e-3 * d0
    lat.close()


def test_runaway_is_detected_and_not_advanced(cl, orc):
    """A non-finite link makes the drift non-finite: the step reports
    CL_ENONFINITE and leaves the links as they were."""
    dims = (4, 4, 4, 4)
    U = orc.init_links(dims, 1)
    U[17, 2, 4] = np.nan
    lat = cl.Lattice(dims, 6.0, 1.0)
    lat.set_links(U)
    with pytest.raises(cl.ClError) as e:
        lat.langevin_step(1e-2, adaptive=True)
    assert e.value.status == cl.CL_ENONFINITE
    got = lat.get_links()
    assert np.array_equal(np.isnan(got), np.isnan(U))
    assert np.array_equal(got[~np.isnan(U)], U[~np.isnan(U)])
    # a healthy lattice next to it is unaffected
    ok = cl.Lattice(dims, 6.0, 1.0)
    ok.init(True)
    assert ok.langevin_step(1e-2) == 1e-2
    ok.close()
    lat.close()


def test_determinism_and_resume(cl):
    dims = (4, 4, 8, 4)
    kw = dict(eps0=1e-2, adaptive=True, n_cool=4, eps_c=1e-2, alpha=1.0, mode=cl.CL_ALPHA_UNORM)
    a = cl.Lattice(dims, 6.0, 0.5, cl.CL_FP64, seed=21)
    b = cl.Lattice(dims, 6.0, 0.5, cl.CL_FP64, seed=21)
    a.init(True)
    b.init(True)
    a.run_steps(4, **kw)
    b.run_steps(2, **kw)
    step, bound = b.get_state()
    links = b.get_links()
    b.close()
    assert step == 2 and bound > 0
    c = cl.Lattice(dims, 6.0, 0.5, cl.CL_FP64, seed=21)
    c.set_links(links)
    c.set_state(step, bound)
    c.run_steps(2, **kw)
    assert np.array_equal(a.get_links(), c.get_links())
    d = cl.Lattice(dims, 6.0, 0.5, cl.CL_FP64, seed=21)
    d.init(True)
    d.run_steps(4, **kw)
    assert np.array_equal(a.get_links(), d.get_links())
    for x in (a, c, d):
        x.close()


def test_config2_shape_trajectory(cl, orc):
    """8^4, beta 6, seed 2, adaptive eps (eps0 1e-2), 10 adaptive-alpha cooling
    steps: per-step eps, distances and plaquette over a short trajectory."""
    dims = (8, 8, 8, 8)
    lat = cl.Lattice(dims, 6.0, 0.0, cl.CL_FP64, seed=2)
    lat.init(True)
    W = orc.init_links(dims, 2)
    obs, _ = orc.run(dims, W, 6.0, 0.0, 2, 4, 1e-2, True, 10, 1e-2, 1.0, 1)
    for n in range(4):
        lat.run_steps(1, 1e-2, True, 10, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
        o = lat.measure()
        assert abs(o["eps"] - obs[n, 6]) < 1e-12 * obs[n, 6]
        assert abs(o["d_pre"] - obs[n, 0]) < 1e-12
        assert abs(o["d"] - obs[n, 1]) < 1e-12
        assert abs(o["plaq"] - complex(obs[n, 2], obs[n, 3])) < 1e-12
    assert relerr(lat.get_links(), W) < 1e-11
    lat.close()


def test_real_langevin_and_cooling_invariants(cl):
    """theta = 0 from an SU(3) start keeps links unitary (cooling is then a
    no-op); on a complex configuration cooling lowers the norm monotonically
    and leaves the plaquette and Q unchanged."""
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(3)
    S = lu.from_c(lu.random_su3(rng, n=lu.volume(dims) * 4)).reshape(-1, 4, 18)
    lat = cl.Lattice(dims, 6.0, 0.0)
    lat.set_links(S)
    for _ in range(5):
        lat.langevin_step(1e-2)
    assert abs(lat.unitarity_norm()) < 1e-13
    lat.close()
    U = lu.random_links(rng, dims, 0.5, 0.3)
    lat = cl.Lattice(dims, 6.0, 1.0)
    lat.set_links(U)
    o0 = lat.measure()
    lat.gauge_cool(20, 1e-2, 1.0, cl.CL_ALPHA_UNORM)
    o1 = lat.measure()
    hu, _ = lat.cool_history()
    assert np.all(np.diff(hu) <= 0)
    assert abs(o1["plaq"] - o0["plaq"]) < 1e-13
    assert abs(o1["q"] - o0["q"]) < 1e-12
    assert o1["d"] < o0["d"]
    lat.close()


@pytest.mark.parametrize("dims,mode", [((24, 24, 24, 16), 2), ((18, 18, 18, 22), 1), ((18, 18, 18, 22), 0)])
def test_d2_cooling_with_chunked_gradient_pass(cl, orc, dims, mode):
    """Cooling on lattices with more chunks of sites than cooling blocks (24^3 x
    16: 1728 over 512; 18^3 x 22: 1003, the last one ragged), so every block
    loops and the prefetching cooling kernels run; with D_2 the gradient-norm
    pass loops too and the next omega kernel's wavefronts sum its partials.
    Links and the alpha / norm history against the oracle (oracle start, not
    the GPU's)."""
    say("chunked cooling", dims, mode)
    U = orc.init_links(dims, 7, 0.3, 0.1)
    lat = cl.Lattice(dims, 6.0, 0.0, cl.CL_FP64)
    lat.set_links(U)
    lat.gauge_cool(2, 1e-2, 1.0, mode)
    W = U.copy()
    un, al = orc.gauge_cool(dims, W, 2, 1e-2, 1.0, mode)
    assert relerr(lat.get_links(), W) < 1e-12
    hu, ha = lat.cool_history()
    np.testing.assert_allclose(hu, un, rtol=1e-13)
    np.testing.assert_allclose(ha, al, rtol=1e-12)
    lat.close()
