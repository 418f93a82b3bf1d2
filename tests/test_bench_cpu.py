"""bench.py's command-line contract on the CPU: it measures one GPU only and
refuses more, with a message, before touching any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_distributed_launch_is_refused():
    r = run([], {"WORLD_SIZE": "2", "RANK": "0", "LOCAL_RANK": "0"})
    assert r.returncode == 2
    assert "WORLD_SIZE=2" in r.stderr


def test_cost_model_and_step_roofline():
    """The byte and flop model the roofline entries use: the sweep floor is one
    read and one write of the link field; the cooling pair moves the field
    three times plus the staged transforms (Omega alone in FP64, both
    Omega - 1 and Omega^-1 - 1 in FP32); the step roofline divides (1 + n_c)
    floors by the step time; counter traffic is only used on a matching
    kernel source."""
    sys.path.insert(0, ROOT)
    import bench
    V = 16 ** 4
    for rs, staged in ((8, 9), (4, 18)):
        field = 4 * V * 18 * rs
        assert bench.floor_bytes("cool_apply", V, rs) == 2 * field
        assert bench.floor_bytes("cool_omega", V, rs) == 0
        om = bench.algorithmic_cost("cool_omega", V, rs, 1.0)["bytes"]
        ap = bench.algorithmic_cost("cool_apply", V, rs, 1.0)["bytes"]
        assert om == field + (V // 2) * staged * rs
        assert ap == 2 * field + (V // 2) * staged * rs
        assert bench.algorithmic_cost("update", V, rs, 1.0)["bytes"] == 3 * field
    res = {"V": V, "ms_per_step": 0.5}
    sr = bench.step_roofline(res, "fp64", 1.0, 10)
    assert sr["floor_bytes_per_step"] == 11 * 4 * V * 2 * 18 * 8
    assert abs(sr["frac_hbm"] - sr["floor_bytes_per_step"] / 0.5e-3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    assert sr["binding_roof"] in ("hbm", "valu")
    # no dims: no counter figures
    assert sr["traffic_bytes_per_step"] is None
    # a lattice without counter runs has none either
    assert bench.measured_step_traffic("fp64", (6, 6, 6, 6), 1.0, 10, 1e-3)["traffic_GBs"] is None
