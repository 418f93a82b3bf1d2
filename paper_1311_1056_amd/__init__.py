"""Complex Langevin + adaptive gauge cooling for SU(3) with a theta term on
MI355X (gfx950).

Thin ctypes binding of the C ABI in include/clgc.h: argument marshalling
only.  Every step of the method runs in the HIP kernels of libclgc.so;
PyTorch only provides device memory and the stream.  If the library is not
built this module raises on import -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: the library then binds to the HIP runtime torch already loaded
# (both export the soname libamdhip64.so.7), so the process has one runtime
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclgc.so")

CL_OK, CL_EINVAL, CL_ENOMEM, CL_EHIP, CL_ENONFINITE, CL_EBUDGET = 0, -1, -2, -3, -4, -5
CL_FP64, CL_MIXED = 0, 1
CL_ALPHA_FIXED, CL_ALPHA_UNORM, CL_ALPHA_GRAD = 0, 1, 2
# fields of one per-step record entry (cl_record_read)
RECORD_FIELDS = ("step", "d_pre", "d", "plaq_re", "plaq_im", "q_re", "q_im", "action_re", "action_im", "eps",
                 "kmax", "alpha")
KERNEL_KINDS = ("init", "unorm", "pack", "clover", "drift", "update", "cool_omega", "cool_apply", "gradnorm",
                "measure", "finalize")


class cl_lattice_desc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("beta", ctypes.c_double), ("theta_re", ctypes.c_double),
                ("theta_im", ctypes.c_double), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class cl_step_desc(ctypes.Structure):
    _fields_ = [("eps0", ctypes.c_double), ("adaptive", ctypes.c_int32), ("drift_bound", ctypes.c_double)]


class cl_cool_desc(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("eps_c", ctypes.c_double), ("alpha", ctypes.c_double),
                ("mode", ctypes.c_int32)]


class cl_obs(ctypes.Structure):
    _fields_ = [("plaq", ctypes.c_double * 2), ("q", ctypes.c_double * 2), ("action", ctypes.c_double * 2),
                ("unorm_d", ctypes.c_double), ("d_pre", ctypes.c_double), ("eps", ctypes.c_double),
                ("kmax", ctypes.c_double), ("alpha", ctypes.c_double), ("bound", ctypes.c_double),
                ("step", ctypes.c_int64)]


class cl_run_desc(ctypes.Structure):
    _fields_ = [("lattice", cl_lattice_desc), ("step", cl_step_desc), ("cool", cl_cool_desc),
                ("n_steps", ctypes.c_int32), ("sigma_x", ctypes.c_double), ("sigma_y", ctypes.c_double),
                ("tag", ctypes.c_uint64), ("keep_links", ctypes.c_int32), ("pad", ctypes.c_int32)]


class cl_run_result(ctypes.Structure):
    _fields_ = [("run_id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("steps_done", ctypes.c_int32), ("obs", cl_obs), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double), ("step_ms_p50", ctypes.c_double),
                ("step_ms_p99", ctypes.c_double), ("link_updates", ctypes.c_int64)]


class cl_server_stats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int32), ("active", ctypes.c_int32), ("finished", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_budget", ctypes.c_size_t),
                ("batch_steps", ctypes.c_int64), ("link_updates", ctypes.c_int64), ("busy_s", ctypes.c_double),
                ("step_ms_p50", ctypes.c_double), ("step_ms_p99", ctypes.c_double),
                ("wait_s_p50", ctypes.c_double), ("wait_s_p99", ctypes.c_double)]


class cl_chain_desc(ctypes.Structure):
    _fields_ = [("n_links", ctypes.c_int32), ("n_chains", ctypes.c_int32), ("beta_re", ctypes.c_double),
                ("beta_im", ctypes.c_double), ("seed", ctypes.c_uint64), ("obs_cap", ctypes.c_int32)]


class cl_chain_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("L", ctypes.c_double * 2), ("d", ctypes.c_double), ("d_pre", ctypes.c_double),
                ("eps", ctypes.c_double), ("kmax", ctypes.c_double), ("sum_L", ctypes.c_double * 2),
                ("sum_d", ctypes.c_double), ("n_sum", ctypes.c_double), ("t_sum", ctypes.c_double)]


class ClError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"clgc error {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(the HIP library is the only implementation; there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp, sz = ctypes.c_void_p, P(ctypes.c_double), ctypes.c_size_t
    sigs = {
        "cl_lattice_bytes": [P(cl_lattice_desc), P(sz)],
        "cl_lattice_create": [P(cl_lattice_desc), vp, sz, vp, P(vp)],
        "cl_lattice_destroy": [vp],
        "cl_lattice_init": [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double],
        "cl_lattice_set_links": [vp, dp, sz],
        "cl_lattice_get_links": [vp, dp, sz],
        "cl_lattice_get_state": [vp, P(ctypes.c_int64), dp],
        "cl_lattice_set_state": [vp, ctypes.c_int64, ctypes.c_double],
        "cl_langevin_step": [vp, P(cl_step_desc), dp],
        "cl_gauge_cool": [vp, P(cl_cool_desc), dp],
        "cl_unitarity_norm": [vp, dp],
        "cl_measure": [vp, P(cl_obs)],
        "cl_compute_drift": [vp, dp, sz],
        "cl_cool_history": [vp, dp, dp, ctypes.c_int, P(ctypes.c_int)],
        "cl_run_steps": [vp, P(cl_step_desc), P(cl_cool_desc), ctypes.c_int],
        "cl_run_prepare": [vp, P(cl_step_desc), P(cl_cool_desc)],
        "cl_record_enable": [vp, ctypes.c_int],
        "cl_record_read": [vp, ctypes.c_int64, ctypes.c_int, dp],
        "cl_server_take_links": [vp, ctypes.c_uint64, dp, sz],
        "cl_measure_links": [vp, P(ctypes.c_int32), ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp],
        "cl_timing_enable": [vp, ctypes.c_int],
        "cl_server_create": [vp, sz, vp, P(vp)],
        "cl_server_submit": [vp, P(cl_run_desc), P(ctypes.c_uint64)],
        "cl_server_step": [vp, P(ctypes.c_int), P(ctypes.c_int)],
        "cl_server_steps": [vp, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int)],
        "cl_server_poll": [vp, P(cl_run_result), ctypes.c_int, P(ctypes.c_int)],
        "cl_server_stats_get": [vp, P(cl_server_stats)],
        "cl_server_destroy": [vp],
        "cl_timing_read": [vp, dp, P(ctypes.c_int64), ctypes.c_int],
        "cl_chain_bytes": [P(cl_chain_desc), P(sz)],
        "cl_chain_create": [P(cl_chain_desc), vp, sz, vp, P(vp)],
        "cl_chain_destroy": [vp],
        "cl_chain_init": [vp, ctypes.c_double, ctypes.c_double],
        "cl_chain_set_links": [vp, dp, sz],
        "cl_chain_get_links": [vp, dp, sz],
        "cl_chain_run": [vp, P(cl_step_desc), P(cl_cool_desc), ctypes.c_int, ctypes.c_int],
        "cl_chain_cool": [vp, P(cl_cool_desc)],
        "cl_chain_drift": [vp, dp, sz, dp],
        "cl_chain_measure": [vp, P(cl_chain_obs), ctypes.c_int],
        "cl_chain_record": [vp, dp, sz],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.cl_last_error.argtypes = []
    lib.cl_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(status):
    if status != CL_OK:
        raise ClError(status, lib.cl_last_error().decode())
    return status


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_desc(dims, beta, theta=0.0, precision=CL_FP64, seed=0):
    th = complex(theta)
    return cl_lattice_desc((ctypes.c_int32 * 4)(*dims), float(beta), th.real, th.imag, int(precision), int(seed))


def measure_links(dev_links, dims, beta, theta, dev_out, stream=None):
    """cl_measure_links: observables of a device link field (a float64 cuda
    tensor in the host layout) into dev_out (7 float64 on the device); no
    allocation, no wait."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(dev_links.device)
    assert dev_links.dtype == torch.float64 and dev_links.is_contiguous()
    assert dev_out.dtype == torch.float64 and dev_out.numel() >= 7
    th = complex(theta)
    _check(lib.cl_measure_links(ctypes.c_void_p(dev_links.data_ptr()), (ctypes.c_int32 * 4)(*dims), float(beta),
                                th.real, th.imag, ctypes.c_void_p(dev_out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))


def cl_lattice_bytes(desc):
    n = ctypes.c_size_t()
    _check(lib.cl_lattice_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


class Lattice:
    """One CL run: links, clover field, drift and control state in a torch
    device buffer, all work on one HIP stream."""

    def __init__(self, dims, beta, theta=0.0, precision=CL_FP64, seed=0, device="cuda:0", stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.beta = float(beta)
        self.theta = complex(theta)
        self.precision = precision
        self.desc = make_desc(self.dims, beta, theta, precision, seed)
        nbytes = cl_lattice_bytes(self.desc)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the caching allocator returns 512-byte aligned blocks; keep 256 of slack anyway
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.buf.data_ptr()
        aligned = (ptr + 255) & ~255
        self.nbytes = nbytes
        h = ctypes.c_void_p()
        _check(lib.cl_lattice_create(ctypes.byref(self.desc), ctypes.c_void_p(aligned), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    # -- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            _check(lib.cl_lattice_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- state -----------------------------------------------------------
    def init(self, perturbed=True, sigma_x=0.3, sigma_y=0.05):
        _check(lib.cl_lattice_init(self.handle, int(perturbed), float(sigma_x), float(sigma_y)))

    def set_links(self, links):
        a = np.ascontiguousarray(np.asarray(links, dtype=np.float64).reshape(-1))
        _check(lib.cl_lattice_set_links(self.handle, _dp(a), a.size))

    def get_links(self):
        a = np.zeros(self.V * 72)
        _check(lib.cl_lattice_get_links(self.handle, _dp(a), a.size))
        return a.reshape(self.V, 4, 18)

    def get_state(self):
        n, b = ctypes.c_int64(), ctypes.c_double()
        _check(lib.cl_lattice_get_state(self.handle, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def set_state(self, step, bound):
        _check(lib.cl_lattice_set_state(self.handle, int(step), float(bound)))

    # -- method ----------------------------------------------------------
    def langevin_step(self, eps0, adaptive=False, drift_bound=0.0, sync=True):
        sd = cl_step_desc(float(eps0), int(adaptive), float(drift_bound))
        if sync:
            e = ctypes.c_double()
            _check(lib.cl_langevin_step(self.handle, ctypes.byref(sd), ctypes.byref(e)))
            return e.value
        _check(lib.cl_langevin_step(self.handle, ctypes.byref(sd), None))
        return None

    def gauge_cool(self, n_steps, eps_c, alpha=1.0, mode=CL_ALPHA_FIXED, sync=True):
        cd = cl_cool_desc(int(n_steps), float(eps_c), float(alpha), int(mode))
        if sync:
            d = ctypes.c_double()
            _check(lib.cl_gauge_cool(self.handle, ctypes.byref(cd), ctypes.byref(d)))
            return d.value
        _check(lib.cl_gauge_cool(self.handle, ctypes.byref(cd), None))
        return None

    def run_steps(self, n, eps0, adaptive, n_cool, eps_c, alpha=1.0, mode=CL_ALPHA_FIXED, drift_bound=0.0):
        sd = cl_step_desc(float(eps0), int(adaptive), float(drift_bound))
        cd = cl_cool_desc(int(n_cool), float(eps_c), float(alpha), int(mode))
        _check(lib.cl_run_steps(self.handle, ctypes.byref(sd), ctypes.byref(cd), int(n)))

    def run_prepare(self, eps0, adaptive, n_cool, eps_c, alpha=1.0, mode=CL_ALPHA_FIXED, drift_bound=0.0):
        """Capture the graphs run_steps replays for these parameters now."""
        sd = cl_step_desc(float(eps0), int(adaptive), float(drift_bound))
        cd = cl_cool_desc(int(n_cool), float(eps_c), float(alpha), int(mode))
        _check(lib.cl_run_prepare(self.handle, ctypes.byref(sd), ctypes.byref(cd)))

    def record_enable(self, on=True):
        _check(lib.cl_record_enable(self.handle, int(on)))

    def record_read(self, first_step, n):
        """(n, 12) array of per-step record entries, columns RECORD_FIELDS."""
        a = np.zeros(int(n) * len(RECORD_FIELDS))
        _check(lib.cl_record_read(self.handle, int(first_step), int(n), _dp(a)))
        return a.reshape(int(n), len(RECORD_FIELDS))

    def unitarity_norm(self):
        d = ctypes.c_double()
        _check(lib.cl_unitarity_norm(self.handle, ctypes.byref(d)))
        return d.value

    def measure(self):
        o = cl_obs()
        _check(lib.cl_measure(self.handle, ctypes.byref(o)))
        return {"plaq": complex(o.plaq[0], o.plaq[1]), "q": complex(o.q[0], o.q[1]),
                "action": complex(o.action[0], o.action[1]), "d": o.unorm_d, "d_pre": o.d_pre,
                "eps": o.eps, "kmax": o.kmax, "alpha": o.alpha, "bound": o.bound, "step": o.step}

    def compute_drift(self):
        a = np.zeros(self.V * 72)
        _check(lib.cl_compute_drift(self.handle, _dp(a), a.size))
        return a.reshape(self.V, 4, 18)

    def cool_history(self):
        un = np.zeros(65)
        al = np.zeros(64)
        n = ctypes.c_int()
        _check(lib.cl_cool_history(self.handle, _dp(un), _dp(al), 65, ctypes.byref(n)))
        return un[:n.value + 1], al[:n.value]

    def timing_enable(self, on=True):
        _check(lib.cl_timing_enable(self.handle, int(on)))

    def timing_read(self):
        """{kernel kind: (total ms, launches)} since timing_enable(True)."""
        n = len(KERNEL_KINDS)
        ms = np.zeros(n)
        cnt = (ctypes.c_int64 * n)()
        _check(lib.cl_timing_read(self.handle, _dp(ms), cnt, n))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS) if cnt[i]}


def _obs_dict(o):
    return {"plaq": complex(o.plaq[0], o.plaq[1]), "q": complex(o.q[0], o.q[1]),
            "action": complex(o.action[0], o.action[1]), "d": o.unorm_d, "d_pre": o.d_pre,
            "eps": o.eps, "kmax": o.kmax, "alpha": o.alpha, "bound": o.bound, "step": o.step}


class Server:
    """Continuous batching of independent CL runs inside one device arena of
    `budget_bytes` (the HBM budget runs are admitted against)."""

    def __init__(self, budget_bytes, device="cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.arena = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.arena.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib.cl_server_create(ctypes.c_void_p(ptr), int(budget_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h)))
        self.handle = h

    def submit(self, dims, beta, theta=0.0, precision=CL_FP64, seed=0, n_steps=1, eps0=1e-2, adaptive=True,
               n_cool=10, eps_c=None, alpha=1.0, mode=CL_ALPHA_UNORM, sigma_x=0.3, sigma_y=0.05, tag=0,
               drift_bound=0.0, keep_links=False):
        d = cl_run_desc(make_desc(dims, beta, theta, precision, seed),
                        cl_step_desc(float(eps0), int(adaptive), float(drift_bound)),
                        cl_cool_desc(int(n_cool), float(eps0 if eps_c is None else eps_c), float(alpha), int(mode)),
                        int(n_steps), float(sigma_x), float(sigma_y), int(tag), int(bool(keep_links)), 0)
        rid = ctypes.c_uint64()
        _check(lib.cl_server_submit(self.handle, ctypes.byref(d), ctypes.byref(rid)))
        return rid.value

    def step(self, max_steps=1):
        a, p = ctypes.c_int(), ctypes.c_int()
        if max_steps == 1:
            _check(lib.cl_server_step(self.handle, ctypes.byref(a), ctypes.byref(p)))
        else:
            _check(lib.cl_server_steps(self.handle, int(max_steps), ctypes.byref(a), ctypes.byref(p)))
        return a.value, p.value

    def poll(self, cap=256):
        buf = (cl_run_result * cap)()
        n = ctypes.c_int()
        _check(lib.cl_server_poll(self.handle, buf, cap, ctypes.byref(n)))
        out = []
        for r in buf[:n.value]:
            out.append({"run_id": r.run_id, "tag": r.tag, "status": r.status, "steps_done": r.steps_done,
                        "obs": _obs_dict(r.obs), "t_submit": r.t_submit, "t_admit": r.t_admit,
                        "t_finish": r.t_finish, "step_ms_p50": r.step_ms_p50, "step_ms_p99": r.step_ms_p99,
                        "link_updates": r.link_updates})
        return out

    def take_links(self, run_id, dims):
        """Final links (V, 4, 18) of a finished run submitted with keep_links."""
        a = np.zeros(int(np.prod(dims)) * 72)
        _check(lib.cl_server_take_links(self.handle, int(run_id), _dp(a), a.size))
        return a.reshape(-1, 4, 18)

    def stats(self):
        st = cl_server_stats()
        _check(lib.cl_server_stats_get(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in cl_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(lib.cl_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chain:
    """n_chains SU(2) Polyakov chains of n_links links (complex beta), in a torch
    device buffer, all work on one HIP stream.  Links are (n_chains, n_links, 8)
    doubles: row-major 2x2 complex, (re, im) interleaved."""

    def __init__(self, n_links, n_chains, beta, seed=0, obs_cap=0, device="cuda:0", stream=None):
        import torch
        b = complex(beta)
        self.n_links, self.n_chains, self.beta = int(n_links), int(n_chains), b
        self.desc = cl_chain_desc(self.n_links, self.n_chains, b.real, b.imag, int(seed), int(obs_cap))
        nbytes = ctypes.c_size_t()
        _check(lib.cl_chain_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.buf.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib.cl_chain_create(ctypes.byref(self.desc), ctypes.c_void_p(aligned), nbytes.value,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(lib.cl_chain_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, sigma_x=0.3, sigma_y=0.05):
        _check(lib.cl_chain_init(self.handle, float(sigma_x), float(sigma_y)))

    def set_links(self, links):
        a = np.ascontiguousarray(np.asarray(links, dtype=np.float64).reshape(-1))
        _check(lib.cl_chain_set_links(self.handle, _dp(a), a.size))

    def get_links(self):
        a = np.zeros(self.n_chains * self.n_links * 8)
        _check(lib.cl_chain_get_links(self.handle, _dp(a), a.size))
        return a.reshape(self.n_chains, self.n_links, 8)

    def run(self, n_steps, eps0, adaptive=False, n_cool=0, eps_c=None, alpha=1.0, mode=CL_ALPHA_FIXED,
            drift_bound=0.0, record=False):
        sd = cl_step_desc(float(eps0), int(adaptive), float(drift_bound))
        cd = cl_cool_desc(int(n_cool), float(eps0 if eps_c is None else eps_c), float(alpha), int(mode))
        _check(lib.cl_chain_run(self.handle, ctypes.byref(sd), ctypes.byref(cd), int(n_steps), int(record)))

    def cool(self, n_steps, eps_c, alpha=1.0, mode=CL_ALPHA_FIXED):
        cd = cl_cool_desc(int(n_steps), float(eps_c), float(alpha), int(mode))
        _check(lib.cl_chain_cool(self.handle, ctypes.byref(cd)))

    def drift(self):
        K = np.zeros(self.n_chains * self.n_links * 8)
        km = np.zeros(self.n_chains)
        _check(lib.cl_chain_drift(self.handle, _dp(K), K.size, _dp(km)))
        return K.reshape(self.n_chains, self.n_links, 8), km

    def measure(self):
        """Per chain: dict of step, status, L, d, d_pre, eps, kmax, n_sum, t_sum and
        mean_L, mean_d: Langevin-time averages (each step weighted by its eps) over the
        steps of the last run."""
        buf = (cl_chain_obs * self.n_chains)()
        _check(lib.cl_chain_measure(self.handle, buf, self.n_chains))
        out = []
        for o in buf:
            t = o.t_sum
            out.append({"step": o.step, "status": o.status, "L": complex(o.L[0], o.L[1]), "d": o.d,
                        "d_pre": o.d_pre, "eps": o.eps, "kmax": o.kmax, "n_sum": o.n_sum, "t_sum": t,
                        "mean_L": complex(o.sum_L[0], o.sum_L[1]) / t if t > 0 else complex("nan"),
                        "mean_d": o.sum_d / t if t > 0 else float("nan")})
        return out

    def record(self, n_steps):
        """(n_steps, n_chains, 6): Re L, Im L, d, eps, kmax, d before cooling."""
        a = np.zeros(int(n_steps) * self.n_chains * 6)
        _check(lib.cl_chain_record(self.handle, _dp(a), a.size))
        return a.reshape(int(n_steps), self.n_chains, 6)
