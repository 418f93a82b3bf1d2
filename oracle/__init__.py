"""FP64 CPU oracle (ctypes wrapper around clgc_oracle.c and chain_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The HIP library never imports it.

Host link layout (shared convention with the library's host API): a float64
array of shape (V, 4, 3, 3) complex, i.e. (V, 4, 18) interleaved doubles,
with sites in lexicographic order, x0 fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "clgc_oracle.c"), os.path.join(_HERE, "chain_oracle.c")]
# CLGC_ORACLE_SANITIZE=1 selects a build under AddressSanitizer and
# UndefinedBehaviorSanitizer (a separate library; the process must preload
# the gcc sanitizer runtimes, as the sanitizer test does)
_SANITIZE = os.environ.get("CLGC_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

_lib = None


def build(force: bool = True) -> str:
    """Compile clgc_oracle.c and chain_oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             *(_SAN_FLAGS if _SANITIZE else []), "-o", tmp, *_SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lp = ctypes.POINTER(ctypes.c_long)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_normal_pair.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [dp]
        L.orc_cl_noise.argtypes = [ctypes.c_uint64, ctypes.c_long, ctypes.c_int, ctypes.c_uint32, dp]
        L.orc_cold_links.argtypes = [ip, dp]
        L.orc_init_links.argtypes = [ip, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, dp]
        L.orc_plaquette.argtypes = [ip, dp, dp]
        L.orc_wilson_action.argtypes = [ip, dp, ctypes.c_double, dp]
        L.orc_topological_charge.argtypes = [ip, dp, dp]
        L.orc_unitarity_norm.argtypes = [ip, dp]
        L.orc_unitarity_norm.restype = ctypes.c_double
        L.orc_drift.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_drift_links.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      lp, ctypes.c_long, dp]
        L.orc_langevin_update.argtypes = [ip, dp, dp, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_langevin_step.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_double, dp, dp]
        L.orc_langevin_step.restype = ctypes.c_int
        L.orc_cool_gradient.argtypes = [ip, dp, ctypes.c_long, dp]
        L.orc_cool_halfsweep.argtypes = [ip, dp, ctypes.c_int, ctypes.c_double]
        L.orc_gauge_cool.argtypes = [ip, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, dp, dp]
        L.orc_gauge_cool.restype = ctypes.c_int
        L.orc_gauge_transform.argtypes = [ip, dp, dp]
        L.orc_expm.argtypes = [dp, dp]
        L.orc_path.argtypes = [ip, dp, ctypes.c_long, ip, ctypes.c_int, dp]
        L.orc_link_stats.argtypes = [ip, dp, dp]
        L.orc_run.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double,
                              ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        # SU(2) Polyakov chain
        c_u64, c_long, c_u32, c_int, c_d = ctypes.c_uint64, ctypes.c_long, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
        L.orc_chain_noise.argtypes = [c_u64, c_long, c_int, c_u32, dp]
        L.orc_chain_init.argtypes = [c_int, c_long, c_u64, c_d, c_d, dp]
        L.orc_chain_loop.argtypes = [c_int, dp, c_int, dp]
        L.orc_chain_drift.argtypes = [c_int, dp, c_d, c_d, dp]
        L.orc_chain_unorm.argtypes = [c_int, dp]
        L.orc_chain_unorm.restype = c_d
        L.orc_chain_measure.argtypes = [c_int, dp, c_d, c_d, dp]
        L.orc_chain_update.argtypes = [c_int, dp, dp, c_d, c_u64, c_long, c_u32]
        L.orc_chain_step.argtypes = [c_int, dp, c_d, c_d, c_u64, c_long, c_u32, c_d, c_int, c_d, dp, dp, dp]
        L.orc_chain_step.restype = c_int
        L.orc_chain_gradient.argtypes = [c_int, dp, dp]
        L.orc_chain_cool_step.argtypes = [c_int, dp, c_d]
        L.orc_chain_cool.argtypes = [c_int, dp, c_int, c_d, c_d, c_int, dp, dp]
        L.orc_chain_cool.restype = c_int
        L.orc_chain_run.argtypes = [c_int, dp, c_d, c_d, c_u64, c_long, c_u32, c_int, c_d, c_int, c_d, dp,
                                    c_int, c_d, c_d, c_int, dp]
        L.orc_chain_run.restype = c_int
        L.orc_chain_expm.argtypes = [dp, dp]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# marshalling helpers

def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,)
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def volume(dims):
    return int(np.prod(dims))


def to_complex(links):
    """(..., 18) interleaved doubles -> (..., 3, 3) complex128."""
    a = np.asarray(links, dtype=np.float64)
    return (a[..., 0::2] + 1j * a[..., 1::2]).reshape(a.shape[:-1] + (3, 3))


def from_complex(m):
    """(..., 3, 3) complex -> (..., 18) interleaved doubles (new array)."""
    m = np.asarray(m, dtype=np.complex128)
    flat = m.reshape(m.shape[:-2] + (9,))
    out = np.empty(m.shape[:-2] + (18,), dtype=np.float64)
    out[..., 0::2] = flat.real
    out[..., 1::2] = flat.imag
    return out


# ----------------------------------------------------------------------------
# wrappers

def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def normal_pair(seed, c0, c1, c2, c3):
    o = np.zeros(2)
    lib().orc_normal_pair(seed, c0, c1, c2, c3, _dp(o))
    return o


def cl_noise(seed, site, mu, step):
    o = np.zeros(8)
    lib().orc_cl_noise(seed, site, mu, step, _dp(o))
    return o


def cold_links(dims):
    d, dp = _dims(dims)
    u = np.zeros((volume(dims), 4, 18))
    lib().orc_cold_links(dp, _dp(u))
    return u


def init_links(dims, seed, sigma_x=0.3, sigma_y=0.05):
    d, dp = _dims(dims)
    u = np.zeros((volume(dims), 4, 18))
    lib().orc_init_links(dp, seed, sigma_x, sigma_y, _dp(u))
    return u


def plaquette(dims, links):
    d, dp = _dims(dims)
    o = np.zeros(2)
    lib().orc_plaquette(dp, _dp(np.ascontiguousarray(links)), _dp(o))
    return complex(o[0], o[1])


def wilson_action(dims, links, beta):
    d, dp = _dims(dims)
    o = np.zeros(2)
    lib().orc_wilson_action(dp, _dp(np.ascontiguousarray(links)), beta, _dp(o))
    return complex(o[0], o[1])


def topological_charge(dims, links):
    d, dp = _dims(dims)
    o = np.zeros(2)
    lib().orc_topological_charge(dp, _dp(np.ascontiguousarray(links)), _dp(o))
    return complex(o[0], o[1])


def unitarity_norm(dims, links):
    """Sum over links of Tr U U^dagger."""
    d, dp = _dims(dims)
    return lib().orc_unitarity_norm(dp, _dp(np.ascontiguousarray(links)))


def distance(dims, links):
    """d = (1/(12 V)) sum Tr(U U^dagger - 1)."""
    return unitarity_norm(dims, links) / (12.0 * volume(dims)) - 1.0


def drift(dims, links, beta, theta=0.0):
    d, dp = _dims(dims)
    th = complex(theta)
    K = np.zeros((volume(dims), 4, 18))
    lib().orc_drift(dp, _dp(np.ascontiguousarray(links)), beta, th.real, th.imag, _dp(K))
    return K


def drift_links(dims, links, beta, theta, sel):
    """Drift of selected links, sel = 4*site + mu; returns (len(sel), 18)."""
    d, dp = _dims(dims)
    th = complex(theta)
    s = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    K = np.zeros((len(s), 18))
    lib().orc_drift_links(dp, _dp(np.ascontiguousarray(links)), beta, th.real, th.imag,
                          s.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(s), _dp(K))
    return K


def langevin_update(dims, links, K, eps, seed, step):
    d, dp = _dims(dims)
    lib().orc_langevin_update(dp, _dp(links), _dp(np.ascontiguousarray(K)), eps, seed, step)


def langevin_step(dims, links, beta, theta, seed, step, eps0, adaptive=False,
                  drift_bound=0.0, bound=0.0):
    """In place.  Returns (eps_n, Kmax_n, bound)."""
    d, dp = _dims(dims)
    th = complex(theta)
    b = np.array([bound])
    o = np.zeros(2)
    rc = lib().orc_langevin_step(dp, _dp(links), beta, th.real, th.imag, seed, step, eps0,
                                 int(adaptive), drift_bound, _dp(b), _dp(o))
    if rc:
        raise RuntimeError(f"orc_langevin_step failed: {rc}")
    return o[0], o[1], b[0]


def cool_gradient(dims, links, site):
    d, dp = _dims(dims)
    f = np.zeros(8)
    lib().orc_cool_gradient(dp, _dp(np.ascontiguousarray(links)), site, _dp(f))
    return f


def cool_halfsweep(dims, links, parity, eps_alpha):
    d, dp = _dims(dims)
    lib().orc_cool_halfsweep(dp, _dp(links), parity, eps_alpha)


def gauge_cool(dims, links, n_steps, eps_c, alpha=1.0, mode=0):
    """In place.  Returns (unorm[n_steps+1], alpha_used[n_steps])."""
    d, dp = _dims(dims)
    un = np.zeros(n_steps + 1)
    al = np.zeros(max(n_steps, 1))
    rc = lib().orc_gauge_cool(dp, _dp(links), n_steps, eps_c, alpha, mode, _dp(un), _dp(al))
    if rc:
        raise RuntimeError(f"orc_gauge_cool failed: {rc}")
    return un, al[:n_steps]


def gauge_transform(dims, links, omega):
    """In place; omega: (V, 18) interleaved or (V, 3, 3) complex."""
    d, dp = _dims(dims)
    om = np.asarray(omega)
    if np.iscomplexobj(om):
        om = from_complex(om)
    om = np.ascontiguousarray(om, dtype=np.float64)
    lib().orc_gauge_transform(dp, _dp(links), _dp(om))


def expm(A):
    """exp of a (3,3) complex matrix."""
    a = from_complex(np.asarray(A, dtype=np.complex128))
    o = np.zeros(18)
    lib().orc_expm(_dp(np.ascontiguousarray(a)), _dp(o))
    return to_complex(o)


def path(dims, links, site, dirs):
    d, dp = _dims(dims)
    dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32))
    o = np.zeros(18)
    lib().orc_path(dp, _dp(np.ascontiguousarray(links)), site,
                   dd.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(dd), _dp(o))
    return to_complex(o)


def link_stats(dims, links):
    """(max |det U - 1|, min (1/3) Tr U U^dagger)."""
    d, dp = _dims(dims)
    o = np.zeros(2)
    lib().orc_link_stats(dp, _dp(np.ascontiguousarray(links)), _dp(o))
    return o[0], o[1]


OBS_FIELDS = ("d_pre", "d_post", "plaq_re", "plaq_im", "q_re", "q_im", "eps", "kmax")


def set_threads(n=0):
    """Set (n > 0) and return the OpenMP thread count of the oracle (timing only)."""
    return lib().orc_set_threads(int(n))


def run(dims, links, beta, theta, seed, n_steps, eps0, adaptive, n_cool, eps_c, alpha=1.0,
        mode=0, step0=0, drift_bound=0.0, bound=0.0):
    """In place on links.  Returns (obs[n_steps, 8], bound)."""
    d, dp = _dims(dims)
    th = complex(theta)
    b = np.array([bound])
    obs = np.zeros((n_steps, 8))
    rc = lib().orc_run(dp, _dp(links), beta, th.real, th.imag, seed, step0, n_steps, eps0,
                       int(adaptive), drift_bound, _dp(b), n_cool, eps_c, alpha, mode, _dp(obs))
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    return obs, b[0]


def cl_noise_field(dims, seed, step):
    """eta_1..eta_8 of every link at CL step `step`: (V, 4, 8)."""
    d, dp = _dims(dims)
    o = np.zeros((volume(dims), 4, 8))
    lib().orc_cl_noise_field.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)]
    lib().orc_cl_noise_field(dp, seed, step, _dp(o))
    return o


# ----------------------------------------------------------------------------
# SU(2) Polyakov chain.  A chain is a float64 array (n, 8): link k as a 2x2
# complex matrix, row-major, (re, im) interleaved; several chains are
# (n_chains, n, 8).

def chain_to_complex(links):
    a = np.asarray(links, dtype=np.float64)
    return (a[..., 0::2] + 1j * a[..., 1::2]).reshape(a.shape[:-1] + (2, 2))


def chain_from_complex(m):
    m = np.asarray(m, dtype=np.complex128)
    out = np.zeros(m.shape[:-2] + (8,))
    out[..., 0::2] = m.real.reshape(m.shape[:-2] + (4,))
    out[..., 1::2] = m.imag.reshape(m.shape[:-2] + (4,))
    return out


def _chain(links):
    a = np.ascontiguousarray(links, dtype=np.float64)
    assert a.shape[-1] == 8
    return a, a.shape[-2]


def chain_noise(seed, chain, k, step):
    o = np.zeros(3)
    lib().orc_chain_noise(seed, chain, k, step, _dp(o))
    return o


def chain_init(n, chain, seed, sigma_x=0.3, sigma_y=0.05):
    u = np.zeros((n, 8))
    lib().orc_chain_init(n, chain, seed, sigma_x, sigma_y, _dp(u))
    return u


def chain_loop(links, k):
    a, n = _chain(links)
    o = np.zeros(8)
    lib().orc_chain_loop(n, _dp(a), k, _dp(o))
    return o


def chain_drift(links, beta):
    a, n = _chain(links)
    b = complex(beta)
    K = np.zeros((n, 8))
    lib().orc_chain_drift(n, _dp(a), b.real, b.imag, _dp(K))
    return K


def chain_unorm(links):
    a, n = _chain(links)
    return lib().orc_chain_unorm(n, _dp(a))


def chain_measure(links, beta):
    """(L, d, S): Polyakov loop Tr(U_0...U_{n-1})/2, distance, action -beta L."""
    a, n = _chain(links)
    b = complex(beta)
    o = np.zeros(5)
    lib().orc_chain_measure(n, _dp(a), b.real, b.imag, _dp(o))
    return complex(o[0], o[1]), o[2], complex(o[3], o[4])


def chain_update(links, K, eps, seed, chain, step):
    """In place on links."""
    n = links.shape[-2]
    lib().orc_chain_update(n, _dp(links), _dp(np.ascontiguousarray(K)), eps, seed, chain, step)


def chain_step(links, beta, seed, chain, step, eps0, adaptive=False, drift_bound=0.0, bound=0.0):
    """In place.  Returns (rc, eps, kmax, bound)."""
    n = links.shape[-2]
    b = complex(beta)
    bd, e, k = np.array([bound]), np.zeros(1), np.zeros(1)
    rc = lib().orc_chain_step(n, _dp(links), b.real, b.imag, seed, chain, step, eps0, int(adaptive), drift_bound,
                              _dp(bd), _dp(e), _dp(k))
    return rc, e[0], k[0], bd[0]


def chain_gradient(links):
    a, n = _chain(links)
    f = np.zeros((n, 3))
    lib().orc_chain_gradient(n, _dp(a), _dp(f))
    return f


def chain_cool_step(links, eps_alpha):
    """In place: one Jacobi cooling step with eps * alpha_ad = eps_alpha."""
    lib().orc_chain_cool_step(links.shape[-2], _dp(links), eps_alpha)


def chain_cool(links, n_cool, eps_c, alpha=1.0, mode=0):
    """In place.  Returns (rc, un[n_cool+1], alpha_used[n_cool])."""
    n = links.shape[-2]
    un, al = np.zeros(n_cool + 1), np.zeros(max(n_cool, 1))
    rc = lib().orc_chain_cool(n, _dp(links), n_cool, eps_c, alpha, mode, _dp(un), _dp(al))
    return rc, un, al[:n_cool]


def chain_run(links, beta, seed, chain, n_steps, eps0, adaptive, n_cool, eps_c, alpha=1.0, mode=0,
              step0=0, drift_bound=0.0, bound=0.0):
    """In place.  Returns (rc, obs[n_steps, 6], bound); obs rows are
    (Re L, Im L, d, eps, kmax, d before cooling)."""
    n = links.shape[-2]
    b = complex(beta)
    bd = np.array([bound])
    obs = np.zeros((n_steps, 6))
    rc = lib().orc_chain_run(n, _dp(links), b.real, b.imag, seed, chain, step0, n_steps, eps0, int(adaptive),
                             drift_bound, _dp(bd), n_cool, eps_c, alpha, mode, _dp(obs))
    return rc, obs, bd[0]


def chain_expm(A):
    a = chain_from_complex(np.asarray(A, dtype=np.complex128).reshape(1, 2, 2))[0]
    o = np.zeros(8)
    lib().orc_chain_expm(_dp(np.ascontiguousarray(a)), _dp(o))
    return chain_to_complex(o)
