"""Seeded SU(2)-chain inputs for the tests and the benchmark (input generation
only: no step of the method).  Links are (..., n, 8) doubles, a row-major
2x2 complex matrix with (re, im) interleaved."""
import numpy as np

PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], complex)


def expm_traceless(A):
    """exp(A) for traceless 2x2 A (batched): A^2 = w 1, so exp(A) = cosh(l) 1 + sinh(l)/l A, l^2 = w."""
    w = A[..., 0, 0] ** 2 + A[..., 0, 1] * A[..., 1, 0]
    l = np.sqrt(w + 0j)
    small = np.abs(l) < 1e-8
    S = np.where(small, 1.0 + w / 6.0, np.sinh(l) / np.where(small, 1.0, l))
    return np.cosh(l)[..., None, None] * np.eye(2) + S[..., None, None] * A


def to_links(U):
    U = np.asarray(U, complex)
    out = np.zeros(U.shape[:-2] + (8,))
    out[..., 0::2] = U.real.reshape(U.shape[:-2] + (4,))
    out[..., 1::2] = U.imag.reshape(U.shape[:-2] + (4,))
    return out


def gauge_rotated_chains(n_chains, n, seed, sv=0.5, sa=0.3, sb=0.3):
    """U_k = Omega_k V_k Omega_{k+1}^{-1} (periodic): V_k = exp(i sigma.x) in SU(2),
    Omega_k = exp(i sigma.(a + i b)) in SL(2,C), all independent normals -- a
    unitary chain moved off SU(2) along its gauge orbit."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0, sv, (n_chains, n, 3))
    c = rng.normal(0, sa, (n_chains, n, 3)) + 1j * rng.normal(0, sb, (n_chains, n, 3))
    V = expm_traceless(1j * np.einsum('cka,aij->ckij', x, PAULI))
    O = expm_traceless(1j * np.einsum('cka,aij->ckij', c, PAULI))
    Oi = expm_traceless(-1j * np.einsum('cka,aij->ckij', c, PAULI))
    return to_links(O @ V @ np.roll(Oi, -1, axis=1))
