"""Independent numpy helpers for the tests: Gell-Mann basis, random group
elements, brute-force lattice paths and closed-form configurations.  They are
written separately from the oracle so that the oracle can be checked against
them; the HIP path never imports them."""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg

LAMBDA = np.zeros((8, 3, 3), dtype=np.complex128)
LAMBDA[0][0, 1] = LAMBDA[0][1, 0] = 1
LAMBDA[1][0, 1] = -1j
LAMBDA[1][1, 0] = 1j
LAMBDA[2][0, 0] = 1
LAMBDA[2][1, 1] = -1
LAMBDA[3][0, 2] = LAMBDA[3][2, 0] = 1
LAMBDA[4][0, 2] = -1j
LAMBDA[4][2, 0] = 1j
LAMBDA[5][1, 2] = LAMBDA[5][2, 1] = 1
LAMBDA[6][1, 2] = -1j
LAMBDA[6][2, 1] = 1j
LAMBDA[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def to_c(a):
    a = np.asarray(a, dtype=np.float64)
    return (a[..., 0::2] + 1j * a[..., 1::2]).reshape(a.shape[:-1] + (3, 3))


def from_c(m):
    m = np.asarray(m, dtype=np.complex128)
    flat = m.reshape(m.shape[:-2] + (9,))
    out = np.empty(m.shape[:-2] + (18,))
    out[..., 0::2] = flat.real
    out[..., 1::2] = flat.imag
    return out


def lie(c):
    """sum_a c_a lambda_a."""
    return np.tensordot(np.asarray(c, dtype=np.complex128), LAMBDA, axes=(0, 0))


def random_sl3c(rng, scale_re=0.4, scale_im=0.2, n=None):
    """exp(i sum_a (x_a + i y_a) lambda_a): in SL(3,C) with det exactly 1 up
    to rounding."""
    shape = () if n is None else (n,)
    c = rng.normal(0, scale_re, shape + (8,)) + 1j * rng.normal(0, scale_im, shape + (8,))
    if n is None:
        return scipy.linalg.expm(1j * lie(c))
    return np.stack([scipy.linalg.expm(1j * lie(ci)) for ci in c])


def random_su3(rng, scale=0.6, n=None):
    return random_sl3c(rng, scale, 0.0, n)


def random_links(rng, dims, scale_re=0.4, scale_im=0.2):
    V = int(np.prod(dims))
    m = random_sl3c(rng, scale_re, scale_im, n=V * 4)
    return from_c(m).reshape(V, 4, 18)


def volume(dims):
    return int(np.prod(dims))


def site(dims, x):
    s = 0
    for m in (3, 2, 1, 0):
        s = s * dims[m] + (x[m] % dims[m])
    return s


def coords(dims, s):
    x = []
    for m in range(4):
        x.append(s % dims[m])
        s //= dims[m]
    return x


def link_c(links, dims, x, mu):
    return to_c(links[site(dims, x), mu])


def walk(links, dims, x, dirs):
    """Product of links along signed hops (+(mu+1) forward, -(mu+1) backward
    with the inverse matrix)."""
    x = list(x)
    M = np.eye(3, dtype=np.complex128)
    for d in dirs:
        mu = abs(d) - 1
        if d > 0:
            M = M @ link_c(links, dims, x, mu)
            x[mu] += 1
        else:
            x[mu] -= 1
            M = M @ np.linalg.inv(link_c(links, dims, x, mu))
    return M


def levi_civita(p):
    """Sign of a permutation of (0,1,2,3)."""
    p = list(p)
    sgn = 1
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                sgn = -sgn
    return sgn


def q_density_literal(links, dims, x):
    """q_L(x) from the definition: -(1/(2^4 32 pi^2)) sum over signed
    mu, nu, rho, sigma in +-1..+-4 of eps~_{mu nu rho sigma} Tr[U_{mu nu} U_{rho sigma}],
    with eps~ antisymmetric under a sign flip of any index and eps~_{1234} = 1;
    U_{mu nu}(x) the plaquette x -> x+mu -> x+mu+nu -> x+nu -> x."""
    plaq = {}
    for a in range(4):
        for b in range(4):
            if a == b:
                continue
            for sa in (1, -1):
                for sb in (1, -1):
                    m, n = sa * (a + 1), sb * (b + 1)
                    plaq[(m, n)] = walk(links, dims, x, [m, n, -m, -n])
    total = 0j
    for perm in itertools.permutations(range(4)):
        eps = levi_civita(perm)
        for signs in itertools.product((1, -1), repeat=4):
            m, n, r, s = [signs[i] * (perm[i] + 1) for i in range(4)]
            e = eps * signs[0] * signs[1] * signs[2] * signs[3]
            total += e * np.trace(plaq[(m, n)] @ plaq[(r, s)])
    return -total / (2 ** 4 * 32 * math.pi ** 2)


def abelian_flux(dims, n12, n34):
    """Uniform abelian flux with H = diag(1,-1,0): every counter-clockwise
    plaquette in the (0,1) plane is exp(i th12 H), in the (2,3) plane
    exp(i th34 H), all others 1; th12 = 2 pi n12/(L0 L1), th34 = 2 pi n34/(L2 L3)."""
    L0, L1, L2, L3 = dims
    th12 = 2 * math.pi * n12 / (L0 * L1)
    th34 = 2 * math.pi * n34 / (L2 * L3)
    h = np.array([1.0, -1.0, 0.0])
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    for s in range(V):
        x0, x1, x2, x3 = coords(dims, s)
        U[s, 0] = np.diag(np.exp(-1j * th12 * x1 * h))
        U[s, 1] = np.diag(np.exp(1j * th12 * L1 * x0 * h)) if x1 == L1 - 1 else np.eye(3)
        U[s, 2] = np.diag(np.exp(-1j * th34 * x3 * h))
        U[s, 3] = np.diag(np.exp(1j * th34 * L3 * x2 * h)) if x3 == L3 - 1 else np.eye(3)
    return from_c(U), th12, th34
