"""Seeded synthetic inputs shared by the oracle and HIP sides of the tests.

This module only draws random numbers and builds plain arrays from them
(numpy generators and numpy's QR factorisation).  It holds none of the
method's arithmetic: no exponentials of the algebra, no plaquettes, no
field or particle updates.  Layouts produced here are the oracle's
array-of-structures layout; ``to_soa``/``from_soa`` convert to and from the
HIP library's structure-of-arrays planes with transposes only.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def haar_su3(g, n):
    """n matrices drawn from Haar measure on U(3) (QR with phase fix), det set to 1."""
    z = (g.normal(size=(n, 3, 3)) + 1j * g.normal(size=(n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def near_identity_su3(g, n, eps):
    """Unitary matrices within O(eps) of 1: polar part of 1 + eps*Z, det set to 1."""
    z = g.normal(size=(n, 3, 3)) + 1j * g.normal(size=(n, 3, 3))
    m = np.eye(3) + eps * z
    u, _, vh = np.linalg.svd(m)
    q = u @ vh
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def mats_to_d(m):
    m = np.ascontiguousarray(m, np.complex128)
    return m.view(np.float64).reshape(m.shape[:-2] + (18,))


def random_state(seed, N, link_kind="haar", eps=0.3, e_scale=0.2, phi_scale=0.2,
                 pi_scale=0.2):
    """Random field state in the oracle layout: U [2,N2,18], E [2,N2,8], phi, pi [N2,8]."""
    g = rng(seed)
    n2 = N * N
    if link_kind == "haar":
        U = haar_su3(g, 2 * n2)
    else:
        U = near_identity_su3(g, 2 * n2, eps)
    U = mats_to_d(U).reshape(2, n2, 18).copy()
    E = e_scale * g.normal(size=(2, n2, 8))
    phi = phi_scale * g.normal(size=(n2, 8))
    pi = pi_scale * g.normal(size=(n2, 8))
    return U, E, phi, pi


def random_algebra(seed, n, scale=1.0):
    return scale * rng(seed).normal(size=(n, 8))


# ---- layout conversion (transposes only) ----------------------------------
def links_to_soa(U):
    """[2,N2,18] -> [2,18,N2]"""
    return np.ascontiguousarray(np.transpose(U, (0, 2, 1)))


def links_from_soa(U):
    return np.ascontiguousarray(np.transpose(U, (0, 2, 1)))


def alg_to_soa(X):
    """[..., N2, 8] -> [..., 8, N2]"""
    return np.ascontiguousarray(np.swapaxes(X, -1, -2))


def alg_from_soa(X):
    return np.ascontiguousarray(np.swapaxes(X, -1, -2))
