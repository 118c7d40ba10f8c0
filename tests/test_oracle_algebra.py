"""Pins of the oracle's SU(3) algebra and random numbers against textbook and
published values (not against the oracle itself)."""
import itertools
import os

import numpy as np
import pytest
import scipy.linalg as sla

from tests import seeded_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_generators_normalised(orc):
    T = [orc.generator(a) for a in range(8)]
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T, atol=0)
        assert abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15


def test_structure_constants_textbook(orc):
    """f_abc and d_abc of the oracle's generators equal the textbook table."""
    T = [orc.generator(a) for a in range(8)]
    f = np.zeros((8, 8, 8))
    d = np.zeros((8, 8, 8))
    for kind, i, j, k, v in _read_golden("su3_structure_constants.txt"):
        i, j, k, v = int(i) - 1, int(j) - 1, int(k) - 1, float(v)
        for perm in itertools.permutations((0, 1, 2)):
            idx = tuple((i, j, k)[p] for p in perm)
            if kind == "f":
                sign = np.linalg.det(np.eye(3)[list(perm)])
                f[idx] = sign * v
            else:
                d[idx] = v
    for a in range(8):
        for b in range(8):
            comm = T[a] @ T[b] - T[b] @ T[a]
            anti = T[a] @ T[b] + T[b] @ T[a]
            want_c = 1j * sum(f[a, b, c] * T[c] for c in range(8))
            want_a = (a == b) / 3.0 * np.eye(3) + sum(d[a, b, c] * T[c] for c in range(8))
            assert np.abs(comm - want_c).max() < 1e-14
            assert np.abs(anti - want_a).max() < 1e-14
            for c in range(8):
                assert abs(orc.dsym(a, b, c) - d[a, b, c]) < 1e-14
    assert abs((d ** 2).sum() - 40.0 / 3.0) < 1e-12


def test_exp_cartan_closed_form(orc):
    for th in (0.0, 1e-9, 0.3, 2.0, -5.0):
        x = np.zeros(8)
        x[2] = th
        want = np.diag([np.exp(0.5j * th), np.exp(-0.5j * th), 1.0])
        assert np.abs(orc.expi(x) - want).max() < 1e-14


def test_exp_matches_library_expm(orc):
    T = np.array([orc.generator(a) for a in range(8)])
    g = si.rng(11)
    for scale in (1e-6, 0.1, 1.0, 4.0):
        for _ in range(20):
            x = scale * g.normal(size=8)
            H = np.einsum("a,aij->ij", x, T)
            want = sla.expm(1j * H)
            got = orc.expi(x)
            assert np.abs(got - want).max() < 2e-14 * max(1.0, scale)
            assert np.abs(got @ got.conj().T - np.eye(3)).max() < 1e-14 * max(1.0, scale)
            assert abs(np.linalg.det(got) - 1.0) < 1e-13 * max(1.0, scale)


def test_projection_of_exponential(orc):
    """[exp(iF)]_X = F + O(F^3), and [M]_X ignores the hermitian part of M."""
    T = np.array([orc.generator(a) for a in range(8)])
    g = si.rng(12)
    for eps in (1e-2, 1e-3):
        x = eps * g.normal(size=8)
        got = orc.proj(orc.expi(x))
        assert np.abs(got - x).max() < 5 * eps ** 3
    x = g.normal(size=8)
    H = np.einsum("a,aij->ij", g.normal(size=8), T)
    M = 1j * np.einsum("a,aij->ij", x, T) + H + 0.7j * np.eye(3)
    assert np.abs(orc.proj(M) - x).max() < 1e-14


def test_philox_known_answers(orc):
    for row in _read_golden("philox4x32_10_kat.txt"):
        v = [int(s, 16) for s in row]
        out = orc.philox(v[4:6], v[0:4])
        assert list(out) == v[6:10]


def test_u53_range_and_exactness(orc):
    assert orc.u53(0, 0) == 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # hi word carries the most significant bits
    assert orc.u53(0, 0x80000000) == 0.5 + 2.0 ** -53


def test_mv_charge_statistics(orc):
    """Each color of the MV charges is N(0, sigma^2), independent of the others."""
    N, sigma = 64, 0.7
    rho = np.concatenate([orc.mv_charges(N, sigma, 99, nuc, sh) for nuc in (0, 1)
                          for sh in (0, 3)])
    n = rho.shape[0]
    mean = rho.mean(axis=0)
    var = rho.var(axis=0)
    assert np.all(np.abs(mean) < 5 * sigma / np.sqrt(n))
    assert np.all(np.abs(var - sigma ** 2) < 5 * sigma ** 2 * np.sqrt(2.0 / n))
    cov = np.cov(rho.T)
    off = cov - np.diag(np.diag(cov))
    assert np.abs(off).max() < 5 * sigma ** 2 / np.sqrt(n)
    # distinct (nucleus, sheet) streams differ
    assert not np.allclose(orc.mv_charges(8, 1.0, 99, 0, 0), orc.mv_charges(8, 1.0, 99, 1, 0))
    assert not np.allclose(orc.mv_charges(8, 1.0, 99, 0, 0), orc.mv_charges(8, 1.0, 99, 0, 1))
