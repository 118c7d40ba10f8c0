"""Pins of the oracle's initial conditions: FFT, Poisson, Wilson lines,
matching and the initial longitudinal field, against brute force, closed
forms and exact invariants."""
import numpy as np
import pytest

from tests import seeded_inputs as si


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9, 12, 32, 96, 384, 512])
def test_fft_matches_direct_dft(orc, n):
    g = si.rng(n)
    x = g.normal(size=n) + 1j * g.normal(size=n)
    k = np.arange(n)
    dft = np.exp(-2j * np.pi * np.outer(k, k) / n) @ x
    assert np.abs(orc.fft(x, -1) - dft).max() < 1e-12 * max(1, n)
    assert np.abs(orc.fft(x, +1) - np.conj(np.exp(-2j * np.pi * np.outer(k, k) / n)) @ x).max() < 1e-12 * max(1, n)


def _dense_lattice_operator(N, m2):
    n2 = N * N
    A = np.zeros((n2, n2))
    for y in range(N):
        for x in range(N):
            i = x + N * y
            A[i, i] = 4.0 + m2
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                j = (x + dx) % N + N * ((y + dy) % N)
                A[i, j] -= 1.0
    return A


@pytest.mark.parametrize("N", [3, 4, 6])
def test_poisson_equals_dense_solve(orc, N):
    m2 = 0.05
    src = si.rng(5).normal(size=N * N)
    want = np.linalg.solve(_dense_lattice_operator(N, m2), src)
    assert np.abs(orc.poisson(N, m2, src) - want).max() < 1e-13


def test_poisson_cosine_mode_eigenvalue(orc):
    N, m2 = 32, 0.01
    xs = np.arange(N)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    kx, ky = 3, 5
    mode = np.cos(2 * np.pi * (kx * X + ky * Y) / N).reshape(-1)
    lam = 4 * np.sin(np.pi * kx / N) ** 2 + 4 * np.sin(np.pi * ky / N) ** 2 + m2
    assert np.abs(orc.poisson(N, m2, mode) - mode / lam).max() < 1e-13


def _plaquettes(N, U):
    Um = U.view(np.complex128).reshape(2, N * N, 3, 3)
    idx = np.arange(N * N)
    xp = (idx % N + 1) % N + N * (idx // N)
    yp = idx % N + N * ((idx // N + 1) % N)
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    return Um[0] @ Um[1][xp] @ dag(Um[0][yp]) @ dag(Um[1])


def test_wilson_lines_unitary_and_pure_gauge(orc):
    N = 16
    V = orc.wilson_line(N, 0.6, 0.01, 3, 1234, 0)
    Vm = V.view(np.complex128).reshape(-1, 3, 3)
    assert np.abs(Vm @ np.conj(np.swapaxes(Vm, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(Vm) - 1).max() < 1e-13
    Un = orc.nucleus_links(N, V)
    P = _plaquettes(N, Un)
    assert np.abs(P - np.eye(3)).max() < 1e-13


def test_wilson_line_single_sheet_is_exp_of_poisson(orc):
    """With one sheet, V = exp(-i Lambda^a T^a) with Lambda the Poisson solution
    of the same charges: checked color by color through the library expm."""
    import scipy.linalg as sla
    N, sigma, m2, seed = 8, 0.5, 0.04, 77
    rho = orc.mv_charges(N, sigma, seed, 1, 0)
    lam = np.stack([orc.poisson(N, m2, rho[:, a]) for a in range(8)], axis=1)
    T = np.array([orc.generator(a) for a in range(8)])
    V = orc.wilson_line(N, sigma, m2, 1, seed, 1).view(np.complex128).reshape(-1, 3, 3)
    for x in range(N * N):
        want = sla.expm(-1j * np.einsum("a,aij->ij", lam[x], T))
        assert np.abs(V[x] - want).max() < 1e-13


def _su2_embed(m2):
    m = np.eye(3, dtype=np.complex128)
    m[:2, :2] = m2
    return m


def test_matching_su2_embedded_closed_form(orc):
    """SU(2)-embedded nuclei: U = What^2 with What = W / sqrt(det W), W = UA + UB."""
    g = si.rng(21)
    for _ in range(20):
        a = g.normal(size=4)
        b = g.normal(size=4)
        su2 = lambda v: (lambda q: np.array([[q[0] + 1j * q[3], q[2] + 1j * q[1]],
                                             [-q[2] + 1j * q[1], q[0] - 1j * q[3]]]))(v / np.linalg.norm(v))
        A2, B2 = su2(a), su2(b)
        W = A2 + B2
        Wh = W / np.sqrt(np.linalg.det(W))
        want = _su2_embed(Wh @ Wh)
        U, it, res = orc.match_link(_su2_embed(A2), _su2_embed(B2))
        assert it >= 0 and res < 1e-13
        assert np.abs(U - want).max() < 1e-12


def test_matching_commuting_inputs(orc):
    """Diagonal (commuting) nuclei: U = UA UB solves the condition."""
    g = si.rng(22)
    for _ in range(10):
        ta, tb = g.normal(size=2), g.normal(size=2)
        A = np.diag(np.exp(1j * np.array([ta[0], ta[1], -ta[0] - ta[1]])))
        B = np.diag(np.exp(1j * np.array([tb[0], tb[1], -tb[0] - tb[1]])))
        U, it, res = orc.match_link(A, B)
        assert res < 1e-13
        assert np.abs(U - A @ B).max() < 1e-13


def test_matching_random_links_residual(orc):
    g = si.rng(23)
    UA = si.near_identity_su3(g, 200, 0.4)
    UB = si.near_identity_su3(g, 200, 0.4)
    T = np.array([orc.generator(a) for a in range(8)])
    for k in range(200):
        U, it, res = orc.match_link(UA[k], UB[k])
        assert it >= 0 and res < 1e-13
        assert np.abs(U @ U.conj().T - np.eye(3)).max() < 1e-13
        # residual recomputed here from the definition of [.]_X
        M = (UA[k] + UB[k]) @ (np.eye(3) + U.conj().T)
        AH = (M - M.conj().T) / 2j
        AH -= np.trace(AH) / 3 * np.eye(3)
        assert np.abs(AH).max() < 1e-12


def test_pi0_weak_field_limit_and_antisymmetry(orc):
    """U^A = e^{i eps a_i}, U^B = e^{i eps b_i}: pi0 -> -i sum_i [a_i, b_i] eps^2."""
    N = 4
    g = si.rng(31)
    T = np.array([orc.generator(a) for a in range(8)])
    a = g.normal(size=(2, 8))
    b = g.normal(size=(2, 8))
    A = [np.einsum("c,cij->ij", a[i], T) for i in range(2)]
    B = [np.einsum("c,cij->ij", b[i], T) for i in range(2)]
    comm = sum(A[i] @ B[i] - B[i] @ A[i] for i in range(2))
    want = -1j * comm
    want8 = np.array([2 * np.real(np.trace(T[c] @ want)) for c in range(8)])
    errs = []
    for eps in (1e-2, 1e-3):
        UA = np.stack([np.stack([orc.expi(eps * a[i])] * (N * N)) for i in range(2)])
        UB = np.stack([np.stack([orc.expi(eps * b[i])] * (N * N)) for i in range(2)])
        UAd = si.mats_to_d(UA).reshape(2, N * N, 18).copy()
        UBd = si.mats_to_d(UB).reshape(2, N * N, 18).copy()
        U = np.zeros_like(UAd)
        for d in range(2):
            for x in range(N * N):
                m, it, res = orc.match_link(UA[d, x], UB[d, x])
                U[d, x] = si.mats_to_d(m)
        p = orc.pi0(N, U, UAd, UBd)
        errs.append(np.abs(p / eps ** 2 - want8).max())
        p_swap = orc.pi0(N, U, UBd, UAd)
        assert np.abs(p + p_swap).max() < 1e-15
    # the error is O(eps): it falls tenfold with eps
    assert errs[1] < 0.2 * errs[0] + 1e-9
    assert errs[1] < 1e-2


def test_init_glasma_invariants(orc):
    """Initial state: matched links unitary, E = 0, Gauss law zero, phi = dtau^2 pi0 / 2."""
    N, dt = 16, 0.125
    s, rc, res = orc.init_glasma(N, 0.6, 0.016, 2, 2307079991, dt)
    assert rc == 0 and res < 1e-13
    Um = s.U.view(np.complex128).reshape(2, -1, 3, 3)
    assert np.abs(Um @ np.conj(np.swapaxes(Um, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(s.E).max() == 0.0
    assert np.abs(s.phi - 0.5 * dt * dt * s.pi).max() < 1e-17
    assert np.abs(orc.gauss(s)).max() < 1e-14


def test_poisson_uv_cut_keeps_low_and_removes_high_modes(orc):
    N, m2 = 32, 0.01
    xs = np.arange(N)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    low = np.cos(2 * np.pi * (2 * X + 1 * Y) / N).reshape(-1)
    high = np.cos(2 * np.pi * (12 * X + 9 * Y) / N).reshape(-1)
    k2 = lambda kx, ky: 4 * np.sin(np.pi * kx / N) ** 2 + 4 * np.sin(np.pi * ky / N) ** 2
    uv2 = 0.5 * (k2(2, 1) + k2(12, 9))
    out = orc.poisson_uv(N, m2, uv2, low + high)
    assert np.abs(out - low / (k2(2, 1) + m2)).max() < 1e-13
    # no cut reproduces the plain solve
    assert np.abs(orc.poisson_uv(N, m2, 0.0, low + high) - orc.poisson(N, m2, low + high)).max() < 1e-15


def test_dipole_of_abelian_plane_wave(orc):
    """V(x) = diag(e^{i alpha ix}, e^{-i alpha ix}, 1): along x,
    Tr V(x) V^dag(x+r) = 2 cos(alpha r) + 1, along y it is 3, so
    D(r) = [(2 cos(alpha r) + 1) / 3 + 1] / 2; D(0) = 1 for any V."""
    N = 12
    alpha = 2 * np.pi * 2 / N
    V = np.zeros((N * N, 3, 3), complex)
    for y in range(N):
        for x in range(N):
            V[x + N * y] = np.diag([np.exp(1j * alpha * x), np.exp(-1j * alpha * x), 1.0])
    D = orc.dipole(N, orc.m2d(V), N // 2)
    r = np.arange(N // 2 + 1)
    assert np.abs(D - ((2 * np.cos(alpha * r) + 1) / 3 + 1) / 2).max() < 1e-14
    W = orc.wilson_line(N, 0.6, 0.01, 2, 3, 0)
    D = orc.dipole(N, W, N // 2)
    assert abs(D[0] - 1.0) < 1e-13 and np.all(D[1:] < 1.0)
