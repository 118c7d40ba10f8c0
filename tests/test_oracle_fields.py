"""Pins of the oracle's field evolution: the leapfrog force is minus the
gradient of the lattice Hamiltonian (brute force on 4^2), the Gauss law is an
exact invariant, weak abelian modes follow the Bessel closed forms, and the
evolution is gauge covariant."""
import numpy as np
import pytest
from scipy.special import jv

from tests import seeded_inputs as si


def _H(orc, N, tau, U, E, phi, pi):
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi = U, E, phi, pi
    return orc.energy(s, tau).sum()


def _left_mul(orc, U, d, x, a, eps):
    U2 = U.copy()
    e = np.zeros(8)
    e[a] = eps
    m = orc.expi(e) @ orc.d2m(U[d, x])
    U2[d, x] = orc.m2d(m)
    return U2


@pytest.mark.parametrize("kind", ["near", "haar"])
def test_force_is_minus_gradient_of_hamiltonian(orc, kind):
    N, tau = 4, 0.7
    U, E, phi, pi = si.random_state(3, N, link_kind=kind, eps=0.5, phi_scale=0.5)
    FE, Fpi = orc.forces(N, tau, U, phi)
    h = 1e-5
    for d in range(2):
        for x in range(N * N):
            for a in range(8):
                Hp = _H(orc, N, tau, _left_mul(orc, U, d, x, a, h), E, phi, pi)
                Hm = _H(orc, N, tau, _left_mul(orc, U, d, x, a, -h), E, phi, pi)
                assert abs(-(Hp - Hm) / (2 * h) - FE[d, x, a]) < 1e-8
    for x in range(N * N):
        for a in range(8):
            p2, m2 = phi.copy(), phi.copy()
            p2[x, a] += h
            m2[x, a] -= h
            dH = (_H(orc, N, tau, U, E, p2, pi) - _H(orc, N, tau, U, E, m2, pi)) / (2 * h)
            assert abs(-dH - Fpi[x, a]) < 1e-8


def test_hamiltonian_kinetic_terms(orc):
    """dH/dE^a = E^a / tau and dH/dpi^a = tau pi^a (the U and phi velocities)."""
    N, tau = 4, 1.3
    U, E, phi, pi = si.random_state(4, N)
    h = 1e-3   # H is quadratic in E and pi: central differences are exact
    for (d, x, a) in [(0, 3, 2), (1, 7, 7), (0, 15, 0)]:
        Ep, Em = E.copy(), E.copy()
        Ep[d, x, a] += h
        Em[d, x, a] -= h
        g = (_H(orc, N, tau, U, Ep, phi, pi) - _H(orc, N, tau, U, Em, phi, pi)) / (2 * h)
        assert abs(g - E[d, x, a] / tau) < 1e-8
    for (x, a) in [(0, 1), (9, 5)]:
        pp, pm = pi.copy(), pi.copy()
        pp[x, a] += h
        pm[x, a] -= h
        g = (_H(orc, N, tau, U, E, phi, pp) - _H(orc, N, tau, U, E, phi, pm)) / (2 * h)
        assert abs(g - tau * pi[x, a]) < 1e-8


def test_gauss_law_conserved_and_links_unitary(orc):
    N, dt = 8, 0.125
    U, E, phi, pi = si.random_state(5, N, link_kind="near", eps=0.6)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 3
    G0 = orc.gauss(s)
    assert np.abs(G0).max() > 0.1     # a generic state violates the constraint
    for _ in range(40):
        orc.field_step(s, dt)
    assert np.abs(orc.gauss(s) - G0).max() < 1e-12
    Um = orc.d2m(s.U)
    assert np.abs(Um @ np.conj(np.swapaxes(Um, -1, -2)) - np.eye(3)).max() < 1e-13


def _run_mode(orc, N, dt, tau_end, setup):
    s = orc.State(N)
    s.U[:] = orc.m2d(np.eye(3))
    setup(s)
    n_end = int(round(tau_end / dt))
    s.n = 1
    while s.n < n_end:
        orc.field_step(s, dt)
    return s


@pytest.mark.parametrize("which", ["longitudinal", "transverse"])
def test_weak_abelian_modes_follow_bessel(orc, which):
    """Weak T^3 mode along x with lattice momentum k: pi = pi0 J0(k tau),
    phi = pi0 tau J1(k tau)/k; a transverse A_y mode: A = A0 J0(k tau).
    The leapfrog error is O(dtau^2): it falls fourfold per halving."""
    N, kx, amp, tau_end = 16, 2, 1e-6, 4.0
    k = 2 * np.sin(np.pi * kx / N)
    xs = np.arange(N * N) % N
    prof = np.cos(2 * np.pi * kx * xs / N)
    errs = []
    for dt in (0.25, 0.125, 0.0625):
        if which == "longitudinal":
            def setup(s, dt=dt):
                s.pi[:, 2] = amp * prof
                s.phi[:, 2] = dt * (0.5 * dt) * s.pi[:, 2]
            s = _run_mode(orc, N, dt, tau_end, setup)
            tau = s.n * dt
            tau_h = (s.n - 0.5) * dt
            e1 = np.abs(s.phi[:, 2] - amp * prof * tau * jv(1, k * tau) / k).max()
            e2 = np.abs(s.pi[:, 2] - amp * prof * jv(0, k * tau_h)).max()
            errs.append(max(e1, e2) / amp)
        else:
            def setup(s):
                for x in range(N * N):
                    s.U[1, x] = orc.m2d(np.diag(np.exp(1j * amp * prof[x] * np.array([0.5, -0.5, 0]))))
            s = _run_mode(orc, N, dt, tau_end, setup)
            tau = s.n * dt
            A = np.array([np.angle(orc.d2m(s.U[1, x])[0, 0]) * 2 for x in range(N * N)])
            errs.append(np.abs(A - amp * prof * jv(0, k * tau)).max() / amp)
    assert errs[0] < 0.05
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


def _gauge_transform(orc, N, Om, U, E, phi, pi):
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    T = np.array([orc.generator(a) for a in range(8)])
    comp = lambda M: 2 * np.real(np.einsum("aij,nji->na", T, M))
    Um = orc.d2m(U)
    idx = np.arange(N * N)
    xp = [(idx % N + 1) % N + N * (idx // N), idx % N + N * ((idx // N + 1) % N)]
    U2 = np.stack([Om @ Um[d] @ dag(Om[xp[d]]) for d in range(2)])
    alg = lambda X: np.einsum("na,aij->nij", X, T)
    E2 = np.stack([comp(Om @ alg(E[d]) @ dag(Om)) for d in range(2)])
    return (orc.m2d(U2).copy(), np.ascontiguousarray(E2), comp(Om @ alg(phi) @ dag(Om)),
            comp(Om @ alg(pi) @ dag(Om)))


def test_evolution_gauge_covariant(orc):
    N, dt = 6, 0.125
    U, E, phi, pi = si.random_state(8, N, link_kind="near", eps=0.5)
    Om = si.haar_su3(si.rng(9), N * N)
    a, b = orc.State(N), orc.State(N)
    a.U, a.E, a.phi, a.pi, a.n = U, E, phi, pi, 2
    b.U, b.E, b.phi, b.pi = _gauge_transform(orc, N, Om, U, E, phi, pi)
    b.n = 2
    for _ in range(10):
        orc.field_step(a, dt)
        orc.field_step(b, dt)
    ta = _gauge_transform(orc, N, Om, a.U, a.E, a.phi, a.pi)
    for x, y in zip(ta, (b.U, b.E, b.phi, b.pi)):
        assert np.abs(x - y).max() < 1e-12


def test_site_sampler_matches_full_step(orc):
    N, dt = 8, 0.125
    U, E, phi, pi = si.random_state(10, N, link_kind="haar")
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 4
    sites = np.array([0, 7, 9, 56, 63, 27], np.int32)
    Un, En, phin, pin, Fs = orc.field_step_sites(s, dt, sites)
    full = s.copy()
    F = orc.field_step(full, dt, want_F=True)
    assert np.abs(Un - np.transpose(full.U, (1, 0, 2))[sites]).max() < 1e-14
    assert np.abs(En - np.transpose(full.E, (1, 0, 2))[sites]).max() < 1e-14
    assert np.abs(phin - full.phi[sites]).max() < 1e-14
    assert np.abs(pin - full.pi[sites]).max() < 1e-14
    assert np.abs(Fs - F[sites]).max() < 1e-14


def test_site_fields_of_uniform_abelian_fields(orc):
    """Uniform T^3 fields give site fields Ex = E1/tau, Ez = pi, and the
    flux-quantised links U_1 = exp(-i b y T^3) a uniform Bz = -2 sin(b/2) T^3."""
    N, dt = 8, 0.125
    s = orc.State(N)
    s.U[:] = orc.m2d(np.eye(3))
    s.E[0, :, 2] = 0.3
    s.pi[:, 2] = 0.2
    s.n = 4
    F = orc.field_step(s, dt, want_F=True)
    tau = 4 * dt
    assert np.abs(F[:, 0, 2] - 0.3 / tau).max() < 1e-14
    assert np.abs(F[:, 2, 2] - 0.2).max() < 1e-14
    assert np.abs(np.delete(F.reshape(-1, 48), [2, 18], axis=1)).max() < 1e-14
    b = 4 * np.pi * 1 / N
    s = orc.State(N)
    ys = np.arange(N * N) // N
    for x in range(N * N):
        s.U[0, x] = orc.m2d(np.diag(np.exp(-1j * b * ys[x] * np.array([0.5, -0.5, 0]))))
        s.U[1, x] = orc.m2d(np.eye(3))
    s.n = 4
    F = orc.field_step(s, dt, want_F=True)
    assert np.abs(F[:, 5, 2] + 2 * np.sin(b / 2)).max() < 1e-13
    rest = F.copy()
    rest[:, 5, 2] = 0
    assert np.abs(rest).max() < 1e-13
