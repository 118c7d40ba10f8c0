"""Pins of the oracle's particle solver (Wong's equations with link-built
color rotations): charge ensemble moments, Casimir conservation, free
streaming, Lorentz-force closed forms in constant abelian fields, the static
(m -> infinity) limit, and gauge invariance of the broadening."""
import numpy as np
import pytest

from tests import seeded_inputs as si

DT = 0.125


def _Q0_components(orc):
    """Diagonal charge with q2 = 4, q3 = 10/3 (roots of l^3 - l - 5/18)."""
    lam = np.sort(np.real(np.roots([1.0, 0.0, -1.0, -5.0 / 18.0])))[::-1]
    M = np.diag(lam).astype(np.complex128)
    T = np.array([orc.generator(a) for a in range(8)])
    return np.array([2 * np.real(np.trace(T[a] @ M)) for a in range(8)])


def _casimirs(orc, Q):
    d = np.array([[[orc.dsym(a, b, c) for c in range(8)] for b in range(8)] for a in range(8)])
    return np.einsum("na,na->n", Q, Q), np.einsum("abc,na,nb,nc->n", d, Q, Q, Q)


def test_charge_ensemble_moments(orc):
    """<Q^a> = 0, <Q^a Q^b> = delta/2, <Q^a Q^b Q^c> = d_abc/4 (Sec. 1)."""
    n = 100000
    P = orc.particles_init(16, 7, 0, 0, 0.0, n)
    Q = P.Q
    q2, q3 = _casimirs(orc, Q[:2000])
    assert np.abs(q2 - 4.0).max() < 1e-13
    assert np.abs(q3 - 10.0 / 3.0).max() < 1e-13
    sd1 = np.sqrt(0.5 / n)
    assert np.abs(Q.mean(0)).max() < 5 * sd1
    C2 = Q.T @ Q / n
    assert np.abs(C2 - 0.5 * np.eye(8)).max() < 5 * np.sqrt(4.0 / n)
    d = np.array([[[orc.dsym(a, b, c) for c in range(8)] for b in range(8)] for a in range(8)])
    C3 = np.einsum("na,nb,nc->abc", Q, Q, Q) / n
    assert np.abs(C3 - d / 4).max() < 5 * np.sqrt(8.0 / n)


def test_particle_positions_and_momenta(orc):
    N, n = 32, 20000
    P = orc.particles_init(N, 3, 1, 0, 0.4, n)
    assert P.cell.min() >= 0 and P.cell.max() < N
    assert P.off.min() >= -0.5 and P.off.max() < 0.5
    pos = (P.cell + P.off) % N
    assert abs(pos.mean() - N / 2 + 0.5 / 1) < 5 * N / np.sqrt(12 * n) + 0.5
    assert np.allclose(np.hypot(P.p[:, 0], P.p[:, 1]), 0.4, atol=1e-15)
    assert np.all(P.p[:, 2] == 0) and np.all(P.eta == 0)
    phi = np.arctan2(P.p[:, 1], P.p[:, 0])
    assert abs(np.cos(phi).mean()) < 5 / np.sqrt(2 * n)
    J = orc.particles_init(N, 3, 2, 1, 0.9, 100)
    assert np.all(J.p[:, 0] == 0.9) and np.all(J.p[:, 1] == 0)


def _coupled(orc, s, P, steps, mass, nform):
    rows, Fs = [], []
    for _ in range(steps):
        U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
        F = orc.field_step(s, DT, want_F=True)
        rows.append(orc.particle_step(s.N, n, DT, U0, phi0, F, P, mass, nform))
        Fs.append(F)
    return np.array(rows), Fs


def _single(orc, N, cell, off, p, Q):
    P = orc.Particles(1)
    P.cell[0] = cell
    P.off[0] = off
    P.p[0] = p
    P.p0[0] = (p[0], p[1], 0.0)
    P.Q[0] = Q
    return P


def _empty_state(orc, N, n0):
    s = orc.State(N)
    s.U[:] = orc.m2d(np.eye(3))
    s.n = n0
    return s


def test_free_streaming(orc):
    """Zero field (U = 1, E = phi = pi = 0): momenta and charge constant,
    straight transverse lines, no transverse broadening, and a lab p_z that is
    conserved up to the O(dtau^2) of the rapidity drift."""
    N, n0, steps = 16, 3, 40
    s = _empty_state(orc, N, n0)
    Q0 = si.random_algebra(1, 1)[0]
    for m, p in ((0.5, (0.3, -0.2, 0.05)), (0.0, (1.0, 0.0, 0.0))):
        P = _single(orc, N, (4, 5), (0.1, -0.2), p, Q0)
        rows, _ = _coupled(orc, s.copy(), P, steps, [m], [0])
        assert np.abs(P.p[0] - np.array(p)).max() < 1e-15
        assert np.abs(P.Q[0] - Q0).max() < 1e-13
        assert np.abs(rows[:, 0, :2]).max() < 1e-15
        tau_h = (n0 + np.arange(steps) + 0.5) * DT
        ptau = np.sqrt(m * m + p[0] ** 2 + p[1] ** 2 + (p[2] / tau_h) ** 2)
        x = 4 + 0.1 + np.sum(DT * p[0] / ptau)
        pos = P.cell[0, 0] + P.off[0, 0]
        assert abs((pos - x + N / 2) % N - N / 2) < 1e-12
    m, p = 0.5, (0.3, -0.2, 0.05)
    errs = []
    for k in (1, 2, 4):
        dt = DT / k
        sk = _empty_state(orc, N, n0 * k)
        P = _single(orc, N, (4, 5), (0.1, -0.2), p, Q0)
        for _ in range(steps * k):
            U0, phi0, n = sk.U.copy(), sk.phi.copy(), sk.n
            F = orc.field_step(sk, dt, want_F=True)
            row = orc.particle_step(N, n, dt, U0, phi0, F, P, [m], [0])
        errs.append(abs(np.sqrt(row[0, 2]) - p[2] / (n0 * DT)))
    assert errs[0] < 2e-2 * p[2] / (n0 * DT)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_constant_transverse_electric_field(orc):
    """Uniform E_1 = eps T^3: p_x = p_x0 + Q^3 eps sum dtau/tau_n (exact for the
    scheme) = Q^3 eps ln(tau/tau0) + O(dtau^2)."""
    N, n0, eps = 16, 4, 0.05
    Q = _Q0_components(orc)
    res = []
    for dt_scale in (1, 2, 4):
        dt = DT / dt_scale
        s = _empty_state(orc, N, n0 * dt_scale)
        s.E[0, :, 2] = eps
        P = _single(orc, N, (3, 3), (0.0, 0.0), (0.0, 0.0, 0.0), Q)
        steps = 24 * dt_scale
        for _ in range(steps):
            U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
            F = orc.field_step(s, dt, want_F=True)
            orc.particle_step(N, n, dt, U0, phi0, F, P, [1.0], [0])
        ns = np.arange(n0 * dt_scale, n0 * dt_scale + steps)
        exact_sum = Q[2] * eps * np.sum(dt / (ns * dt))
        assert abs(P.p[0, 0] - exact_sum) < 1e-13
        assert abs(P.p[0, 1]) < 1e-15 and abs(P.p[0, 2]) < 1e-15
        assert np.abs(P.Q[0] - Q).max() < 1e-12
        t0, t1 = (n0 - 0.5 / dt_scale) * DT, (n0 + 24 - 0.5 / dt_scale) * DT
        res.append(abs(P.p[0, 0] - Q[2] * eps * np.log(t1 / t0)))
    assert res[0] / res[1] > 3.0 and res[1] / res[2] > 3.0


def test_constant_longitudinal_electric_field(orc):
    """Uniform E_z = pi = eps T^3: hyperbolic motion, lab p_z = Q^3 eps (t - t0)."""
    N, n0, eps, m = 8, 4, 0.08, 0.7
    Q = _Q0_components(orc)
    errs = []
    for k in (1, 2, 4):
        dt = DT / k
        s = _empty_state(orc, N, n0 * k)
        s.pi[:, 2] = eps
        P = _single(orc, N, (2, 2), (0.0, 0.0), (0.0, 0.0, 0.0), Q)
        rows = []
        steps = 40 * k
        for _ in range(steps):
            U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
            eta_before = P.eta[0]
            F = orc.field_step(s, dt, want_F=True)
            rows.append(orc.particle_step(N, n, dt, U0, phi0, F, P, [m], [0]))
        tau_end = (n0 * k + steps - 0.5) * dt
        pz = np.sqrt(rows[-1][0, 2]) * np.sign(Q[2] * eps)
        # lab time of the last half step, at the mean of the last two rapidities
        t = tau_end * np.cosh(0.5 * (eta_before + P.eta[0]))
        t0 = (n0 * k - 0.5) * dt
        errs.append(abs(pz - Q[2] * eps * (t - t0)))
        assert np.abs(P.Q[0] - Q).max() < 1e-12
    assert errs[0] < 2e-2 * abs(Q[2] * eps * 40 * DT)
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5


def test_constant_magnetic_field_circular_orbit(orc):
    """Flux-quantised links U_1 = exp(-i b y T^3) give a uniform B_z: the
    momentum turns at the Boris angle 2 atan(b_z dtau / (2 p^tau)) per step,
    clockwise for positive b_z, with |p| conserved."""
    N, n0, steps = 16, 2, 30
    b = 4 * np.pi * 1 / N
    Beff = 2 * np.sin(b / 2)
    Q = _Q0_components(orc)
    s = _empty_state(orc, N, n0)
    ys = np.arange(N * N) // N
    for x in range(N * N):
        s.U[0, x] = orc.m2d(np.diag(np.exp(-1j * b * ys[x] * np.array([0.5, -0.5, 0]))))
    m, p0 = 0.6, 0.8
    P = _single(orc, N, (5, 9), (0.0, 0.0), (p0, 0.0, 0.0), Q)
    _coupled(orc, s, P, steps, [m], [0])
    bz = -Q[2] * Beff
    theta = 2 * np.arctan(bz * DT / (2 * np.hypot(m, p0)))
    ang = np.arctan2(P.p[0, 1], P.p[0, 0])
    assert abs(np.hypot(P.p[0, 0], P.p[0, 1]) - p0) < 1e-13
    wrap = lambda a: (a + np.pi) % (2 * np.pi) - np.pi
    assert abs(wrap(ang - (-steps * theta))) < 1e-12
    omega = bz / np.hypot(m, p0)
    # Boris phase error relative to the cyclotron angle is (omega dtau)^2 / 12
    assert abs(wrap(ang + steps * DT * omega)) < 2 * (omega * DT) ** 2 / 12 * abs(steps * DT * omega)
    assert np.abs(P.Q[0] - Q).max() < 1e-12


def test_static_limit_is_electric_field_integral(orc):
    """m -> infinity: delta p_x = sum_n dtau Q^a E_x^a(tau_n) at the fixed cell,
    the lattice form of Eq. (4) for one charge."""
    N = 12
    s, rc, _ = orc.init_glasma(N, 0.6, 0.016, 1, 77, DT)
    P = orc.particles_init(N, 77, 0, 0, 0.0, 64)
    Q0 = P.Q.copy()
    cells = P.cell.copy()
    rows, Fs = _coupled(orc, s, P, 30, [1e12], [1])
    assert np.array_equal(P.cell, cells)
    idx = cells[:, 0] + N * cells[:, 1]
    for k in (0, 1):
        want = sum(DT * np.einsum("na,na->n", Q0, F[idx, k]) for F in Fs)
        assert np.abs(P.p[:, k] - want).max() < 1e-10
    assert np.abs(P.Q - Q0).max() < 1e-12


def test_casimirs_conserved_in_glasma(orc):
    N = 12
    s, rc, _ = orc.init_glasma(N, 0.8, 0.016, 1, 5, DT)
    P1 = orc.particles_init(N, 5, 0, 1, 1.0, 50)
    P2 = orc.particles_init(N, 5, 1, 0, 0.3, 50)
    P = orc.Particles(100)
    for k in ("cell", "off", "eta", "p", "Q", "p0", "species"):
        getattr(P, k)[:] = np.concatenate([getattr(P1, k), getattr(P2, k)])
    P.species[50:] = 1
    q2a, q3a = _casimirs(orc, P.Q)
    cells = P.cell.copy()
    _coupled(orc, s, P, 60, [0.0, 0.5], [1, 2])
    q2b, q3b = _casimirs(orc, P.Q)
    assert np.abs(q2b - q2a).max() < 1e-12 and np.abs(q3b - q3a).max() < 1e-12
    assert np.any(P.cell != cells)       # the jets crossed cells


def test_broadening_gauge_invariant(orc):
    """A random gauge transformation of the initial fields and charges leaves
    every particle's momentum history unchanged."""
    from tests.test_oracle_fields import _gauge_transform
    N = 10
    s, rc, _ = orc.init_glasma(N, 0.7, 0.016, 1, 11, DT)
    # evolve a few steps first so that E, phi and pi are all non-zero
    for _ in range(3):
        orc.field_step(s, DT)
    P = orc.particles_init(N, 11, 0, 1, 0.9, 40)
    Om = si.haar_su3(si.rng(4), N * N)
    g = s.copy()
    g.U, g.E, g.phi, g.pi = _gauge_transform(orc, N, Om, s.U, s.E, s.phi, s.pi)
    Pg = P.copy()
    T = np.array([orc.generator(a) for a in range(8)])
    idx = P.cell[:, 0] + N * P.cell[:, 1]
    Qm = np.einsum("na,aij->nij", P.Q, T)
    Qg = Om[idx] @ Qm @ np.conj(np.swapaxes(Om[idx], -1, -2))
    Pg.Q = np.ascontiguousarray(2 * np.real(np.einsum("aij,nji->na", T, Qg)))
    ra, _ = _coupled(orc, s, P, 30, [0.3], [1])
    rb, _ = _coupled(orc, g, Pg, 30, [0.3], [1])
    assert np.abs(ra - rb).max() < 1e-12
    assert np.abs(P.p - Pg.p).max() < 1e-12
    assert np.array_equal(P.cell, Pg.cell)


def test_static_correlator_is_charge_average_of_static_quarks(orc):
    """Eq. (4): the correlator sum_a (I_i^a)^2 / 2 at every site equals the
    mean square momentum of static quarks (m -> infinity) over charges with
    <Q^a Q^b> = delta^ab / 2.  The eight charges Q = e_b (unit algebra
    vectors) at every site give sum_b (delta p_i)^2 = sum_b (I_i^b)^2 exactly
    for the transverse momenta; the lab-frame longitudinal momentum of the
    push agrees with the E_z integral to O(dtau^2)."""
    N, steps = 8, 24
    s, rc, _ = orc.init_glasma(N, 0.6, 0.016, 1, 91, DT)
    s2 = s.copy()
    P = orc.Particles(8 * N * N)
    for x in range(N * N):
        for b in range(8):
            i = 8 * x + b
            P.cell[i] = (x % N, x // N)
            P.Q[i, b] = 1.0
    rows, _ = _coupled(orc, s, P, steps, [1e12], [1])
    stat = orc.static_series(s2, DT, steps, n0=1)
    assert np.all(stat[:, 3] == N * N)
    for i in (0, 1):
        assert np.abs(rows[:, 0, i] - 2.0 * stat[:, i]).max() < 1e-10 * np.abs(stat[:, i]).max()
    rel_z = np.abs(rows[:, 0, 2] - 2.0 * stat[:, 2]).max() / np.abs(stat[:, 2]).max()
    print("static limit, longitudinal: max relative difference %.2e" % rel_z)
    assert rel_z < 0.05, rel_z
    # the correlator grows from zero and a later start excludes earlier fields
    s3, _, _ = orc.init_glasma(N, 0.6, 0.016, 1, 91, DT)
    late = orc.static_series(s3, DT, steps, n0=10)
    assert np.all(late[:9, 3] == 0) and np.all(late[9:, 3] == N * N)
    assert np.all(late[:9, :3] == 0) and late[9, 0] < stat[9, 0]


def test_lightlike_correlator_is_charge_average_of_lightlike_jets(orc):
    """Eq. (5): the transported-field correlator equals the mean square
    momentum of massless jets with p_x -> infinity (p_x = 1e12, velocity 1 to
    double precision) started at every site centre, over the eight basis
    charges Q = e_b, so sum_b (delta p_y)^2 = sum_b (I_y^b)^2 exactly; the
    lab-frame longitudinal momentum agrees to O(dtau^2).  The jets cross
    cells every eight steps, so the colour transport is exercised."""
    N, steps = 8, 40
    s, rc, _ = orc.init_glasma(N, 0.6, 0.016, 1, 93, DT)
    s2 = s.copy()
    P = orc.Particles(8 * N * N)
    for x in range(N * N):
        for b in range(8):
            i = 8 * x + b
            P.cell[i] = (x % N, x // N)
            P.Q[i, b] = 1.0
            P.p[i, 0] = P.p0[i, 0] = 1e12
    rows, _ = _coupled(orc, s, P, steps, [0.0], [1])
    ll = orc.lightlike_series(s2, DT, steps, n0=1)
    assert np.all(ll[:, 3] == N * N)
    assert np.abs(rows[:, 0, 1] - 2.0 * ll[:, 1]).max() < 1e-10 * np.abs(ll[:, 1]).max()
    rel_z = np.abs(rows[:, 0, 2] - 2.0 * ll[:, 2]).max() / np.abs(ll[:, 2]).max()
    print("lightlike limit, longitudinal: max relative difference %.2e" % rel_z)
    assert rel_z < 0.05, rel_z
    # the jets moved 5 cells, so the colour transport took part
    assert np.all(P.cell[:, 0] == (np.repeat(np.arange(N * N) % N, 8) + 5) % N)
