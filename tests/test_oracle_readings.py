"""Pins of two readings of the paper that no other pin sees: the sign of the
transverse magnetic site fields B_x, B_y (built from the covariant gradient
of phi = A_eta) and the direction of the colour rotation along eta.

Both are fixed against consequences of Eq. (2) that do not go through the
oracle's own formulas:

* Translation invariance in eta makes the canonical longitudinal momentum
  P_eta - Q^a A_eta^a a constant of the motion (Noether).  In an abelian field
  phi^3(x, tau) T^3 it changes only through the electric part (d phi / d tau,
  i.e. E_z, whose sign the constant-E_z pin fixes) and the magnetic part
  (v_i d phi / d x_i, i.e. B_y and B_x).  A sign flip of B_x or B_y breaks the
  conservation by twice the spatial part.
* The colour equation of Eq. (2), dQ/dtau = -i [A_mu, Q] dx^mu/dtau, with
  A_eta = phi gives dQ/deta = -i [phi, Q] for a move along eta.  A charge
  carried around a closed (x, eta) loop must then come back conjugated by the
  loop's holonomy, built from the same link convention U = exp(+i A a) as the
  transverse links (the transverse plaquette loop does the same).

The matrices the tests compare against are built here with numpy and scipy
from the textbook Gell-Mann generators, not with the oracle's exponential."""
import numpy as np
import pytest
import scipy.linalg

from tests import seeded_inputs as si

DT = 0.125


def _gell_mann():
    """T^a = lambda^a / 2 (textbook Gell-Mann matrices)."""
    l = np.zeros((8, 3, 3), np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l / 2


T = _gell_mann()


def _mat(x8):
    return np.einsum("a,aij->ij", x8, T)


def _comps(M):
    return np.array([2 * np.real(np.trace(T[a] @ M)) for a in range(8)])


def _Q0():
    """Diagonal charge with q2 = 4 and q3 = 10/3: it commutes with T^3 fields."""
    lam = np.sort(np.real(np.roots([1.0, 0.0, -1.0, -5.0 / 18.0])))[::-1]
    return _comps(np.diag(lam).astype(np.complex128))


def test_gell_mann_basis_matches_oracle_generators(orc):
    for a in range(8):
        assert np.abs(orc.generator(a) - T[a]).max() < 1e-15


def _abelian_scalar_state(orc, N, n0, eps, k, axis):
    """U = 1, E = pi = 0, phi^3 = eps sin(theta x_axis), theta = 2 pi k / N."""
    s = orc.State(N)
    s.U[:] = orc.m2d(np.eye(3))
    xs = np.arange(N * N) % N if axis == 0 else np.arange(N * N) // N
    theta = 2 * np.pi * k / N
    s.phi[:, 2] = eps * np.sin(theta * xs)
    s.n = n0
    return s, xs, theta


@pytest.mark.parametrize("axis", [0, 1])
def test_site_magnetic_field_of_a_scalar_gradient(orc, axis):
    """phi^3 = eps sin(theta x) with U = 1: the central covariant difference is
    eps sin(theta) cos(theta x), so B_y = +D_x phi / tau (F_{x eta} = d_x A_eta
    over tau); for a y mode B_x = -D_y phi / tau.  Everything else vanishes
    except E_z, the time-averaged pi built by the phi Laplacian."""
    N, n0, eps, k = 24, 5, 0.07, 2
    s, xs, theta = _abelian_scalar_state(orc, N, n0, eps, k, axis)
    tau = n0 * DT
    F = orc.field_step(s, DT, want_F=True)
    grad = eps * np.sin(theta) * np.cos(theta * xs)
    if axis == 0:
        assert np.abs(F[:, 4, 2] - grad / tau).max() < 1e-15        # B_y^3
        assert np.abs(F[:, 3]).max() < 1e-15                        # B_x
    else:
        assert np.abs(F[:, 3, 2] + grad / tau).max() < 1e-15        # B_x^3
        assert np.abs(F[:, 4]).max() < 1e-15                        # B_y
    # E_z = (pi^{n-1/2} + pi^{n+1/2}) / 2 with pi^{n+1/2} = dtau / tau Lap phi
    lap = -4 * np.sin(theta / 2) ** 2 * eps * np.sin(theta * xs)
    assert np.abs(F[:, 2, 2] - 0.5 * DT / tau * lap).max() < 1e-15
    rest = F.copy()
    rest[:, 2, 2] = rest[:, 3, 2] = rest[:, 4, 2] = 0
    assert np.abs(rest).max() < 1e-15


def _canonical_drift(orc, axis, flip_check=False):
    """Run one particle across an abelian phi^3 mode; return the change of
    P_eta and of the canonical momentum P_eta - Q^3 phi^3(X(tau), tau)."""
    N, n0, eps, k, steps = 64, 8, 0.3, 1, 160
    s, xs, theta = _abelian_scalar_state(orc, N, n0, eps, k, axis)
    Q = _Q0()
    m = 0.3
    P = orc.Particles(1)
    cell = [20, 11] if axis == 0 else [11, 20]
    P.cell[0] = cell
    p = np.zeros(3)
    p[axis] = 0.9
    P.p[0] = p
    P.p0[0] = (p[0], p[1], 0.0)
    P.Q[0] = Q

    def amp(st):
        basis = np.sin(theta * xs)
        return float(st.phi[:, 2] @ basis / (basis @ basis))

    def pos(PP):
        return float(PP.cell[0, axis] + PP.off[0, axis])

    # the kicks at tau_{n0} .. tau_{n0+K-1} integrate the scalar's change
    # along the path from tau_{n0-1/2} to tau_{n0+K-1/2}: take both ends at
    # those half steps (the start backed up by half a step of the same drift)
    A, X = [amp(s)], [pos(P)]
    for _ in range(steps):
        U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
        F = orc.field_step(s, DT, want_F=True)
        orc.particle_step(N, n, DT, U0, phi0, F, P, [m], [0])
        A.append(amp(s))
        X.append(pos(P))
    phi_at = lambda a, x: a * np.sin(theta * x)
    start = phi_at(1.5 * A[0] - 0.5 * A[1], 1.5 * X[0] - 0.5 * X[1])
    end = phi_at(0.5 * (A[-2] + A[-1]), 0.5 * (X[-2] + X[-1]))
    dphi = Q[2] * (end - start)
    A0, X0, X_now = A[0], X[0], X[-1]
    dP = float(P.p[0, 2])
    return dP, dP - dphi, Q[2] * A0 * (np.sin(theta * X_now) - np.sin(theta * X0))


@pytest.mark.parametrize("axis", [0, 1])
def test_canonical_longitudinal_momentum_is_conserved(orc, axis):
    """Noether charge of eta translations: P_eta - Q^a phi^a at the particle
    stays constant while the particle crosses a third of an abelian phi mode
    that also evolves in time.  The change of P_eta is dominated by the
    magnetic (spatial-gradient) part, so a flipped B_y (axis x) or B_x (axis y)
    would break the balance by twice that part."""
    dP, drift, spatial = _canonical_drift(orc, axis)
    print("axis %d: dP_eta %.4e, canonical drift %.2e, spatial part %.4e" % (axis, dP, drift, spatial))
    assert abs(spatial) > 0.5 * abs(dP) > 0
    assert abs(drift) < 0.01 * abs(dP)


def test_eta_rotation_direction_is_eq2_colour_equation(orc):
    """A move by a small d_eta in a cell with scalar phi rotates the charge by
    dQ = -i [phi, Q] d_eta (Eq. (2) with A_eta = phi); no force (F = 0) and no
    transverse motion, so nothing else touches Q."""
    N, n = 6, 7
    g = si.rng(31)
    U = si.mats_to_d(si.haar_su3(g, 2 * N * N)).reshape(2, N * N, 18)
    phi = 0.6 * g.normal(size=(N * N, 8))
    F = np.zeros((N * N, 6, 8))
    Q = si.random_algebra(32, 1)[0]
    P = orc.Particles(1)
    P.cell[0] = (2, 3)
    m, vz = 0.5, 1e-4
    th = (n + 0.5) * DT
    P.p[0] = (0.0, 0.0, vz * m / np.sqrt(1 - vz * vz) * th)
    P.Q[0] = Q
    orc.particle_step(N, n, DT, U, phi, F, P, [m], [0])
    deta = P.eta[0]
    assert abs(deta - DT * vz / th) < 1e-15
    x = 2 + N * 3
    Pm, Qm = _mat(phi[x]), _mat(Q)
    want = -1j * (Pm @ Qm - Qm @ Pm)
    got = (P.Q[0] - Q) / deta
    # second order term: deta * |phi|^2 |Q| / 2
    assert np.abs(got - _comps(want)).max() < 5 * deta * np.abs(phi[x]).max() ** 2 * np.abs(Q).max() * 8
    assert np.abs(_comps(want)).max() > 0.1


def _set_eta_velocity(P, m, th, deta):
    """P_eta giving the rapidity step deta over dtau at tau_{n+1/2} = th."""
    v = deta * th / DT
    P.p[0] = (0.0, 0.0, v * m / np.sqrt(1 - v * v) * th)


def test_charge_around_a_closed_x_eta_loop(orc):
    """Carry a charge around the closed loop x -> x+1 (link crossing) ->
    eta + d_eta (at x+1) -> x (crossing back) -> eta - d_eta (at x).  It must
    return as P^dag Q P with the loop holonomy
    P = U_x(x) exp(i phi(x+1) d_eta) U_x(x)^dag exp(-i phi(x) d_eta),
    the eta links taken in the same exp(+i A a) convention as the transverse
    links, exactly as the transverse plaquette loop returns P^dag Q P.  The
    opposite rotation sense returns the charge conjugated by another matrix."""
    N, n0 = 6, 9
    g = si.rng(41)
    U = si.mats_to_d(si.haar_su3(g, 2 * N * N)).reshape(2, N * N, 18)
    phi = 0.8 * g.normal(size=(N * N, 8))
    F = np.zeros((N * N, 6, 8))
    Q = si.random_algebra(42, 1)[0]
    m = 0.5
    P = orc.Particles(1)
    P.cell[0] = (2, 3)
    P.off[0] = (0.45, 0.0)
    P.Q[0] = Q
    x = 2 + N * 3
    xp = 3 + N * 3
    # 1: cross +x (no eta motion)
    P.p[0] = (2.0, 0.0, 0.0)
    orc.particle_step(N, n0, DT, U, phi, F, P, [m], [0])
    assert tuple(P.cell[0]) == (3, 3) and P.eta[0] == 0.0
    # 2: move in eta at x+1 (no transverse motion)
    _set_eta_velocity(P, m, (n0 + 1.5) * DT, 0.06)
    orc.particle_step(N, n0 + 1, DT, U, phi, F, P, [m], [0])
    d_eta = P.eta[0]
    assert abs(d_eta - 0.06) < 1e-12 and tuple(P.cell[0]) == (3, 3)
    # 3: cross back to x
    P.p[0] = (-2.0, 0.0, 0.0)
    orc.particle_step(N, n0 + 2, DT, U, phi, F, P, [m], [0])
    assert tuple(P.cell[0]) == (2, 3)
    # 4: move back in eta by exactly d_eta at x
    _set_eta_velocity(P, m, (n0 + 3.5) * DT, -d_eta)
    orc.particle_step(N, n0 + 3, DT, U, phi, F, P, [m], [0])
    assert abs(P.eta[0]) < 1e-14
    Ux = orc.d2m(U[0, x])
    hol = Ux @ scipy.linalg.expm(1j * d_eta * _mat(phi[xp])) @ Ux.conj().T @ \
        scipy.linalg.expm(-1j * d_eta * _mat(phi[x]))
    want = _comps(hol.conj().T @ _mat(Q) @ hol)
    assert np.abs(P.Q[0] - want).max() < 1e-13
    # the other rotation sense is a different holonomy: the pin can tell
    alt = Ux @ scipy.linalg.expm(-1j * d_eta * _mat(phi[xp])) @ Ux.conj().T @ \
        scipy.linalg.expm(1j * d_eta * _mat(phi[x]))
    assert np.abs(_comps(alt.conj().T @ _mat(Q) @ alt) - want).max() > 1e-2


def test_transverse_plaquette_loop_uses_the_same_convention(orc):
    """The reference for the loop above: a charge carried around the
    transverse plaquette x -> x+1 -> x+1+2 -> x+2 -> x by link crossings
    returns as P^dag Q P with P = U_1(x) U_2(x+1) U_1(x+2)^dag U_2(x)^dag."""
    N, n0 = 6, 9
    g = si.rng(43)
    U = si.mats_to_d(si.haar_su3(g, 2 * N * N)).reshape(2, N * N, 18)
    phi = np.zeros((N * N, 8))
    F = np.zeros((N * N, 6, 8))
    Q = si.random_algebra(44, 1)[0]
    P = orc.Particles(1)
    P.cell[0] = (2, 3)
    P.off[0] = (0.45, 0.45)
    P.Q[0] = Q
    moves = [(2.0, 0.0), (0.0, 2.0), (-2.0, 0.0), (0.0, -2.0)]
    cells = [(3, 3), (3, 4), (2, 4), (2, 3)]
    for k, ((px, py), c) in enumerate(zip(moves, cells)):
        P.p[0] = (px, py, 0.0)
        orc.particle_step(N, n0 + k, DT, U, phi, F, P, [0.5], [0])
        assert tuple(P.cell[0]) == c
    L = lambda d, ix, iy: orc.d2m(U[d, ix % N + N * (iy % N)])
    Pl = L(0, 2, 3) @ L(1, 3, 3) @ L(0, 2, 4).conj().T @ L(1, 2, 3).conj().T
    want = _comps(Pl.conj().T @ _mat(Q) @ Pl)
    assert np.abs(P.Q[0] - want).max() < 1e-13
