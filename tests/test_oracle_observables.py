"""Pins of the observable post-processing (Eq. (3)): the central difference
of a quadratic broadening history is exact, and the unit conversion follows
from hbar c."""
import numpy as np


def test_central_difference_exact_on_quadratic(orc):
    dt, nform, steps = 0.125, 3, 20
    # <dp^2> = c (tau_h - tau_f)^2 sampled on the half-step grid, zero before formation
    c = np.array([0.7, -0.2, 1.3])
    series = np.zeros((steps, 4))
    tau_f = (nform + 1 - 0.5) * dt      # first active row is n = nform (k = nform - 1)
    for k in range(steps):
        n = k + 1
        if n < nform:
            continue
        tau_h = (n + 0.5) * dt
        series[k, :3] = 10 * c * (tau_h - tau_f + dt) ** 2
        series[k, 3] = 10
    ks, rates = orc.coefficients(series, dt)
    assert ks[0] == nform - 1
    for k, r in zip(ks[1:], rates[1:]):
        tau_n = (k + 1) * dt
        assert np.abs(r - 2 * c * (tau_n - tau_f + dt)).max() < 1e-12
    # the formation row differences against zero
    assert np.abs(rates[0] - series[nform - 1, :3] / 10 / dt).max() < 1e-12


def test_unit_conversion():
    from oracle import oracle as O
    a_fm = 0.125
    a_gev = a_fm / 0.1973269804
    f2, fk = O.to_physical(a_fm)
    assert abs(f2 * a_gev ** 2 - 1) < 1e-15
    assert abs(fk * a_gev ** 2 * a_fm - 1) < 1e-15
