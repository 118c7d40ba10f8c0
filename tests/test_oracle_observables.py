"""Pins of the observable post-processing (Eq. (3)): the central difference
of a quadratic broadening history is exact, and the unit conversion follows
from hbar c."""
import numpy as np
import pytest


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


def _synthetic_events(seed, E, rows, first, equal_counts):
    g = np.random.default_rng(seed)
    S = np.zeros((E, rows, 4))
    for e in range(E):
        n = 1000.0 if equal_counts else float(g.integers(500, 1500))
        for k in range(first, rows):
            S[e, k, 3] = n
            S[e, k, :3] = n * (0.1 * (k - first + 1) + g.normal(scale=0.05, size=3) ** 2)
    return S


def test_scan_jackknife_of_linear_observables_is_the_standard_error(orc):
    """For a mean over events with equal counts the delete-one jackknife
    error is exactly the standard error of the per-event means, and the
    pooled mean is the mean of the event means (textbook identities)."""
    E, rows, first = 7, 12, 3
    S = _synthetic_events(3, E, rows, first, True)
    a_fm, dt = 0.05, 0.00625
    out = orc.scan_statistics(S, 0, dt, a_fm)
    f2, fk = orc.to_physical(a_fm)
    assert out.shape == (rows - first, 14)
    means_A = (S[:, first:, 0] + S[:, first:, 1]) / S[:, first:, 3] * f2
    means_B = S[:, first:, 2] / S[:, first:, 3] * f2
    for col, m in ((2, means_A), (4, means_B)):
        assert np.allclose(out[:, col], m.mean(0), rtol=1e-13, atol=0)
        assert np.allclose(out[:, col + 1], m.std(0, ddof=1) / np.sqrt(E), rtol=1e-11, atol=0)
    # rates: per-event central differences (the formation row differences against zero)
    rates_A = np.diff(np.concatenate([np.zeros((E, 1)), means_A], axis=1), axis=1) / (dt / a_fm) * (fk / f2)
    assert np.allclose(out[:, 8], rates_A.mean(0), rtol=1e-12)
    assert np.allclose(out[:, 9], rates_A.std(0, ddof=1) / np.sqrt(E), rtol=1e-10)
    rates_B = np.diff(np.concatenate([np.zeros((E, 1)), means_B], axis=1), axis=1) / (dt / a_fm) * (fk / f2)
    tot = rates_A + rates_B
    assert np.allclose(out[:, 12], tot.mean(0), rtol=1e-12)
    assert np.allclose(out[:, 13], tot.std(0, ddof=1) / np.sqrt(E), rtol=1e-10)
    assert np.allclose(out[:, 0], (np.arange(first, rows) + 1.5) * dt)
    assert np.allclose(out[:, 1], (np.arange(first, rows) + 1) * dt)


def test_scan_jackknife_of_identical_events_has_no_error(orc):
    S1 = _synthetic_events(4, 1, 10, 2, True)
    S = np.repeat(S1, 5, axis=0)
    out = orc.scan_statistics(S, 1, 0.01, 0.1)
    assert np.all(out[:, 3::2] < 1e-9 * (np.abs(out[:, 2::2]) + 1e-300))
    # and the pooled values equal the single event's means and rates
    mean, act = orc.mean_broadening(S1[0])
    f2, fk = orc.to_physical(0.1)
    assert np.allclose(out[:, 2], mean[act, 1] * f2, rtol=1e-13)
    assert np.allclose(out[:, 4], mean[act, 2] * f2, rtol=1e-13)
    ks, rates = orc.coefficients(S1[0], 0.1)
    assert np.allclose(out[:, 8], rates[:, 1] * fk, rtol=1e-12)
    assert np.allclose(out[:, 10], rates[:, 2] * fk, rtol=1e-12)


def test_scan_jackknife_of_a_ratio_by_brute_force(orc):
    """The ratio's jackknife recomputed here from explicit leave-one-out
    pools (unequal counts, so the pooled mean weights events by count)."""
    E, rows, first = 5, 8, 1
    S = _synthetic_events(5, E, rows, first, False)
    out = orc.scan_statistics(S, 0, 0.02, 0.1)
    k = 4
    vals = []
    for i in range(E):
        keep = [e for e in range(E) if e != i]
        A = (S[keep, k, 0] + S[keep, k, 1]).sum() / S[keep, k, 3].sum()
        B = S[keep, k, 2].sum() / S[keep, k, 3].sum()
        vals.append(B / A)
    vals = np.array(vals)
    err = np.sqrt((E - 1) / E * ((vals - vals.mean()) ** 2).sum())
    A = (S[:, k, 0] + S[:, k, 1]).sum() / S[:, k, 3].sum()
    B = S[:, k, 2].sum() / S[:, k, 3].sum()
    row = out[k - first]
    assert abs(row[6] - B / A) < 1e-14 and abs(row[7] - err) < 1e-14


def test_library_scan_statistics_match_oracle(orc):
    """gl_scan_statistics (host code of the library, no GPU needed) against
    the oracle's jackknife on synthetic series, both kinds, and its errors."""
    import paper_2307_07999_amd as g
    for kind, seed in ((0, 6), (1, 7)):
        S = _synthetic_events(seed, 6, 15, 4, kind == 1)
        got = g.glasma.scan_statistics(S, kind, 0.004, 0.08)
        want = orc.scan_statistics(S, kind, 0.004, 0.08)
        assert got.shape == want.shape
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    S = _synthetic_events(8, 3, 6, 1, True)
    S[1, 2, 3] = 0.0                      # an event without particles in one row
    with pytest.raises(g.GlasmaError):
        g.glasma.scan_statistics(S, 0, 0.01, 0.1)
    with pytest.raises(g.GlasmaError):
        g.glasma.scan_statistics(S[:1], 0, 0.01, 0.1)
