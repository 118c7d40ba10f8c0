"""The paper's parameter scans with event statistics (Sec. 2, "Heavy
quarks" and "Jets", Figs. 1 and 2).

* Heavy quarks (Fig. 1): beauty quarks with initial transverse momentum
  p_T(tau_form) in {0, 2, 5, 10} GeV, formed at tau_form = 1/(2 m_T):
  <dp_T^2>, <dp_L^2>, their ratio and kappa_T, kappa_L against
  delta tau = tau - tau_form, beside static quarks (Eq. (4)) started at
  the formation step of the beauty quarks at rest, so that the static and
  dynamical curves share the delta tau axis.
* Jets (Fig. 2): quarks formed at tau_form = 0 moving along x with
  p_x(tau_form) in {1, 2, 5, 10} GeV for several masses, labelled by p_x / m:
  <dp_y^2>, <dp_z^2>, their ratio and qhat_y, qhat_z, beside lightlike jets
  (Eq. (5)).

Every scan point is one particle species of every event, so all points see
the same Glasma backgrounds.  Each event runs the coupled solver with both
field correlators (gl_run), and the observables are averaged over the
particles and the events with delete-one jackknife errors over the events
(gl_scan_statistics).  Everything numerical runs in libglasma.so; this module
sets the events up and collects their series.
"""
import math
import time

import numpy as np

from . import glasma as G

BEAUTY_GEV = 4.18
HEAVY_PT_GEV = (0.0, 2.0, 5.0, 10.0)
JET_PX_GEV = (1.0, 2.0, 5.0, 10.0)
# The paper does not list the jet masses of Fig. 2; the workloads' charm
# and beauty masses span p_x / m from 0.24 to 7.9.
JET_MASSES_GEV = (1.27, 4.18)
# the paper's totals, quoted for context (its lattice and normalisations are
# not given): kappa_peak 19-22 GeV^2/fm at delta tau 0.03-0.05 fm/c for the
# beauty quarks, qhat_peak 24-30 GeV^2/fm at tau 0.04 fm/c for the jets
PAPER_KAPPA_PEAK = (19.0, 22.0)
PAPER_KAPPA_PEAK_DTAU = (0.03, 0.05)
PAPER_QHAT_PEAK = (24.0, 30.0)
PAPER_QHAT_PEAK_TAU = 0.04


def scan_points():
    """(label, kind, mass [GeV], p0 [GeV], tau_form [fm] (< 0: 1/(2 m_T)))"""
    pts = [("beauty pT=%g" % pt, G.KIND_HEAVY_QUARK, BEAUTY_GEV, pt, -1.0) for pt in HEAVY_PT_GEV]
    for m in JET_MASSES_GEV:
        for px in JET_PX_GEV:
            pts.append(("jet px=%g m=%g (px/m=%.3g)" % (px, m, px / m), G.KIND_JET, m, px, 0.0))
    return pts


def _correlator_series(rows, a_fm, n_rows):
    """Correlator rows (tau_{k+3/2} [fm], <dp_x^2>, <dp_y^2>, <dp_z^2> [GeV^2],
    sites) back to the raw series layout: sums over the sites in lattice
    units (GeV^2 times a^2) and the site count, at row k."""
    a_gev = a_fm / G.HBARC_GEV_FM
    s = np.zeros((n_rows, 4))
    k = np.rint(rows[:, 0] / (0.125 * a_fm) - 1.5).astype(int)
    s[k, :3] = rows[:, 1:4] * a_gev ** 2 * rows[:, 4:5]
    s[k, 3] = rows[:, 4]
    return s


def run_scan(n_events=16, N=512, L_fm=10.0, sheets=50, g2mu=2.767, m_ir=0.2, n_per=100000, precision=64,
             seed=2307079995, tau_max=1.0, keep_events=False):
    """Run the scan: n_events MV events, each with every scan point as a
    species of n_per particles, the lightlike correlator from tau = 0 (the
    jets' formation) and the static one from the formation step of the
    beauty quarks at rest, coupled to tau_max.  Event e draws its charges and particles with seed + e.
    Returns a dict with the per-event raw series, the statistics of every
    point and correlator (gl_scan_statistics rows) and the wall time."""
    import torch
    if n_events < 2:
        raise ValueError("the jackknife errors need n_events >= 2")
    pts = scan_points()
    a_fm = L_fm / N
    steps = int(math.ceil(tau_max / (0.125 * a_fm) - 1e-9)) - 1
    series, stat_s, ll_s, nforms = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in range(n_events):
        ev = G.Event(N, L_fm, 0.125, precision=precision, max_steps=steps, max_particles=n_per * len(pts),
                     static_correlator=True, lightlike_correlator=True)
        ev.init_glasma(g2mu, m_ir, sheets, seed + e)
        for (_, kind, m, p0, tf) in pts:
            ev.add_species(m, p0, kind, n_per, seed + e, tau_form_fm=tf)
        # Eq. (4) integrates from the static quarks' start; the figure sets
        # it on the delta tau axis of the dynamical quarks, so it starts on
        # the formation step of the beauty quarks with p_T0 = 0 (point 0)
        n_static = ev.species_info(0)[0]
        ev.static_start(n_static * 0.125 * a_fm)
        ev.lightlike_start(0.0)
        ev.run(steps)
        ser = ev.series()
        series.append(ser[:, :len(pts), :].copy())
        stat_s.append(_correlator_series(ev.static_broadening(), a_fm, steps))
        ll_s.append(_correlator_series(ev.lightlike_broadening(), a_fm, steps))
        if e == 0:
            nforms = [ev.species_info(k)[0] for k in range(len(pts))]
        ev.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    series = np.stack(series)           # [events][rows][points][4]
    dt_fm = 0.125 * a_fm
    out = {"n_events": n_events, "N": N, "L_fm": L_fm, "sheets": sheets, "g2mu_GeV": g2mu,
           "particles_per_point": n_per, "precision": precision, "coupled_steps": steps,
           "points": [p[0] for p in pts], "wall_s": wall, "s_per_event": wall / n_events,
           "particle_steps_per_s": n_events * n_per * len(pts) * steps / wall,
           "stats": [], "static": None, "lightlike": None,
           "static_start_fm": n_static * dt_fm}
    for k, (label, kind, m, p0, tf) in enumerate(pts):
        out["stats"].append(G.scan_statistics(series[:, :, k, :], kind, dt_fm, a_fm))
    out["nform"] = nforms
    out["static"] = G.scan_statistics(np.stack(stat_s), G.KIND_HEAVY_QUARK, dt_fm, a_fm)
    out["lightlike"] = G.scan_statistics(np.stack(ll_s), G.KIND_JET, dt_fm, a_fm)
    if keep_events:
        out["series"] = series
        out["static_series"] = np.stack(stat_s)
        out["lightlike_series"] = np.stack(ll_s)
    return out


def _peak(rows, tau0):
    """Largest total rate of a statistics table, its error and its time
    after tau0 (the particles' start)."""
    if len(rows) == 0:
        return None
    i = int(np.argmax(rows[:, 12]))
    return {"total": float(rows[i, 12]), "err": float(rows[i, 13]), "tau_fm": float(rows[i, 1]),
            "dtau_fm": float(rows[i, 1] - tau0)}


def _at(rows, tau, col):
    if len(rows) == 0:
        return None
    i = int(np.argmin(np.abs(rows[:, 0] - tau)))
    return [float(rows[i, col]), float(rows[i, col + 1])]


def _late(rows, tau0):
    """After the peak of the total rate: the lowest longitudinal rate
    d<B>/dtau (kappa_L or qhat_z; value, error, delta tau after tau0) and
    both rates at the last row (value, error)."""
    if len(rows) == 0:
        return None
    i = int(np.argmax(rows[:, 12]))
    j = i + int(np.argmin(rows[i:, 10]))
    return {"rate_B_min": [float(rows[j, 10]), float(rows[j, 11])], "rate_B_min_dtau_fm": float(rows[j, 1] - tau0),
            "rate_A_end": [float(rows[-1, 8]), float(rows[-1, 9])],
            "rate_B_end": [float(rows[-1, 10]), float(rows[-1, 11])]}


def _curve(rows, tau0):
    return {"peak": _peak(rows, tau0), "ratio_at_0.3fm": _at(rows, tau0 + 0.3, 6),
            "A_end": _at(rows, rows[-1, 0], 2) if len(rows) else None,
            "B_end": _at(rows, rows[-1, 0], 4) if len(rows) else None,
            "late": _late(rows, tau0)}


def summary(res):
    """Per scan point: the peak of the total rate (value, jackknife error,
    delta tau after the start), the anisotropy <B>/<A> at delta tau = 0.3 fm
    (the end of the Glasma stage the paper names), the broadenings at the
    last step and the late rates (the lowest longitudinal rate after the
    peak, both rates at the last step: the paper reports kappa_T and qhat_y
    levelling off at zero while kappa_L and qhat_z turn negative); the same
    for the two correlators, timed from their own starts."""
    pts = scan_points()
    out = {}
    for k, (label, kind, m, p0, tf) in enumerate(pts):
        # delta tau counts from the formation time itself (the particles
        # start at the first step at or after it)
        tau0 = tf if tf >= 0 else G.HBARC_GEV_FM / (2.0 * math.hypot(m, p0))
        out[label] = _curve(res["stats"][k], tau0)
    for name, tau0 in (("static", res["static_start_fm"]), ("lightlike", 0.0)):
        out[name] = _curve(res[name], tau0)
    return out
