"""Learned surrogate of the broadening observables, trained on runs of the
solver itself and falling back to the solver outside its training domain.

Inputs (Q_s [GeV], quark mass [GeV], initial p_T [GeV], formation time
[fm], tau [fm]) map to the total transport coefficient [GeV^2/fm] and the
transverse momentum broadening [GeV^2] at tau: for heavy quarks kappa_T +
kappa_L and <dp_T^2> = <dp_x^2 + dp_y^2>; for massless jets along x the
paper's qhat_y + qhat_z and the broadening transverse to the jet,
<dp_y^2 + dp_z^2>.  Everything numerical runs in libglasma.so: the
solver (batched events) produces the labels, gl_mlp_* trains and evaluates
the network; this module only draws parameters, assembles the (input, label)
rows the solver returns and decides between network and solver.
"""
import math
import time

import numpy as np

from . import glasma as G

HBARC = G.HBARC_GEV_FM
MASSES = (0.0, 1.27, 4.18)
QS_RANGE = (1.0, 3.0)
PT_RANGE = (0.0, 10.0)
JET_PT_MIN = 0.5
TAU_MAX = 1.0
M_IR = 0.2
# Q_s / g^2 mu of the MV Wilson lines (dipole definition D(sqrt(2)/Q_s) =
# exp(-1/2)), measured with gl_calibrate_g2mu at L = 10 fm, 50 sheets,
# m_IR = 0.2 GeV: 0.722 at 512^2, 0.7245 at 256^2
QS_OVER_G2MU = 0.722
# network inputs: Q_s, m, p_T0, tau_form and the square root of the time
# since the particles start, sqrt(tau - tau_start).  The solver starts them at
# the first step at or after tau_form, tau_start = ceil(tau_form / dtau) dtau,
# so curves of different lattice spacings line up at their start; the square
# root spreads the sharp rise right after formation over the input range.
IN_LO = np.array([QS_RANGE[0], 0.0, PT_RANGE[0], 0.0, 0.0], np.float32)
# p_T0 bins of the trust table (per quark mass)
PT_BINS = np.array([0.0, 10.0 / 3.0, 20.0 / 3.0, 10.0], np.float32)
IN_HI = np.array([QS_RANGE[1], MASSES[-1], PT_RANGE[1], 0.2, math.sqrt(TAU_MAX)], np.float32)
# the surrogate reproduces the 512^2, L = 10 fm solver (time step a/8)
REF_N, REF_L_FM = 512, 10.0
REF_DTAU_FM = 0.125 * REF_L_FM / REF_N


def tau_form(m, pt):
    return HBARC / (2.0 * math.sqrt(m * m + pt * pt))


def tau_start(m, pt, dtau_fm=REF_DTAU_FM):
    """First time step at or after the formation time (the solver's rule)."""
    return max(1, math.ceil(tau_form(m, pt) / dtau_fm - 1e-12)) * dtau_fm


def features(qs, m, pt, since_start):
    since_start = np.maximum(np.asarray(since_start, np.float64), 0.0)
    one = np.ones_like(since_start)
    return np.stack([qs * one, m * one, pt * one, tau_form(m, pt) * one, np.sqrt(since_start)],
                    axis=1).astype(np.float32)


def draw_params(n, seed):
    """Q_s ~ U[1, 3] GeV, m ~ U{0, 1.27, 4.18} GeV, p_T0 ~ U[0, 10] GeV (jets U[0.5, 10])."""
    g = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        qs = g.uniform(*QS_RANGE)
        m = float(g.choice(MASSES))
        pt = g.uniform(JET_PT_MIN if m == 0 else PT_RANGE[0], PT_RANGE[1])
        out.append((qs, m, pt))
    return out


def in_domain(qs, m, pt, tau):
    if not (QS_RANGE[0] <= qs <= QS_RANGE[1]):
        return False
    if min(abs(m - mm) for mm in MASSES) > 1e-6:
        return False
    if not (PT_RANGE[0] <= pt <= PT_RANGE[1]) or (m == 0 and pt < JET_PT_MIN):
        return False
    return bool(np.all((np.asarray(tau) >= 0) & (np.asarray(tau) <= TAU_MAX)))


def _curve(ev, jet):
    """(tau_n, total coefficient, transverse broadening at tau_n) of species 0
    of a finished event (the broadening is averaged from the half steps)."""
    br = ev.broadening(0)       # tau_{n+1/2}, <dpx2>, <dpy2>, <dpz2>, n
    if len(br) == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    if jet:
        q = ev.qhat(0)          # tau, qhat_y, qhat_z
        tau, coef = q[:, 0], q[:, 1] + q[:, 2]
        dpt = br[:, 2] + br[:, 3]
    else:
        k = ev.kappa(0)         # tau, tau - tau_form, kappa_T, kappa_L
        tau, coef = k[:, 0], k[:, 2] + k[:, 3]
        dpt = br[:, 1] + br[:, 2]
    prev = np.concatenate([[0.0], dpt[:-1]])
    return tau, coef, 0.5 * (dpt + prev)


def solver_curves(params, N, L_fm, n_particles, seed, precision=32, sheets=50, batch=64,
                  tune_cache=None, uv_cut=0.0):
    """Run the solver for each (Q_s, m, p_T0); returns a list of curves
    (tau, kappa, dpT2) and the GPU wall time spent per curve."""
    import torch
    curves = []
    a_fm = L_fm / N
    steps = int(math.ceil(TAU_MAX / (0.125 * a_fm) - 1e-9)) - 1
    t0 = time.perf_counter()
    for c0 in range(0, len(params), batch):
        chunk = params[c0:c0 + batch]
        evs = []
        for k, (qs, m, pt) in enumerate(chunk):
            ev = G.Event(N, L_fm, 0.125, precision=precision, max_steps=steps,
                         max_particles=n_particles)
            ev.init_glasma(qs / QS_OVER_G2MU, M_IR, sheets, seed + c0 + k, uv_cut)
            ev.add_species(m, pt, G.KIND_JET if m == 0 else G.KIND_HEAVY_QUARK, n_particles,
                           seed + 7919 * (c0 + k) + 1)
            evs.append(ev)
        b = G.Batch(evs)
        b.autotune(tune_cache)
        b.run(steps)
        b.stream.synchronize()
        torch.cuda.synchronize()
        for ev, (qs, m, pt) in zip(evs, chunk):
            curves.append(_curve(ev, m == 0))
        b.close()
        for ev in evs:
            ev.close()
    torch.cuda.synchronize()
    return curves, (time.perf_counter() - t0) / max(len(params), 1)


def rows(params, curves):
    """Network rows of solver curves; each curve is aligned on its own start
    (its first row is the first step after formation)."""
    X, Y = [], []
    for (qs, m, pt), (tau, kap, dpt) in zip(params, curves):
        if len(tau) == 0:
            continue
        X.append(features(qs, m, pt, tau - tau[0]))
        Y.append(np.stack([kap, dpt], axis=1))
    return np.concatenate(X).astype(np.float32), np.concatenate(Y).astype(np.float32)


class Surrogate:
    def __init__(self, seed=1, max_samples=1 << 20):
        self.net = G.MLP(5, 256, 3, 2, max_batch=4096, max_samples=max_samples, seed=seed)
        self.trained = False

    # the Glasma has one physical scale, Q_s: the network models kappa / Q_s^3
    # and <dp_T^2> / Q_s^2 (dimensionless up to the mass and p_T dependence)
    OUT_POWERS = np.array([3.0, 2.0], np.float32)

    def fit(self, X, Y, epochs=40, batch=4096, lr=1e-3, seed=0):
        Ys = Y / X[:, :1] ** self.OUT_POWERS[None, :]
        mu, sd = Ys.mean(0), Ys.std(0)
        sd = np.where(sd > 0, sd, 1.0)
        self.net.set_scaling(IN_LO, IN_HI, mu, sd)
        self.net.set_output_power(0, self.OUT_POWERS)
        losses = self.net.train(X, Y, epochs=epochs, batch=batch, lr=lr, seed=seed)
        self.trained = True
        return losses

    def predict(self, qs, m, pt, tau):
        """kappa and <dp_T^2> at tau as the 512^2 solver gives them (zero
        before its particles start)."""
        tau = np.asarray(tau, np.float64)
        since = tau - tau_start(m, pt)
        Y = self.net.infer(features(qs, m, pt, since)).cpu().numpy()
        live = since >= -1e-9
        return np.where(live, Y[:, 0], 0.0), np.where(live, Y[:, 1], 0.0)

    def set_trust(self, err_table, err_max=0.05):
        """Trust region of the queries: the training box, the three masses
        and three p_T0 bins, with the held-out kappa error of each
        (mass, p_T0 bin) cell; cells above err_max fall back to the solver."""
        lo = IN_LO.copy()
        hi = IN_HI.copy()
        hi[3] = tau_form(0.0, JET_PT_MIN) + 1e-6      # the largest formation time in the domain
        self.net.set_trust(lo, hi, 1, np.array(MASSES, np.float32), 1e-3, 2, PT_BINS, err_table, err_max)
        self.trusted = True

    def query(self, qs, m, pt, tau, N=512, L_fm=10.0, n_particles=100000, seed=12345):
        """kappa(tau), <dp_T^2>(tau) and the verdict of gl_surrogate_query: 0
        when the network answered, else the solver did (1: outside the
        training domain, 2: a cell whose held-out error is above the bound,
        3: no trust table yet)."""
        tau = np.asarray(tau, np.float64)
        verdict = 3
        if self.trained and getattr(self, "trusted", False) and (m > 0 or pt >= JET_PT_MIN):
            since = tau - tau_start(m, pt)
            Y, verdict = self.net.query(features(qs, m, pt, since))
            if Y is not None:
                live = since >= -1e-9
                return np.where(live, Y[:, 0], 0.0), np.where(live, Y[:, 1], 0.0), 0
        elif self.trained and getattr(self, "trusted", False):
            verdict = 1
        (t, k, d), = solver_curves([(qs, m, pt)], N, L_fm, n_particles, seed, batch=1)[0]
        return np.interp(tau, t, k), np.interp(tau, t, d), verdict


def curve_error(pred, ref):
    """max |pred - ref| / max |ref| over the curve."""
    return float(np.abs(pred - ref).max() / max(np.abs(ref).max(), 1e-30))


def cell_of(m, pt):
    """(mass class, p_T0 bin) of a parameter point, as gl_surrogate_query bins it."""
    k = int(np.argmin([abs(m - mm) for mm in MASSES]))
    b = int(np.clip(np.searchsorted(PT_BINS, pt, side="right") - 1, 0, len(PT_BINS) - 2))
    return k, b


def trust_table(params, errors):
    """Largest held-out kappa error per (mass, p_T0 bin) cell; cells without a
    held-out point get infinity (never trusted)."""
    t = np.full((len(MASSES), len(PT_BINS) - 1), np.inf, np.float32)
    for (qs, m, pt), e in zip(params, errors):
        k, b = cell_of(m, pt)
        t[k, b] = e if not np.isfinite(t[k, b]) else max(t[k, b], e)
    return t


def mean_curves(runs):
    """Per point, the mean curve of several solver runs (same time grid)."""
    out = []
    for per_point in zip(*runs):
        tau = per_point[0][0]
        out.append((tau, np.mean([c[1] for c in per_point], axis=0), np.mean([c[2] for c in per_point], axis=0)))
    return out


def protocol(n_train_coarse=2000, n_train_fine=1024, n_heldout=192, n_avg=4, n_part_train=10000,
             n_part_fine=100000, n_part_heldout=100000, epochs=60, fine_epochs=120, err_max=0.05,
             seed=20230718, log=print):
    """The surrogate workload end to end on the GPU.

    1. training data from the solver: n_train_coarse runs at 256^2 and
       n_train_fine runs at 512^2 (L = 10 fm, n_part_train particles each);
    2. held-out points run n_avg times at 512^2 with other seeds: their mean
       is the reference curve (label noise down by sqrt(n_avg)), and one run
       against the mean of the others is the solver's own noise floor;
    3. network A trained on the 256^2 runs only (the specified training set),
       network B the same then fine-tuned on the 512^2 runs;
    4. errors on the held-out curves (max |pred - ref| / max |ref|), and the
       trust region of the queries: the even held-out points calibrate the
       error of each (mass, p_T0 bin) cell (about ten per cell, so that a
       cell's largest error is seen), the odd ones test what the queries
       answer (coverage and error of the network's answers);
    5. the time per kappa(tau) curve of the network and of the solver.
    """
    import torch
    rep = {}
    t = time.perf_counter()
    pc = draw_params(n_train_coarse, seed)
    cc, tpc_c = solver_curves(pc, 256, 10.0, n_part_train, seed + 1)
    Xc, Yc = rows(pc, cc)
    pf = draw_params(n_train_fine, seed + 2)
    cf, tpc_f = solver_curves(pf, 512, 10.0, n_part_fine, seed + 3)
    Xf, Yf = rows(pf, cf)
    rep["data_s"] = time.perf_counter() - t
    rep["train_rows"] = [int(len(Xc)), int(len(Xf))]
    log("surrogate: data %.1f s, rows %s" % (rep["data_s"], rep["train_rows"]))
    hp = draw_params(n_heldout, seed + 4)
    runs = []
    for r in range(n_avg):
        hc_r, tpc_h = solver_curves(hp, 512, 10.0, n_part_heldout, seed + 5 + 7919 * r)
        runs.append(hc_r)
    rep["solver_s_per_curve"] = tpc_h
    ref = mean_curves(runs)
    rest = mean_curves(runs[1:])
    noise = np.array([curve_error(a[1], b[1]) for a, b in zip(runs[0], rest)])
    rep["reference"] = "mean of %d solver runs per held-out point (%d particles each)" % (n_avg, n_part_heldout)
    rep["noise_floor_kappa"] = {"what": "one solver run against the mean of the other %d" % (n_avg - 1),
                                "median": float(np.median(noise)), "p90": float(np.percentile(noise, 90)),
                                "max": float(np.max(noise))}

    def errors(sur, idx):
        ek, ed = [], []
        for i in idx:
            (qs, m, pt), (tau, k, d) = hp[i], ref[i]
            kp, dp = sur.predict(qs, m, pt, tau)
            ek.append(curve_error(kp, k))
            ed.append(curve_error(dp, d))
        return np.array(ek), np.array(ed)

    def evaluate(sur):
        ek, ed = errors(sur, range(n_heldout))
        out = {"kappa_median": float(np.median(ek)), "kappa_p90": float(np.percentile(ek, 90)),
               "kappa_max": float(np.max(ek)), "dpT2_median": float(np.median(ed)),
               "dpT2_max": float(np.max(ed))}
        ms = np.array([m for _, m, _ in hp])
        for mm in MASSES:
            sel = ms == mm
            if sel.any():
                out["kappa_median_m%.2f" % mm] = float(np.median(ek[sel]))
        return out

    t = time.perf_counter()
    A = Surrogate(seed=seed, max_samples=max(len(Xc), len(Xf)) + 1)
    la = A.fit(Xc, Yc, epochs=epochs, lr=1e-3, seed=1)
    B = Surrogate(seed=seed, max_samples=max(len(Xc), len(Xf)) + 1)
    B.fit(Xc, Yc, epochs=epochs, lr=1e-3, seed=1)
    # fine-tune on the 512^2 runs with the coarse runs' output scaling kept
    lb = B.net.train(Xf, Yf, epochs=fine_epochs, batch=4096, lr=3e-4, seed=2)
    torch.cuda.synchronize()
    rep["train_s"] = time.perf_counter() - t
    rep["loss_final"] = [float(la[-1]), float(lb[-1])]
    rep["coarse_only"] = evaluate(A)
    rep["c5_as_specified"] = "coarse_only: trained on the 2000 runs at 256^2 alone"
    rep["fine_tuned"] = evaluate(B)
    ek_all, _ = errors(B, range(n_heldout))
    worst = np.argsort(ek_all)[::-1][:3]
    rep["fine_tuned_worst"] = [{"qs_GeV": round(hp[i][0], 3), "m_GeV": hp[i][1], "pT0_GeV": round(hp[i][2], 3),
                                "kappa_err": round(float(ek_all[i]), 4), "cell": list(cell_of(hp[i][1], hp[i][2])),
                                "noise_of_one_run": round(float(noise[i]), 4)} for i in worst]
    # trust region: calibrate on the even held-out points, test on the odd ones
    cal, test = list(range(0, n_heldout, 2)), list(range(1, n_heldout, 2))
    ek_cal, _ = errors(B, cal)
    table = trust_table([hp[i] for i in cal], ek_cal)
    B.set_trust(table, err_max)
    ek_test, _ = errors(B, test)
    answered = []
    for i in test:
        qs, m, pt = hp[i]
        tau = ref[i][0]
        _, verdict = B.net.query(features(qs, m, pt, tau - tau_start(m, pt)))
        answered.append(verdict == 0)
    answered = np.array(answered)
    rep["trust"] = {"err_max": err_max, "cells_trusted": int(np.sum(table <= err_max)), "cells": int(table.size),
                    "calibration_points": len(cal), "test_points": len(test),
                    "test_coverage": float(answered.mean()),
                    "test_kappa_err_answered": None if not answered.any() else
                    {"median": float(np.median(ek_test[answered])), "p90": float(np.percentile(ek_test[answered], 90)),
                     "max": float(np.max(ek_test[answered]))},
                    "test_kappa_err_all": {"median": float(np.median(ek_test)),
                                           "p90": float(np.percentile(ek_test, 90)), "max": float(np.max(ek_test))},
                    "table": [[None if not np.isfinite(v) else round(float(v), 4) for v in row] for row in table]}
    tau = np.linspace(0.0025, 1.0, 410)
    B.predict(2.0, 4.18, 2.0, tau)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = 50
    for _ in range(reps):
        B.predict(2.0, 4.18, 2.0, tau)
    torch.cuda.synchronize()
    rep["mlp_s_per_curve"] = (time.perf_counter() - t) / reps
    # a batch of curves in one inference call
    Xq = np.tile(features(2.0, 4.18, 2.0, tau - tau_start(4.18, 2.0)), (64, 1))
    Xd = B.net._dev(Xq, 5)
    B.net.infer(Xd)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        B.net.infer(Xd)
    torch.cuda.synchronize()
    rep["mlp_s_per_curve_batched64"] = (time.perf_counter() - t) / reps / 64
    rep["speedup"] = rep["solver_s_per_curve"] / rep["mlp_s_per_curve"]
    rep["speedup_batched"] = rep["solver_s_per_curve"] / rep["mlp_s_per_curve_batched64"]
    # a query outside the training domain goes to the solver
    _, _, verdict = B.query(3.5, 1.27, 2.0, tau[:100], N=64, L_fm=10.0 * 64 / 512, n_particles=1000)
    rep["fallback_outside_domain"] = bool(verdict == 1)
    log("surrogate: %s" % rep)
    return rep
