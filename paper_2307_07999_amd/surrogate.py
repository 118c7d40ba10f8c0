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
QS_OVER_G2MU = 0.6          # reading of "Q_s = 2 GeV": g^2 mu = Q_s / 0.6
IN_LO = np.array([QS_RANGE[0], 0.0, PT_RANGE[0], 0.0, 0.0], np.float32)
IN_HI = np.array([QS_RANGE[1], MASSES[-1], PT_RANGE[1], 0.2, TAU_MAX], np.float32)


def tau_form(m, pt):
    return HBARC / (2.0 * math.sqrt(m * m + pt * pt))


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
    X, Y = [], []
    for (qs, m, pt), (tau, kap, dpt) in zip(params, curves):
        tf = tau_form(m, pt)
        for t, k, d in zip(tau, kap, dpt):
            X.append((qs, m, pt, tf, t))
            Y.append((k, d))
    return np.asarray(X, np.float32), np.asarray(Y, np.float32)


class Surrogate:
    def __init__(self, seed=1, max_samples=1 << 20):
        self.net = G.MLP(5, 256, 3, 2, max_batch=4096, max_samples=max_samples, seed=seed)
        self.trained = False

    def fit(self, X, Y, epochs=40, batch=4096, lr=1e-3, seed=0):
        mu, sd = Y.mean(0), Y.std(0)
        sd = np.where(sd > 0, sd, 1.0)
        self.net.set_scaling(IN_LO, IN_HI, mu, sd)
        losses = self.net.train(X, Y, epochs=epochs, batch=batch, lr=lr, seed=seed)
        self.trained = True
        return losses

    def predict(self, qs, m, pt, tau):
        tau = np.asarray(tau, np.float64)
        X = np.stack([np.full_like(tau, qs), np.full_like(tau, m), np.full_like(tau, pt),
                      np.full_like(tau, tau_form(m, pt)), tau], axis=1).astype(np.float32)
        Y = self.net.infer(X).cpu().numpy()
        return Y[:, 0], Y[:, 1]

    def query(self, qs, m, pt, tau, N=512, L_fm=10.0, n_particles=100000, seed=12345):
        """kappa(tau), <dp_T^2>(tau) and whether the solver was used instead
        of the network (outside the training domain, or before training)."""
        if self.trained and in_domain(qs, m, pt, tau):
            k, d = self.predict(qs, m, pt, tau)
            return k, d, False
        (t, k, d), = solver_curves([(qs, m, pt)], N, L_fm, n_particles, seed, batch=1)[0]
        return np.interp(tau, t, k), np.interp(tau, t, d), True


def curve_error(pred, ref):
    """max |pred - ref| / max |ref| over the curve."""
    return float(np.abs(pred - ref).max() / max(np.abs(ref).max(), 1e-30))
