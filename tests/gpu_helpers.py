"""Shared set-up for the GPU parity tests: configurations of the paper's
workloads and conversion between the oracle's array-of-structures layout and
the library's structure-of-arrays layout (transposes only)."""
import math

import numpy as np

HBARC = 0.1973269804

# 32^2 parity configuration: L = 4 fm, g^2 mu = 1 GeV, m = 0.2 GeV, 1 sheet,
# dtau = a/8 to tau = 1 fm, 1000 charm quarks (m = 1.27 GeV, p_T0 = 0)
C1 = dict(N=32, L=4.0, g2mu=1.0, m_ir=0.2, sheets=1, dtau=0.125, tau_max=1.0, seed=2307079991)


def lattice(cfg):
    a_fm = cfg["L"] / cfg["N"]
    a_gev = a_fm / HBARC
    sigma = cfg["g2mu"] * a_gev / math.sqrt(cfg["sheets"])
    m2 = (cfg["m_ir"] * a_gev) ** 2
    return a_fm, a_gev, sigma, m2


def n_steps(cfg):
    """coupled steps after the initial half step so that tau reaches tau_max"""
    a_fm = cfg["L"] / cfg["N"]
    return int(math.ceil(cfg["tau_max"] / (cfg["dtau"] * a_fm) - 1e-9)) - 1


def state_oracle_to_soa(s):
    U = np.ascontiguousarray(np.transpose(s.U, (0, 2, 1)))
    E = np.ascontiguousarray(np.transpose(s.E, (0, 2, 1)))
    return U, E, np.ascontiguousarray(s.phi.T), np.ascontiguousarray(s.pi.T)


def state_soa_to_oracle(orc, U, E, phi, pi, N, n):
    s = orc.State(N)
    s.U = np.ascontiguousarray(np.transpose(U, (0, 2, 1)))
    s.E = np.ascontiguousarray(np.transpose(E, (0, 2, 1)))
    s.phi = np.ascontiguousarray(phi.T)
    s.pi = np.ascontiguousarray(pi.T)
    s.n = n
    return s


def particles_gpu_to_oracle(orc, d):
    P = orc.Particles(len(d["species"]))
    P.cell = np.ascontiguousarray(d["cell"].T)
    P.off = np.ascontiguousarray(d["off"].T)
    P.eta = np.ascontiguousarray(d["eta"])
    P.p = np.ascontiguousarray(d["p"].T)
    P.Q = np.ascontiguousarray(d["Q"].T)
    P.p0 = np.ascontiguousarray(d["p0"].T)
    P.species = np.ascontiguousarray(d["species"])
    return P


def particles_oracle_to_gpu(P):
    return dict(cell=np.ascontiguousarray(P.cell.T), off=np.ascontiguousarray(P.off.T),
                eta=P.eta.copy(), p=np.ascontiguousarray(P.p.T), Q=np.ascontiguousarray(P.Q.T),
                p0=np.ascontiguousarray(P.p0.T), species=P.species.copy())


def rel_err(got, want):
    scale = np.abs(want).max()
    return np.abs(got - want).max() / (scale if scale > 0 else 1.0)
