"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  The product path (``paper_2307_07999_amd``)
never does.  Array layouts are the oracle's own (array-of-structures, see
``glasma_oracle.h``); converting to the HIP library's structure-of-arrays
layout is done by the tests with plain numpy transposes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glasma_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile the oracle with plain g++ (-O2, no fast-math, no OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-o", _LIB_PATH, _SRC])
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_U32 = ctypes.POINTER(ctypes.c_uint32)


def _declare(L):
    c_int, c_double, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    sig = {
        "orc_generator": (None, [c_int, _D]),
        "orc_dsym": (c_double, [c_int, c_int, c_int]),
        "orc_expi": (None, [_D, _D]),
        "orc_expm": (None, [_D, _D]),
        "orc_proj": (None, [_D, _D]),
        "orc_philox": (None, [_U32, _U32, _U32]),
        "orc_u53": (c_double, [ctypes.c_uint32, ctypes.c_uint32]),
        "orc_mv_charges": (None, [c_int, c_double, c_u64, c_int, c_int, _D]),
        "orc_fft": (c_int, [c_int, _D, c_int]),
        "orc_poisson": (c_int, [c_int, c_double, _D, _D]),
        "orc_wilson_line": (c_int, [c_int, c_double, c_double, c_int, c_u64, c_int, _D]),
        "orc_poisson_uv": (c_int, [c_int, c_double, c_double, _D, _D]),
        "orc_wilson_line_uv": (c_int, [c_int, c_double, c_double, c_double, c_int, c_u64, c_int, _D]),
        "orc_init_glasma_uv": (c_int, [c_int, c_double, c_double, c_double, c_int, c_u64, c_double,
                                       _D, _D, _D, _D, _D]),
        "orc_nucleus_links": (None, [c_int, _D, _D]),
        "orc_match_link": (c_int, [_D, _D, _D, c_double, c_int, _D]),
        "orc_pi0": (None, [c_int, _D, _D, _D, _D]),
        "orc_init_glasma": (c_int, [c_int, c_double, c_double, c_int, c_u64, c_double,
                                    _D, _D, _D, _D, _D]),
        "orc_forces": (None, [c_int, c_double, _D, _D, _D, _D]),
        "orc_field_step": (None, [c_int, c_int, c_double, _D, _D, _D, _D, _D]),
        "orc_field_step_sites": (None, [c_int, c_int, c_double, _D, _D, _D, _D, c_int, _I,
                                        _D, _D, _D, _D, _D]),
        "orc_energy": (None, [c_int, c_double, _D, _D, _D, _D, _D]),
        "orc_gauss": (None, [c_int, _D, _D, _D, _D, _D]),
        "orc_particles_init": (None, [c_int, c_u64, c_int, c_int, c_double, c_int, _I, _D,
                                      _D, _D, _D, _D]),
        "orc_particle_step": (None, [c_int, c_int, c_double, _D, _D, _D, c_int, _I, _D, _D,
                                     _D, _D, _D, _I, c_int, _D, _I, _D]),
        "orc_run": (c_int, [c_int, c_double, c_double, c_int, c_u64, c_double, c_int, c_int,
                            _I, _D, _D, _I, _I, _D, _D, _D, _D, _I, _D, _D, _D, _D, _D,
                            _I, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def _u(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(_U32)


# ---- matrices as numpy complex (3,3) <-> 18 doubles ------------------------
def m2d(m):
    return np.ascontiguousarray(np.asarray(m, np.complex128).reshape(-1, 3, 3)).view(
        np.float64).reshape(np.shape(m)[:-2] + (18,))


def d2m(d):
    d = np.ascontiguousarray(d, dtype=np.float64)
    return d.view(np.complex128).reshape(d.shape[:-1] + (3, 3))


def generator(a):
    out = np.zeros(18)
    lib().orc_generator(a, _d(out))
    return d2m(out)


def dsym(a, b, c):
    return lib().orc_dsym(a, b, c)


def expi(x8):
    x8 = np.ascontiguousarray(x8, np.float64)
    out = np.zeros(18)
    lib().orc_expi(_d(x8), _d(out))
    return d2m(out)


def expm(A):
    a = m2d(A).copy()
    out = np.zeros(18)
    lib().orc_expm(_d(a), _d(out))
    return d2m(out)


def proj(M):
    a = m2d(M).copy()
    out = np.zeros(8)
    lib().orc_proj(_d(a), _d(out))
    return out


def philox(key, ctr):
    k = np.ascontiguousarray(key, np.uint32)
    c = np.ascontiguousarray(ctr, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_u(k), _u(c), _u(out))
    return out


def u53(lo, hi):
    return lib().orc_u53(lo, hi)


def mv_charges(N, sigma, seed, nucleus, sheet):
    out = np.zeros((N * N, 8))
    lib().orc_mv_charges(N, sigma, seed, nucleus, sheet, _d(out))
    return out


def fft(x, sign=-1):
    d = np.ascontiguousarray(np.asarray(x, np.complex128)).view(np.float64).copy()
    rc = lib().orc_fft(len(x), _d(d), sign)
    assert rc == 0
    return d.view(np.complex128)


def poisson(N, m2, src):
    src = np.ascontiguousarray(src, np.float64).reshape(N * N)
    out = np.zeros(N * N)
    assert lib().orc_poisson(N, m2, _d(src), _d(out)) == 0
    return out


def wilson_line(N, sigma, m2, n_sheets, seed, nucleus, uv2=0.0):
    V = np.zeros((N * N, 18))
    assert lib().orc_wilson_line_uv(N, sigma, m2, uv2, n_sheets, seed, nucleus, _d(V)) == 0
    return V


def poisson_uv(N, m2, uv2, src):
    src = np.ascontiguousarray(src, np.float64).reshape(N * N)
    out = np.zeros(N * N)
    assert lib().orc_poisson_uv(N, m2, uv2, _d(src), _d(out)) == 0
    return out


def dipole(N, V, rmax):
    """Dipole correlator of a Wilson line, D(r) = (1/3) < Re Tr V(x) V^dag(x+r) >,
    averaged over the sites x and the two lattice directions of the
    separation, for r = 0..rmax (lattice units).  V [N*N][18]."""
    M = d2m(np.asarray(V)).reshape(N, N, 3, 3)          # [y][x]
    Md = np.conj(np.swapaxes(M, -1, -2))
    D = np.zeros(rmax + 1)
    for r in range(rmax + 1):
        sx = np.roll(Md, -r, axis=1)                     # V^dag(x + r e_x)
        sy = np.roll(Md, -r, axis=0)                     # V^dag(x + r e_y)
        tx = np.real(np.einsum("yxij,yxji->yx", M, sx)).mean()
        ty = np.real(np.einsum("yxij,yxji->yx", M, sy)).mean()
        D[r] = (tx + ty) / 6.0
    return D


def nucleus_links(N, V):
    out = np.zeros((2, N * N, 18))
    lib().orc_nucleus_links(N, _d(np.ascontiguousarray(V)), _d(out))
    return out


def match_link(UA, UB, tol=1e-13, max_iter=100):
    ua, ub = m2d(UA).copy(), m2d(UB).copy()
    out = np.zeros(18)
    res = np.zeros(1)
    it = lib().orc_match_link(_d(ua), _d(ub), _d(out), tol, max_iter, _d(res))
    return d2m(out), it, float(res[0])


def pi0(N, U, UA, UB):
    out = np.zeros((N * N, 8))
    lib().orc_pi0(N, _d(np.ascontiguousarray(U)), _d(np.ascontiguousarray(UA)),
                  _d(np.ascontiguousarray(UB)), _d(out))
    return out


class State:
    """Oracle field state in its own layout: U [2,N2,18], E [2,N2,8], phi/pi [N2,8]."""

    def __init__(self, N):
        self.N = N
        n2 = N * N
        self.U = np.zeros((2, n2, 18))
        self.E = np.zeros((2, n2, 8))
        self.phi = np.zeros((n2, 8))
        self.pi = np.zeros((n2, 8))
        self.n = 1

    def copy(self):
        s = State(self.N)
        s.U, s.E, s.phi, s.pi, s.n = (self.U.copy(), self.E.copy(), self.phi.copy(),
                                      self.pi.copy(), self.n)
        return s


def init_glasma(N, sigma, m2, n_sheets, seed, dtau, uv2=0.0):
    s = State(N)
    res = np.zeros(1)
    rc = lib().orc_init_glasma_uv(N, sigma, m2, uv2, n_sheets, seed, dtau, _d(s.U), _d(s.E),
                                  _d(s.phi), _d(s.pi), _d(res))
    return s, rc, float(res[0])


def forces(N, tau, U, phi):
    FE = np.zeros((2, N * N, 8))
    Fpi = np.zeros((N * N, 8))
    lib().orc_forces(N, tau, _d(np.ascontiguousarray(U)), _d(np.ascontiguousarray(phi)),
                     _d(FE), _d(Fpi))
    return FE, Fpi


def field_step(s, dtau, want_F=False):
    """Advance an oracle State by one leapfrog step in place; returns F^n or None."""
    F = np.zeros((s.N * s.N, 6, 8)) if want_F else None
    lib().orc_field_step(s.N, s.n, dtau, _d(s.U), _d(s.E), _d(s.phi), _d(s.pi),
                         _d(F) if want_F else None)
    s.n += 1
    return F


def field_step_sites(s, dtau, sites):
    sites = np.ascontiguousarray(sites, np.int32)
    k = len(sites)
    U_new = np.zeros((k, 2, 18))
    E_new = np.zeros((k, 2, 8))
    phi_new = np.zeros((k, 8))
    pi_new = np.zeros((k, 8))
    F = np.zeros((k, 6, 8))
    lib().orc_field_step_sites(s.N, s.n, dtau, _d(s.U), _d(s.E), _d(s.phi), _d(s.pi), k,
                               _i(sites), _d(U_new), _d(E_new), _d(phi_new), _d(pi_new),
                               _d(F))
    return U_new, E_new, phi_new, pi_new, F


def energy(s, tau):
    out = np.zeros(4)
    lib().orc_energy(s.N, tau, _d(s.U), _d(s.E), _d(s.phi), _d(s.pi), _d(out))
    return out


def gauss(s):
    G = np.zeros((s.N * s.N, 8))
    lib().orc_gauss(s.N, _d(s.U), _d(s.E), _d(s.phi), _d(s.pi), _d(G))
    return G


class Particles:
    """Oracle particle arrays (array-of-structures per quantity)."""

    def __init__(self, n):
        self.cell = np.zeros((n, 2), np.int32)
        self.off = np.zeros((n, 2))
        self.eta = np.zeros(n)
        self.p = np.zeros((n, 3))
        self.Q = np.zeros((n, 8))
        self.p0 = np.zeros((n, 3))
        self.species = np.zeros(n, np.int32)

    @property
    def n(self):
        return len(self.eta)

    def copy(self):
        q = Particles(self.n)
        for k in ("cell", "off", "eta", "p", "Q", "p0", "species"):
            setattr(q, k, getattr(self, k).copy())
        return q

    def subset(self, idx):
        q = Particles(len(idx))
        for k in ("cell", "off", "eta", "p", "Q", "p0", "species"):
            setattr(q, k, np.ascontiguousarray(getattr(self, k)[idx]))
        return q


def particles_init(N, seed, species_id, kind, p0, n):
    P = Particles(n)
    lib().orc_particles_init(N, seed, species_id, kind, p0, n, _i(P.cell), _d(P.off),
                             _d(P.eta), _d(P.p), _d(P.Q), _d(P.p0))
    P.species[:] = species_id
    return P


def particle_step(N, n, dtau, U, phi, F, P, mass, nform):
    mass = np.ascontiguousarray(mass, np.float64)
    nform = np.ascontiguousarray(nform, np.int32)
    ns = len(mass)
    series = np.zeros((ns, 4))
    lib().orc_particle_step(N, n, dtau, _d(np.ascontiguousarray(U)),
                            _d(np.ascontiguousarray(phi)), _d(np.ascontiguousarray(F)),
                            P.n, _i(P.cell), _d(P.off), _d(P.eta), _d(P.p), _d(P.Q),
                            _d(P.p0), _i(P.species), ns, _d(mass), _i(nform), _d(series))
    return series


def static_series(s, dtau, n_steps, n0=1):
    """Static-quark momentum broadening from electric-field correlators
    (Sec. 2, Eq. (4)) on the lattice.  A static quark keeps its colour charge
    and its site, so delta p_i = sum_n dtau Q^a E_i^a(x, tau_n) with the
    local-frame site fields the particles read; with <Q^a Q^b> = delta^ab / 2
    its mean square over the charges is (1/2) sum_a (I_i^a)^2 for
    I_i^a(x) = sum_n dtau E_i^a(x, tau_n).  Accumulates I over the steps
    n >= n0 while advancing the State; row k (step n = s.n + k, time
    tau_{n+1/2}) holds the sums over sites of (1/2) sum_a (I_i^a)^2 for
    i = x, y, z and the number of sites (0 before n0)."""
    n2 = s.N * s.N
    I = np.zeros((n2, 3, 8))
    rows = np.zeros((n_steps, 4))
    for k in range(n_steps):
        n = s.n
        F = field_step(s, dtau, want_F=True)
        if n >= n0:
            I += dtau * F[:, 0:3, :]
            rows[k, :3] = 0.5 * (I ** 2).sum(axis=(0, 2))
            rows[k, 3] = n2
    return rows


def lightlike_series(s, dtau, n_steps, n0=1):
    """Lightlike-jet momentum broadening from parallel-transported field
    correlators (Sec. 2, Eq. (5)) on the lattice.  A jet starting at the
    centre of site x0 at step n0 moves along +x at the speed of light: at step
    n = n0 + k it sits in the cell x0 + floor(k dtau + 1/2) (the NGP rule of
    the particle push), feels F_x = E_x, F_y = E_y - B_z, F_z = E_z + B_y of the
    local-frame site fields there, and its colour frame is carried by W, the
    product of the x links it crossed, each taken at its crossing step (W is
    multiplied by U_x(cell) at the tau_n of a step whose drift ends in the
    next cell).  I_i^a(x0) = sum_n dtau [W F_i W^dag]^a and, with
    <Q^a Q^b> = delta^ab / 2, row k (step n = s.n + k, time tau_{n+1/2}) holds
    the sums over start sites of (1/2) sum_a (I_i^a)^2, i = x, y, z, and the
    number of sites (0 before n0).  Advances the State."""
    N = s.N
    n2 = N * N
    x0 = np.arange(n2) % N
    y0 = np.arange(n2) // N
    T = np.array([generator(a) for a in range(8)])
    W = np.broadcast_to(np.eye(3, dtype=np.complex128), (n2, 3, 3)).copy()
    I = np.zeros((n2, 3, 8))
    rows = np.zeros((n_steps, 4))
    for k in range(n_steps):
        n = s.n
        U1 = d2m(s.U[0]).copy()          # x links at tau_n
        F = field_step(s, dtau, want_F=True)
        if n < n0:
            continue
        j = n - n0
        shift = int(np.floor(j * dtau + 0.5))
        c = (x0 + shift) % N + N * y0
        f = F[c]
        for i, Fi in enumerate((f[:, 0], f[:, 1] - f[:, 5], f[:, 2] + f[:, 4])):
            M = np.einsum("na,aij->nij", Fi, T)
            Mt = W @ M @ np.conj(np.swapaxes(W, 1, 2))
            I[:, i] += dtau * 2.0 * np.real(np.einsum("aij,nji->na", T, Mt))
        rows[k, :3] = 0.5 * (I ** 2).sum(axis=(0, 2))
        rows[k, 3] = n2
        if int(np.floor((j + 1) * dtau + 0.5)) > shift:
            W = W @ U1[c]
    return rows


def run(N, sigma, m2, n_sheets, seed, dtau, n_steps, species):
    """species: list of dicts with kind, mass, p0, nform, n (lattice units)."""
    ns = len(species)
    kind = np.array([s["kind"] for s in species], np.int32)
    mass = np.array([s["mass"] for s in species], np.float64)
    p0 = np.array([s["p0"] for s in species], np.float64)
    nform = np.array([s["nform"] for s in species], np.int32)
    npart = np.array([s["n"] for s in species], np.int32)
    tot = int(npart.sum())
    st = State(N)
    P = Particles(tot)
    series = np.zeros((n_steps, ns, 4))
    rc = lib().orc_run(N, sigma, m2, n_sheets, seed, dtau, n_steps, ns, _i(kind), _d(mass),
                       _d(p0), _i(nform), _i(npart), _d(st.U), _d(st.E), _d(st.phi),
                       _d(st.pi), _i(P.cell), _d(P.off), _d(P.eta), _d(P.p), _d(P.Q),
                       _d(P.p0), _i(P.species), _d(series))
    st.n = 1 + n_steps
    return st, P, series, rc


# ---- observables: the derivative of Eq. (3) on the half-step grid ----------
HBARC_GEV_FM = 0.1973269804


def mean_broadening(series_s):
    """series_s [n_steps, 4] of one species -> <dp_x^2>, <dp_y^2>, <dp_z^2> per row
    (lattice units) and the active mask; rows with no active particle are 0."""
    series_s = np.asarray(series_s, np.float64)
    n = series_s[:, 3]
    mean = np.where(n[:, None] > 0, series_s[:, :3] / np.maximum(n, 1)[:, None], 0.0)
    return mean, n > 0


def coefficients(series_s, dtau):
    """Instantaneous coefficients d<dp_i^2>/dtau at tau_n (lattice units) as the
    central difference of the half-step means; the value before formation is
    zero.  Returns (row index k of tau_n, rates [*, 3])."""
    mean, active = mean_broadening(series_s)
    ks, rates = [], []
    for k in range(len(mean)):
        if not active[k]:
            continue
        prev = mean[k - 1] if (k > 0 and active[k - 1]) else np.zeros(3)
        ks.append(k)
        rates.append((mean[k] - prev) / dtau)
    return np.array(ks, np.int64), np.array(rates).reshape(-1, 3)


def to_physical(a_fm):
    """Factors turning lattice <dp^2> into GeV^2 and lattice rates into GeV^2/fm."""
    a_gev = a_fm / HBARC_GEV_FM
    return 1.0 / a_gev ** 2, 1.0 / (a_gev ** 2 * a_fm)


def scan_statistics(series_events, kind, dtau_fm, a_fm):
    """Event statistics of one species' broadening over several Glasma events
    (Sec. 2: <dp_i^2> averaged over the particle trajectories and over
    events), written out plainly.  series_events [E][rows][4] holds each
    event's raw series (sums of dp_x^2, dp_y^2, dp_z^2 and the count, lattice
    units).  Components: A = dp_x^2 + dp_y^2, B = dp_z^2 for heavy quarks
    (kind 0); A = dp_y^2, B = dp_z^2 for jets along x (kind 1).  For every row
    with active particles: the pooled means <A>, <B> (GeV^2), their ratio, the
    rates of Eq. (3) as central differences on the half-step grid and their
    sum, the total rate (GeV^2/fm), each from all events and from every sample that leaves one
    event out; the error is the delete-one jackknife (Quenouille, Tukey)
    sqrt((E-1)/E sum_i (f_(i) - mean_i f_(i))^2).  Returns rows (tau_{k+3/2},
    tau_{k+1}, <A>, err, <B>, err, <B>/<A>, err, rate A, err, rate B, err,
    total rate, err)."""
    S = np.asarray(series_events, np.float64)
    E, rows = S.shape[0], S.shape[1]
    a_gev = a_fm / HBARC_GEV_FM
    f2 = 1.0 / a_gev ** 2
    fk = f2 / a_fm
    dtau_lat = dtau_fm / a_fm

    def components(e, k):
        if kind == 0:
            return S[e, k, 0] + S[e, k, 1], S[e, k, 2]
        return S[e, k, 1], S[e, k, 2]

    def pooled(k, skip):
        sa = sb = n = 0.0
        for e in range(E):
            if e == skip:
                continue
            a, b = components(e, k)
            sa += a
            sb += b
            n += S[e, k, 3]
        if n > 0:
            return sa / n, sb / n, True
        return 0.0, 0.0, False

    def observables(k, skip):
        A, B, _ = pooled(k, skip)
        Ap, Bp, prev = pooled(k - 1, skip) if k > 0 else (0.0, 0.0, False)
        if not prev:
            Ap = Bp = 0.0
        ratio = B / A if A != 0 else 0.0
        ra, rb = (A - Ap) / dtau_lat * fk, (B - Bp) / dtau_lat * fk
        return [A * f2, B * f2, ratio, ra, rb, ra + rb]

    out = []
    for k in range(rows):
        if not any(S[e, k, 3] > 0 for e in range(E)):
            continue
        full = observables(k, None)
        loo = [observables(k, i) for i in range(E)]
        row = [(k + 1.5) * dtau_fm, (k + 1) * dtau_fm]
        for j in range(6):
            mean = sum(f[j] for f in loo) / E
            var = sum((f[j] - mean) ** 2 for f in loo) * (E - 1) / E
            row += [full[j], var ** 0.5]
        out.append(row)
    return np.array(out).reshape(-1, 14)
