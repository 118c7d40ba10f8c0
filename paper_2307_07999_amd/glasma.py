"""Thin Python binding of the C-ABI in include/glasma.h.

Argument marshalling only: every step of the method runs in the HIP kernels
of libglasma.so.  PyTorch provides the device workspace and the stream.  The
library must be built (``python paper_2307_07999_amd/build.py``); loading
fails loudly otherwise.
"""
import ctypes
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglasma.so")
HBARC_GEV_FM = 0.1973269804

GL_OK, GL_EINVAL, GL_ESTATE, GL_ENOTCONV, GL_ENUMERIC, GL_EDEVICE, GL_ENOMEM = 0, -1, -2, -3, -4, -5, -6
GL_MAX_SPECIES = 16
KIND_HEAVY_QUARK, KIND_JET = 0, 1


class GlasmaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("glasma status %d: %s" % (status, msg))
        self.status = status


class LatticeDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("L_fm", ctypes.c_double), ("dtau_over_a", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reunit_every", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("max_particles", ctypes.c_int64),
                ("static_correlator", ctypes.c_int32), ("lightlike_correlator", ctypes.c_int32)]


class MVDesc(ctypes.Structure):
    _fields_ = [("g2mu_GeV", ctypes.c_double), ("m_ir_GeV", ctypes.c_double),
                ("n_sheets", ctypes.c_int32), ("uv_cut_GeV", ctypes.c_double)]


class SpeciesDesc(ctypes.Structure):
    _fields_ = [("mass_GeV", ctypes.c_double), ("p0_GeV", ctypes.c_double), ("kind", ctypes.c_int32),
                ("tau_form_fm", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("gauss_max", ctypes.c_double), ("gauss_rel", ctypes.c_double),
                ("unitarity_max", ctypes.c_double), ("energy", ctypes.c_double * 4),
                ("casimir2_dev", ctypes.c_double), ("casimir3_dev", ctypes.c_double),
                ("nonfinite", ctypes.c_int32)]


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_VP = ctypes.c_void_p

_SIGS = {
    "gl_required_bytes": [ctypes.POINTER(LatticeDesc), ctypes.POINTER(ctypes.c_size_t)],
    "gl_event_create": [ctypes.POINTER(LatticeDesc), _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)],
    "gl_init_glasma": [_VP, ctypes.POINTER(MVDesc), ctypes.c_uint64],
    "gl_init_glasma_from_charges": [_VP, _VP, ctypes.c_int32, ctypes.c_double],
    "gl_add_species": [_VP, ctypes.POINTER(SpeciesDesc), ctypes.c_int64, ctypes.c_uint64, _I32],
    "gl_evolve_fields": [_VP, ctypes.c_int32],
    "gl_push_particles": [_VP],
    "gl_run": [_VP, ctypes.c_int32],
    "gl_broadening": [_VP, ctypes.c_int32, _D, ctypes.c_int32, _I32],
    "gl_kappa": [_VP, ctypes.c_int32, _D, ctypes.c_int32, _I32],
    "gl_qhat": [_VP, ctypes.c_int32, _D, ctypes.c_int32, _I32],
    "gl_series": [_VP, _D, ctypes.c_int32, _I32],
    "gl_static_start": [_VP, ctypes.c_double],
    "gl_dipole": [_VP, ctypes.c_int32, ctypes.c_int32, _D],
    "gl_saturation_scale": [_VP, _D],
    "gl_calibrate_g2mu": [_VP, _VP, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, _D, _D],
    "gl_static_broadening": [_VP, _D, ctypes.c_int32, _I32],
    "gl_lightlike_start": [_VP, ctypes.c_double],
    "gl_lightlike_broadening": [_VP, _D, ctypes.c_int32, _I32],
    "gl_rates_from_series": [_D, ctypes.c_int32, ctypes.c_double, _D],
    "gl_diagnostics": [_VP, ctypes.POINTER(Diag)],
    "gl_set_state": [_VP, _D, _D, _D, _D, ctypes.c_int64],
    "gl_get_state": [_VP, _D, _D, _D, _D, _I64],
    "gl_get_site_fields": [_VP, _D],
    "gl_set_particles": [_VP, ctypes.c_int32, ctypes.POINTER(SpeciesDesc), ctypes.c_int64, _I32, _D, _D,
                         _D, _D, _D, _I32],
    "gl_get_particles": [_VP, ctypes.c_int64, _I64, _I32, _D, _D, _D, _D, _D, _I32],
    "gl_species_info": [_VP, ctypes.c_int32, _I32, _D],
    "gl_get_wilson_line": [_VP, ctypes.c_int32, _D],
    "gl_draw_charges": [_VP, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _D],
    "gl_event_info": [_VP, _D, _D, _I64],
    "gl_sync": [_VP],
    "gl_profile_enable": [_VP, ctypes.c_int32],
    "gl_profile_read": [_VP, _D, _I64],
    "gl_set_sort_period": [_VP, ctypes.c_int32],
    "gl_batch_required_bytes": [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "gl_batch_create": [ctypes.POINTER(_VP), ctypes.c_int32, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)],
    "gl_batch_autotune": [_VP, ctypes.c_char_p],
    "gl_batch_config": [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "gl_batch_info": [_VP, _I32, _I32, _I32, _I32, _I32],
    "gl_batch_run": [_VP, ctypes.c_int32],
    "gl_batch_status": [_VP, _I32],
    "gl_max_particles": [ctypes.c_int32, _I64],
    "gl_scan_statistics": [_D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                           _D, ctypes.c_int32, _I32],
    "gl_set_check_period": [_VP, ctypes.c_int32],
    "gl_set_graph_steps": [_VP, ctypes.c_int32],
    "gl_graph_stats": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "gl_set_match_params": [_VP, ctypes.c_int32, ctypes.c_double],
    "gl_checkpoint": [_VP, ctypes.c_char_p],
    "gl_restore": [_VP, ctypes.c_char_p],
}

_lib = None


def lib():
    """Load libglasma.so (never a fallback: raise if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libglasma.so is not built; run `python paper_2307_07999_amd/build.py` "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.gl_event_destroy.argtypes = [_VP]
        L.gl_event_destroy.restype = None
        L.gl_batch_destroy.argtypes = [_VP]
        L.gl_batch_destroy.restype = None
        L.gl_status_string.argtypes = [ctypes.c_int32]
        L.gl_status_string.restype = ctypes.c_char_p
        L.gl_last_error.argtypes = []
        L.gl_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != GL_OK:
        raise GlasmaError(status, lib().gl_last_error().decode())
    return status


def _need(ok, what):
    # argument checks that stay on under python -O: the C side trusts these sizes
    if not ok:
        raise ValueError(what)


def _d(a):
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous float64 array")
    return a.ctypes.data_as(_D)


def _i(a):
    if a.dtype != np.int32 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous int32 array")
    return a.ctypes.data_as(_I32)


def _keep_until_done(torch, ws, stream, device):
    """A workspace allocated on the current stream but used on another one
    is not handed out again before that stream's work queued at its release
    has finished."""
    if stream.cuda_stream != torch.cuda.current_stream(device).cuda_stream:
        ws.record_stream(stream)


def lattice_spacing(N, L_fm):
    a_fm = L_fm / N
    return a_fm, a_fm / HBARC_GEV_FM


def required_bytes(N, L_fm, dtau_over_a=0.125, precision=64, reunit_every=16, max_steps=512,
                   max_particles=0):
    d = LatticeDesc(N, L_fm, dtau_over_a, precision, reunit_every, max_steps, max_particles)
    out = ctypes.c_size_t(0)
    check(lib().gl_required_bytes(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def max_particles(precision=64):
    """Largest particle capacity an event of this precision accepts."""
    out = ctypes.c_int64(0)
    check(lib().gl_max_particles(precision, ctypes.byref(out)))
    return out.value


def stream_probe(kind, variant, blocks, src_ptr, dst_ptr, nbytes, dst_bytes, reps, stream_handle):
    """Mean milliseconds per launch of the library's streaming kernel
    (gl_stream_probe: kind 0 copy, 1 read, 2 write) over device buffers."""
    L = lib()
    if not getattr(L, "_stream_declared", False):
        L.gl_stream_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, _VP, ctypes.c_size_t,
                                      ctypes.c_size_t, ctypes.c_int32, _VP, _D]
        L.gl_stream_probe.restype = ctypes.c_int32
        L.gl_stream_last_error.argtypes = []
        L.gl_stream_last_error.restype = ctypes.c_char_p
        L._stream_declared = True
    ms = ctypes.c_double(0)
    st = L.gl_stream_probe(kind, variant, blocks, _VP(src_ptr), _VP(dst_ptr), nbytes, dst_bytes, reps,
                           _VP(stream_handle), ctypes.byref(ms))
    if st != GL_OK:
        raise GlasmaError(st, L.gl_stream_last_error().decode())
    return ms.value


def scan_statistics(series, kind, dtau_fm, a_fm):
    """Event statistics of one species' series from several events (see
    gl_scan_statistics): series [n_events, rows, 4] -> rows of (tau_half,
    tau, <A>, err, <B>, err, <B>/<A>, err, rate A, err, rate B, err, total
    rate, err)."""
    s = np.ascontiguousarray(series, np.float64)
    _need(s.ndim == 3 and s.shape[2] == 4, "series must be [n_events, rows, 4]")
    n = ctypes.c_int32(0)
    check(lib().gl_scan_statistics(_d(s), s.shape[0], s.shape[1], kind, dtau_fm, a_fm, None, 0, ctypes.byref(n)))
    out = np.zeros((max(n.value, 1), 14))
    check(lib().gl_scan_statistics(_d(s), s.shape[0], s.shape[1], kind, dtau_fm, a_fm, _d(out), n.value,
                                   ctypes.byref(n)))
    return out[:n.value]


def rates_from_series(series_s, dtau):
    s = np.ascontiguousarray(series_s, np.float64)
    rates = np.zeros((s.shape[0], 3))
    check(lib().gl_rates_from_series(_d(s), s.shape[0], dtau, _d(rates)))
    return rates


class Event:
    """One Glasma event with its particles, on a torch-allocated workspace."""

    def __init__(self, N, L_fm, dtau_over_a=0.125, precision=64, reunit_every=16, max_steps=512,
                 max_particles=0, device="cuda", stream=None, static_correlator=False,
                 lightlike_correlator=False):
        import torch
        self.torch = torch
        self.N, self.L_fm, self.precision = N, L_fm, precision
        self.desc = LatticeDesc(N, L_fm, dtau_over_a, precision, reunit_every, max_steps, max_particles,
                                1 if static_correlator else 0, 1 if lightlike_correlator else 0)
        nbytes = ctypes.c_size_t(0)
        check(lib().gl_required_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.nbytes = nbytes.value
        self.device = torch.device(device)
        self._ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _keep_until_done(torch, self._ws, self.stream, self.device)
        h = _VP()
        check(lib().gl_event_create(ctypes.byref(self.desc), _VP(self._ws_ptr), self.nbytes,
                                    _VP(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n2 = N * N
        self.a_fm, self.a_gev = lattice_spacing(N, L_fm)
        self.dtau = dtau_over_a
        self.species = []

    def close(self):
        held = getattr(self, "_held_by", None)
        if held is not None and held() is not None and getattr(held(), "_h", None):
            raise GlasmaError(GL_ESTATE, "the event is held by a batch: close the batch first")
        if getattr(self, "_h", None):
            lib().gl_event_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- initial conditions ------------------------------------------------
    def init_glasma(self, g2mu_GeV, m_ir_GeV, n_sheets, seed, uv_cut_GeV=0.0):
        mv = MVDesc(g2mu_GeV, m_ir_GeV, n_sheets, uv_cut_GeV)
        return check(lib().gl_init_glasma(self._h, ctypes.byref(mv), seed))

    def init_glasma_from_charges(self, rho, m_ir_GeV):
        """rho: contiguous torch float64 device tensor [2, n_sheets, 8, N*N] or
        [2, n_sheets, 8, N, N] (lattice units); the library reads all of it."""
        if rho.dtype != self.torch.float64 or not rho.is_contiguous() or rho.device.type != "cuda":
            raise ValueError("rho must be a contiguous float64 tensor on the GPU")
        N = self.N
        shape = tuple(rho.shape)
        if not (len(shape) in (4, 5) and shape[0] == 2 and shape[1] >= 1 and shape[2] == 8 and
                shape[3:] in ((N * N,), (N, N))):
            raise ValueError("rho must have shape (2, n_sheets, 8, %d) or (2, n_sheets, 8, %d, %d), got %s"
                             % (N * N, N, N, shape))
        return check(lib().gl_init_glasma_from_charges(self._h, _VP(rho.data_ptr()), shape[1], m_ir_GeV))

    def add_species(self, mass_GeV, p0_GeV, kind, n, seed, tau_form_fm=-1.0):
        sp = SpeciesDesc(mass_GeV, p0_GeV, kind, tau_form_fm)
        sid = ctypes.c_int32(-1)
        check(lib().gl_add_species(self._h, ctypes.byref(sp), n, seed, ctypes.byref(sid)))
        self.species.append(dict(mass_GeV=mass_GeV, p0_GeV=p0_GeV, kind=kind, n=n,
                                 tau_form_fm=tau_form_fm))
        return sid.value

    # ---- evolution -----------------------------------------------------------
    def evolve_fields(self, n_steps):
        return check(lib().gl_evolve_fields(self._h, n_steps))

    def push_particles(self):
        return check(lib().gl_push_particles(self._h))

    def run(self, n_steps):
        return check(lib().gl_run(self._h, n_steps))

    def sync(self):
        return check(lib().gl_sync(self._h))

    # ---- observables ---------------------------------------------------------
    def _rows(self, fn, species, width):
        n = ctypes.c_int32(0)
        check(fn(self._h, species, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), width))
        check(fn(self._h, species, _d(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def broadening(self, species):
        return self._rows(lib().gl_broadening, species, 5)

    def dipole(self, nucleus, rmax):
        """D(r), r = 0..rmax, of the stored Wilson line of one nucleus."""
        D = np.zeros(rmax + 1)
        check(lib().gl_dipole(self._h, nucleus, rmax, _d(D)))
        return D

    def saturation_scale(self):
        """Q_s [GeV] of the stored Wilson lines, D(sqrt(2)/Q_s) = exp(-1/2)."""
        q = ctypes.c_double(0)
        check(lib().gl_saturation_scale(self._h, ctypes.byref(q)))
        return q.value

    def calibrate_g2mu(self, qs_GeV, m_ir_GeV, n_sheets, seed, n_seeds=2, g2mu_start=0.0, uv_cut_GeV=0.0):
        """g^2 mu [GeV] whose MV Wilson lines have Q_s = qs_GeV; returns (g2mu, Q_s reached)."""
        mv = MVDesc(g2mu_start, m_ir_GeV, n_sheets, uv_cut_GeV)
        g, q = ctypes.c_double(0), ctypes.c_double(0)
        check(lib().gl_calibrate_g2mu(self._h, ctypes.byref(mv), qs_GeV, seed, n_seeds, ctypes.byref(g),
                                      ctypes.byref(q)))
        return g.value, q.value

    def static_start(self, tau_start_fm=0.0):
        """Start the static-quark correlator of Eq. (4) at tau_start_fm."""
        return check(lib().gl_static_start(self._h, tau_start_fm))

    def _corr_rows(self, fn):
        n = ctypes.c_int32(0)
        check(fn(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), 5))
        check(fn(self._h, _d(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def static_broadening(self):
        """Rows (tau_{n+1/2} [fm], <dp_x^2>, <dp_y^2>, <dp_z^2> [GeV^2], sites)."""
        return self._corr_rows(lib().gl_static_broadening)

    def lightlike_start(self, tau_start_fm=0.0):
        """Start the lightlike-jet correlator of Eq. (5) at tau_start_fm."""
        return check(lib().gl_lightlike_start(self._h, tau_start_fm))

    def lightlike_broadening(self):
        """Rows (tau_{n+1/2} [fm], <dp_x^2>, <dp_y^2>, <dp_z^2> [GeV^2], sites)."""
        return self._corr_rows(lib().gl_lightlike_broadening)

    def kappa(self, species):
        return self._rows(lib().gl_kappa, species, 4)

    def qhat(self, species):
        return self._rows(lib().gl_qhat, species, 3)

    def series(self):
        n = ctypes.c_int32(0)
        check(lib().gl_series(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), GL_MAX_SPECIES, 4))
        check(lib().gl_series(self._h, _d(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def diagnostics(self):
        d = Diag()
        st = lib().gl_diagnostics(self._h, ctypes.byref(d))
        if st not in (GL_OK, GL_ENUMERIC):
            check(st)
        return dict(gauss_max=d.gauss_max, gauss_rel=d.gauss_rel, unitarity_max=d.unitarity_max,
                    energy=list(d.energy), casimir2_dev=d.casimir2_dev, casimir3_dev=d.casimir3_dev,
                    nonfinite=d.nonfinite, status=st)

    def set_check_period(self, every):
        """Finite-value checks inside run() every `every` steps (0: off)."""
        return check(lib().gl_set_check_period(self._h, every))

    def set_graph_steps(self, steps):
        """run() replays whole blocks of `steps` steps from a captured HIP
        graph (0: direct launches); needs a non-null stream."""
        return check(lib().gl_set_graph_steps(self._h, steps))

    def graph_stats(self):
        """(graphs launched, graphs instantiated) by run() so far."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        check(lib().gl_graph_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_match_params(self, max_iter, tol):
        return check(lib().gl_set_match_params(self._h, max_iter, tol))

    def checkpoint(self, path):
        return check(lib().gl_checkpoint(self._h, os.fsencode(path)))

    def restore(self, path):
        return check(lib().gl_restore(self._h, os.fsencode(path)))

    # ---- host transfers (tests, checkpoints) ---------------------------------
    def set_state(self, U, E, phi, pi, n):
        arrs = [np.ascontiguousarray(a, np.float64) for a in (U, E, phi, pi)]
        _need(arrs[0].size == 36 * self.n2 and arrs[1].size == 16 * self.n2 and arrs[2].size == 8 * self.n2
              and arrs[3].size == 8 * self.n2, "U, E, phi, pi must hold 36, 16, 8 and 8 values per site")
        return check(lib().gl_set_state(self._h, *[_d(a) for a in arrs], n))

    def get_state(self):
        U = np.zeros((2, 18, self.n2))
        E = np.zeros((2, 8, self.n2))
        phi = np.zeros((8, self.n2))
        pi = np.zeros((8, self.n2))
        n = ctypes.c_int64(0)
        check(lib().gl_get_state(self._h, _d(U), _d(E), _d(phi), _d(pi), ctypes.byref(n)))
        return U, E, phi, pi, n.value

    def site_fields(self):
        F = np.zeros((6, 8, self.n2))
        check(lib().gl_get_site_fields(self._h, _d(F)))
        return F

    def set_particles(self, species_descs, cell, off, eta, p, Q, p0, species):
        n = len(species)
        sp = (SpeciesDesc * len(species_descs))(*[SpeciesDesc(*d) for d in species_descs])
        arr = lambda a, t: np.ascontiguousarray(a, t)
        check(lib().gl_set_particles(self._h, len(species_descs), sp, n, _i(arr(cell, np.int32)),
                                     _d(arr(off, np.float64)), _d(arr(eta, np.float64)),
                                     _d(arr(p, np.float64)), _d(arr(Q, np.float64)),
                                     _d(arr(p0, np.float64)), _i(arr(species, np.int32))))

    def get_particles(self):
        n = ctypes.c_int64(0)
        check(lib().gl_get_particles(self._h, 0, ctypes.byref(n), None, None, None, None, None, None,
                                     None))
        k = n.value
        out = dict(cell=np.zeros((2, k), np.int32), off=np.zeros((2, k)), eta=np.zeros(k),
                   p=np.zeros((3, k)), Q=np.zeros((8, k)), p0=np.zeros((3, k)),
                   species=np.zeros(k, np.int32))
        if k:
            check(lib().gl_get_particles(self._h, k, ctypes.byref(n), _i(out["cell"]), _d(out["off"]),
                                         _d(out["eta"]), _d(out["p"]), _d(out["Q"]), _d(out["p0"]),
                                         _i(out["species"])))
        return out

    def species_info(self, s):
        nf = ctypes.c_int32(0)
        m = ctypes.c_double(0)
        check(lib().gl_species_info(self._h, s, ctypes.byref(nf), ctypes.byref(m)))
        return nf.value, m.value

    def wilson_line(self, nucleus):
        V = np.zeros((18, self.n2))
        check(lib().gl_get_wilson_line(self._h, nucleus, _d(V)))
        return V

    def draw_charges(self, seed, nucleus, sheet, sigma):
        rho = np.zeros((8, self.n2))
        check(lib().gl_draw_charges(self._h, seed, nucleus, sheet, sigma, _d(rho)))
        return rho

    def set_sort_period(self, every):
        return check(lib().gl_set_sort_period(self._h, every))

    def profile(self, on=True, period=1):
        """Time every period-th launch of each hot-path kernel class (off: on=False)."""
        return check(lib().gl_profile_enable(self._h, period if on else 0))

    def profile_read(self):
        """(ms[5], launches[5]) of the timed launches per kernel class: field step
        (with the site fields), correlators, push, series reduction (one launch per
        up to 16 pushes), push that also applies a sort (once per sort period)."""
        ms = np.zeros(5)
        cnt = np.zeros(5, np.int64)
        check(lib().gl_profile_read(self._h, _d(ms), cnt.ctypes.data_as(_I64)))
        return ms, cnt

    def info(self):
        a = ctypes.c_double(0)
        dt = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        check(lib().gl_event_info(self._h, ctypes.byref(a), ctypes.byref(dt), ctypes.byref(n)))
        return a.value, dt.value, n.value


class Batch:
    """Events stepped in lock-step by the flattened multi-event kernels, with
    the step loop replayed from a captured hipGraph."""

    def __init__(self, events, stream=None):
        import torch
        self.events = list(events)
        arr = (_VP * len(self.events))(*[e._h for e in self.events])
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        check(lib().gl_batch_required_bytes(arr, len(self.events), ctypes.byref(nbytes)))
        dev = self.events[0].device
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        # a stream of its own (default priority): the legacy default stream
        # cannot be captured into a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        _keep_until_done(torch, self._ws, self.stream, dev)
        h = _VP()
        check(lib().gl_batch_create(arr, len(self.events), _VP(ptr), nbytes.value,
                                    _VP(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        for e in self.events:
            e._held_by = weakref.ref(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_batch_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, cache_json=None):
        return check(lib().gl_batch_autotune(self._h, cache_json.encode() if cache_json else None))

    def config(self, shape=0, grid_mult=4, sort_every=16, graph_steps=32):
        return check(lib().gl_batch_config(self._h, shape, grid_mult, sort_every, graph_steps))

    def info(self):
        v = [ctypes.c_int32(0) for _ in range(5)]
        check(lib().gl_batch_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(shape=v[0].value, tile=(v[1].value, v[2].value), grid_mult=v[3].value,
                    graph_steps=v[4].value)

    def run(self, n_steps):
        return check(lib().gl_batch_run(self._h, n_steps))

    def status(self):
        """Per event, the first step at which it failed (masked), or -1."""
        out = np.zeros(len(self.events), np.int32)
        check(lib().gl_batch_status(self._h, _i(out)))
        return out


class MLPDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


def _mlp_check(status):
    if status != GL_OK:
        raise GlasmaError(status, lib().gl_mlp_last_error().decode())
    return status


def _mlp_declare(L):
    _F = ctypes.POINTER(ctypes.c_float)
    sig = {
        "gl_mlp_required_bytes": [ctypes.POINTER(MLPDesc), ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
        "gl_mlp_create": [ctypes.POINTER(MLPDesc), ctypes.c_int64, _VP, ctypes.c_size_t, _VP, ctypes.c_uint64,
                          ctypes.POINTER(_VP)],
        "gl_mlp_set_scaling": [_VP, _F, _F, _F, _F],
        "gl_mlp_set_output_power": [_VP, ctypes.c_int32, _F],
        "gl_mlp_train": [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                         ctypes.c_uint64, _F],
        "gl_mlp_infer": [_VP, _VP, _VP, ctypes.c_int64],
        "gl_mlp_infer_noalloc": [_VP, _VP, _VP, ctypes.c_int64],
        "gl_mlp_set_trust": [_VP, _F, _F, ctypes.c_int32, ctypes.c_int32, _F, ctypes.c_float, ctypes.c_int32,
                             ctypes.c_int32, _F, _F, ctypes.c_float],
        "gl_surrogate_query": [_VP, _F, ctypes.c_int64, _F, _I32],
        "gl_mlp_grads": [_VP, _VP, _VP, ctypes.c_int32, _F, _F],
        "gl_mlp_params": [_VP, _F, _F, _I64],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    L.gl_mlp_destroy.argtypes = [_VP]
    L.gl_mlp_destroy.restype = None
    L.gl_mlp_last_error.argtypes = []
    L.gl_mlp_last_error.restype = ctypes.c_char_p


def _f(a):
    if a.dtype != np.float32 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous float32 array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """The surrogate network on a torch-allocated workspace (see gl_mlp_* in glasma.h)."""

    def __init__(self, n_in=5, width=256, depth=3, n_out=2, max_batch=4096, max_samples=1 << 20,
                 seed=1, device="cuda", stream=None):
        import torch
        self.torch = torch
        L = lib()
        if not getattr(L, "_mlp_declared", False):
            _mlp_declare(L)
            L._mlp_declared = True
        self.desc = MLPDesc(n_in, width, depth, n_out, max_batch)
        nbytes = ctypes.c_size_t(0)
        _mlp_check(L.gl_mlp_required_bytes(ctypes.byref(self.desc), max_samples, ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _keep_until_done(torch, self._ws, self.stream, self.device)
        h = _VP()
        _mlp_check(L.gl_mlp_create(ctypes.byref(self.desc), max_samples, _VP(ptr), nbytes.value,
                                   _VP(self.stream.cuda_stream), seed, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64(0)
        _mlp_check(L.gl_mlp_params(h, None, None, ctypes.byref(n)))
        self.n_params = n.value
        self.n_in, self.n_out = n_in, n_out

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_mlp_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scaling(self, in_lo, in_hi, out_mean, out_std):
        a = [np.ascontiguousarray(v, np.float32) for v in (in_lo, in_hi, out_mean, out_std)]
        _mlp_check(lib().gl_mlp_set_scaling(self._h, *[_f(x) for x in a]))

    def set_output_power(self, col, powers):
        p = np.ascontiguousarray(powers, np.float32)
        _mlp_check(lib().gl_mlp_set_output_power(self._h, col, _f(p)))

    def _dev(self, a, cols):
        t = self.torch.as_tensor(np.ascontiguousarray(a, np.float32)).reshape(-1, cols)
        return t.to(self.device).contiguous()

    def train(self, X, Y, epochs, batch, lr, seed=0):
        """X, Y: host arrays or torch device tensors (float32)."""
        Xd = X if hasattr(X, "data_ptr") else self._dev(X, self.n_in)
        Yd = Y if hasattr(Y, "data_ptr") else self._dev(Y, self.n_out)
        losses = np.zeros(max(epochs, 1), np.float32)
        _mlp_check(lib().gl_mlp_train(self._h, _VP(Xd.data_ptr()), _VP(Yd.data_ptr()), Xd.shape[0], epochs,
                                      batch, lr, seed, _f(losses)))
        return losses[:epochs]

    def infer(self, X):
        Xd = X if hasattr(X, "data_ptr") else self._dev(X, self.n_in)
        Yd = self.torch.empty((Xd.shape[0], self.n_out), dtype=self.torch.float32, device=self.device)
        _mlp_check(lib().gl_mlp_infer(self._h, _VP(Xd.data_ptr()), _VP(Yd.data_ptr()), Xd.shape[0]))
        return Yd

    def infer_noalloc(self, X, Y=None):
        """Inference through gl_mlp_infer_noalloc (no device allocation in the
        library; Y, if given, is the caller's output tensor)."""
        Xd = X if hasattr(X, "data_ptr") else self._dev(X, self.n_in)
        Yd = Y if Y is not None else self.torch.empty((Xd.shape[0], self.n_out), dtype=self.torch.float32,
                                                      device=self.device)
        _mlp_check(lib().gl_mlp_infer_noalloc(self._h, _VP(Xd.data_ptr()), _VP(Yd.data_ptr()), Xd.shape[0]))
        return Yd

    def set_trust(self, lo, hi, class_col, classes, class_tol, bin_col, bin_edges, err, err_max):
        """Trust region for query(): box, classes of one column, bins of another
        and the held-out error per (class, bin) cell (gl_mlp_set_trust)."""
        f = lambda v: np.ascontiguousarray(v, np.float32)
        lo, hi, classes, bin_edges, err = f(lo), f(hi), f(classes), f(bin_edges), f(err)
        _need(err.shape == (len(classes), len(bin_edges) - 1), "err must be [classes, bins]")
        _mlp_check(lib().gl_mlp_set_trust(self._h, _f(lo), _f(hi), class_col, len(classes), _f(classes), class_tol,
                                          bin_col, len(bin_edges) - 1, _f(bin_edges), _f(err), err_max))

    def query(self, X):
        """(Y or None, verdict): the network's outputs for host rows X when the
        trust region covers them all (gl_surrogate_query); None and the
        verdict (1 outside the domain, 2 untrusted cell) otherwise."""
        Xh = np.ascontiguousarray(X, np.float32).reshape(-1, self.n_in)
        Y = np.zeros((Xh.shape[0], self.n_out), np.float32)
        v = ctypes.c_int32(-1)
        _mlp_check(lib().gl_surrogate_query(self._h, _f(Xh), Xh.shape[0], _f(Y), ctypes.byref(v)))
        return (Y if v.value == 0 else None), v.value

    def grads(self, X, Y):
        Xd, Yd = self._dev(X, self.n_in), self._dev(Y, self.n_out)
        g = np.zeros(self.n_params, np.float32)
        loss = np.zeros(1, np.float32)
        _mlp_check(lib().gl_mlp_grads(self._h, _VP(Xd.data_ptr()), _VP(Yd.data_ptr()), Xd.shape[0], _f(g),
                                      _f(loss)))
        return g, float(loss[0])

    def params(self, set_to=None):
        if set_to is not None:
            v = np.ascontiguousarray(set_to, np.float32)
            _need(v.size == self.n_params, "set_to must hold every parameter")
            _mlp_check(lib().gl_mlp_params(self._h, None, _f(v), None))
        out = np.zeros(self.n_params, np.float32)
        _mlp_check(lib().gl_mlp_params(self._h, _f(out), None, None))
        return out
