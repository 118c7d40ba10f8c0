"""MI355X (gfx950) library for the boost-invariant SU(3) Glasma coupled to a
colored-particle-in-cell solution of Wong's equations, after Avramescu et al.,
Hard Probes 2023.  The compute path is libglasma.so (HIP); this package is its
thin Python binding."""
from .glasma import (MLP, Batch, Event, GlasmaError, KIND_HEAVY_QUARK, KIND_JET, lib, rates_from_series,  # noqa: F401
                     max_particles, required_bytes, GL_OK, GL_EINVAL, GL_ESTATE, GL_ENOTCONV, GL_ENUMERIC,
                     GL_EDEVICE, GL_ENOMEM)
