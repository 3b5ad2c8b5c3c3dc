"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds geometry (meshes, boundary tags, curved midside nodes),
seeded boundary-waveform coefficients and boundary-data evaluation. It holds
none of the method's arithmetic (no assembly, no solve, no synthesis), so
that the oracle and the GPU path can be fed identical inputs while sharing
no code.
"""
from .meshes import channel_mesh, pipe_mesh, pipe_mesh_for_tets, Mesh  # noqa: F401
from .waveforms import harmonic_coefficients, period_set  # noqa: F401
from . import cases  # noqa: F401
