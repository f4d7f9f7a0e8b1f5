"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package holds no arithmetic of the wave-packet method itself: it only
produces inputs -- momentum bin boundaries, partial-wave potentials evaluated
at caller-supplied momenta, and seeded parameter draws.  Both the oracle and
the GPU library compute their own Gauss nodes, projections, eigenpairs,
resolvents and observables from these inputs.
"""
from . import grids, potentials, configs  # noqa: F401
