"""FP64 CPU oracle for the wave-packet continuum discretisation (WPCD) path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2106_00454_amd``); the only inputs both sides share come from
the ``synth`` package.

Modules
-------
* ``wpcd``        -- the method step by step, plain NumPy/LAPACK in FP64.
* ``observables`` -- S-matrix, phase shifts (incl. Stapp mixing), kinematics,
                     linear interpolation and the total cross section.
* ``mi``          -- an independent Lippmann-Schwinger matrix-inversion solver.
* ``yamaguchi``   -- the closed-form on-shell T-matrix of the Yamaguchi
                     separable potential, with a finite momentum cut-off.

Parity status of each function is stated in its module docstring; functions
without an independent pin say "parity unpinned".
"""
from . import wpcd, observables, mi, yamaguchi  # noqa: F401
