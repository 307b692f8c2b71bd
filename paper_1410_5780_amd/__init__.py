"""pv3d: GPU shadow-map shading losses for PV generators on MI355X (gfx950).

The package holds the Python side of the C-ABI library ``libpv3d.so``:

* :mod:`paper_1410_5780_amd.pv3d` -- ctypes binding of ``include/pv3d.h``
  (argument marshalling only; every step of the path runs in HIP kernels).
* :mod:`paper_1410_5780_amd.workloads` -- seeded synthetic inputs (scenes,
  PV generators, sun sweeps). It holds none of the method's arithmetic.
* :mod:`paper_1410_5780_amd.serve` -- the request driver for the serving path.

Importing the package does not load the shared library; the binding loads it
on first use and raises if it is missing.
"""

__all__ = ["pv3d", "workloads"]
