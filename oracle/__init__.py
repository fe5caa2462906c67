"""FP64 CPU oracle for slice-and-match orientation determination.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The GPU library never does, and shares no code, tables or constants with it.

Plain, slow, obviously correct NumPy in float64.  Each function cites the
passage of the SpiniFEL paper (arXiv 2109.05339) it follows:

* slicing, section II-A: M model images on a fixed orientation set as the
  type-2 (uniform -> nonuniform) NUFFT of the autocorrelation;
* orientation matching, section II-B: every image against every model image,
  Euclidean distance, nearest model image wins;
* merging, section II-C, Eq. (1)-(2): the type-1 NUFFT A* (with weights D)
  as the adjoint of slicing, and the regularised normal equations of
  Eq. (2) with their Toeplitz form, conjugate gradients and the L-curve;
* phasing, section II-D: error reduction, hybrid input-output and
  shrinkwrap between the density and its measured Fourier amplitudes.

The paper fixes no NUFFT internals; it names the ES-kernel library of its
reference [barnett2019parallel].  The readings used (kernel, width, shape
parameter, grid, support rule, sign convention) are listed in the module
docstrings and pinned against exact direct sums in ``tests/``.

Parity status: every function below is pinned by a CPU test (closed forms,
brute force, library routines or invariants), except where its docstring
says "parity unpinned".
"""
from . import es, geometry, nudft, nufft, match, grad, normal, phasing  # noqa: F401
