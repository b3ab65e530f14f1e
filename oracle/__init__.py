"""Plain CPU oracle for the Riccati-sweep method (complex FP64, NumPy).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(the HIP library and its Python binding) never does.

The oracle is written from the paper (Sec. II, II.A, III.A, App. C, App. D,
App. E, App. F) and shares no code, tables or helpers with the HIP path.
Each function cites the passage it follows.  Where the paper is silent, the
reading taken is stated in the docstring of the function that implements it.

Modules
  tables    Ozaki poles/residues, Fermi-surface quadrature, basis functions
  geometry  grain shapes, mask, rotated lattices, trajectory segments
  sweep     interpolation, implicit-midpoint Riccati march, Green's
            functions, rotate-back, specular boundary taps
  fields    external gauges, 2D Laplacian Green's function, A-solve
  scf       one iteration map, Picard SCF loop, LDOS
  bulk      closed forms of the homogeneous state (pins)
  annulus   London-Maxwell closed forms of a screened annulus (pins)
  disc      superflow free energy of an unscreened disc (pins)
"""
from . import tables, geometry, sweep, fields, scf, bulk, annulus, disc  # noqa: F401
