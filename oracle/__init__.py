"""FP64 CPU oracle for the HISQ even/odd Dslash, its normal operator and solvers.

TEST INFRASTRUCTURE ONLY.  The product path (the HIP library and its Python
binding) never imports, links or runs anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg do.
It shares no code with the HIP path: the only common module is ``synth``, which
draws the seeded inputs and holds none of the operator or solver arithmetic.

Parts:
* ``hisq_oracle.c`` (built to ``_hisq_oracle.so`` by ``oracle.build``): the
  Dslash, the normal operator, CG, true residuals - plain site loops in FP64;
* ``core``: ctypes wrappers, multi-shift by independent CGs;
* ``dense``: dense-matrix construction on tiny lattices and the free-field
  closed-form spectrum;
* ``gauge``: gauge transformations and the plaquette (pins of the covariance
  tests);
* ``nn``: the gauge-covariant preconditioner network and its gradient;
* ``rational``: rational functions of the normal operator (partial-fraction
  sums by independent CGs, exact dense powers, Zolotarev's approximation of
  x^(-1/2));
* ``smear``: HISQ link smearing (fat7, U(3) projection, fat7 with Lepage term,
  Naik links) in FP64 numpy.
"""

from .core import (  # noqa: F401
    dslash,
    dslash_phased,
    dslash_sites,
    normal_op,
    cg,
    multishift_cg,
    true_residual,
    num_threads,
    library_path,
)
