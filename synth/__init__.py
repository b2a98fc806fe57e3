"""Seeded synthetic inputs for the polynomial-homotopy Newton path.

This package is the only code shared between the CPU oracle (``oracle/``)
and the HIP path (``paper_1109_0545_amd``).  It draws random numbers and
rounds transcendental constants to double-double / quad-double limbs; it
holds none of the method's arithmetic (no monomial products, no Jacobian,
no elimination).
"""

from .systems import (  # noqa: F401
    CONFIGS,
    Config,
    System,
    limbs_of,
    make_system,
    random_point,
    start_root,
    unit_phasor,
)
