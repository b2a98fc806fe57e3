"""CPU oracle for the double-double / quad-double Newton path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the only common inputs come from the seeded generators in ``synth/``.

Everything here is written from the paper (Verschelde & Yoffe, "Quality Up in
Polynomial Homotopy Continuation by Multithreaded Path Tracking", 2011) and
from textbook definitions, plainly and slowly:

* ``numbers``  -- exact values of multiword (DD/QD) numbers, Gaussian rationals
* ``arith``    -- exact results of the multiword operations (Section 1:
  double-double / quad-double arithmetic)
* ``evaluate`` -- the plain definition of a sparse system, its Jacobian and the
  total-degree homotopy (Section 4 array Y; Section 6 derivative monomials)
* ``newton``   -- Newton's method with the loop of Algorithm 4.1, linear solve
  by a library LU (mpmath.lu_solve)
* ``track``    -- path tracking with the loop of Algorithm 3.1, endpoint
  refinement, an FP64 tracker used to identify start roots, correct digits
* ``mlp``      -- FP64 reference of the step-size network (not in the paper)
* ``quality``  -- speedup and quality-up arithmetic of Section 2

Parity status of each function is stated in its docstring; see also the
module headers.
"""
