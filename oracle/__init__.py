"""Plain CPU oracle for particle-wise higher-order SPH ray fields.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  The GPU library
(``paper_2401_02896_amd``) never imports, links or reads anything from here, and
nothing here imports the GPU library: the two share no code.

Everything follows "Particle-Wise Higher-Order SPH Field Approximation for DVR"
(arXiv 2401.02896) step by step, in float64 and, for the quantized
accumulation, in Python integers (no wrap-around).  Each function names the
passage of the paper it implements.  The modules are:

* ``kernels``  - SPH kernels w(r), their constants kappa, kappa' and the column
  integral of a kernel along a line (closed form).
* ``quanta``   - the quantization error estimate Q_D and the choice of the length
  quantum tau and value quantum sigma (Sec. 4.4, App. A.4/A.5).
* ``lut``      - the candidate space, its basis, the L2-optimal projection of the
  ray-restricted kernel for fixed knots, the knot optimisation and the table
  of localized difference coefficients (Sec. 3.2-3.4, App. A.1/A.2).
* ``geometry`` - rays, camera ray generation, the particle/ray relation
  (distance parameter and closest-point parameter, Fig. 1) and the hit test.
* ``grid``     - the multi-level Morton grid the library indexes particles with
  (no counterpart in the paper; defined so that its keys can be checked).
* ``knots``    - quantized knots of one particle on one ray, with the integer
  closure rules (Sec. 4.3, App. A.3).
* ``field``    - per-ray sort and exact integer accumulation (Eq. accumulation
  rule), exact pieces, the ray's peak and the error-bounded merge.
* ``render``   - classification and front-to-back compositing.

Parity status of every function is recorded in its module docstring.
"""
