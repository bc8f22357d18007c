"""Plain CPU oracle for the two-dimensional Fourier Continuation (2D-FC) hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product (the ``paper_2010_03901_amd``
package and its C-ABI library) imports, links or calls anything here; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` do.  The oracle shares no code, tables or helpers with the HIP
path: it builds its own FC-Gram tables (mpmath), its own geometry and its own
interpolation, following Bruno & Paul, "Two-dimensional Fourier Continuation
and applications" (arXiv 2010.03901) step by step.

Modules
  fcgram    -- Gram basis, oversampled Gram values, SVD trigonometric matching,
               continuation matrices A and A_r (Sec. 2.2, Remark 2.2)
  fc1d      -- the full 1D-FC of Sec. 2.3 (used only to pin the tables)
  curves    -- boundary parametrisations q(theta), normals, curvature
  plan      -- "Geometrical Setup": boundary grid, admissibility,
               classification of H, proximity map, foot of the normal,
               matching stencils (Sec. 3.1, 3.2, 3.3, 3.4 and Sec. 3.5 steps 1-4)
  extend    -- "Cartesian Evaluation": matching values, blending to zero on
               V+_{B,C_r}, interpolation onto H and assembly (Sec. 3.2, 3.4,
               Sec. 3.5 steps 5-6)
  spectral  -- 2D FFT (Sec. 3.5 step 7), Poisson particular solution
               (Sec. 4.1), Fourier-Forwarding modal propagation (Sec. 4.2)

Precision: float64 throughout, except that the matching-value step and the
Gram projection Q^T f_D are evaluated in numpy.longdouble (x87 80-bit) and the
FC-Gram tables in mpmath (50 digits); see ``extend.matching_values``.
"""
