"""FP64 CPU oracle for the FC-DOM time step of the 2-D time-domain RTE.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
NumPy/mpmath restatement of what the method computes (Gaggioli & Bruno,
"Parallel inverse-problem solver for time-domain optical tomography with
perfect parallel scaling", Sec. 2-4).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The HIP library never imports, links or reads anything here, and
this package imports nothing from the library: the only code both sides see
is the seeded input description in ``workloads``.

Modules
  fc_gram  -- Gram basis and blend-to-zero continuation tables (Sec. 4.3)
  fc       -- FC-Gram continuation + filtered spectral derivative and its
              transpose (Sec. 4.3, eqs. RTEFCSum, FFilter, RTEFCSumder)
  physics  -- ordinates, Henyey-Greenstein matrix, Fresnel law, boundary map,
              beams and detectors (Sec. 2, 3.1, 4.1)
  solver   -- AB4 forward solve, misfit, exact discrete adjoint and gradient
              (Sec. 3.2-3.6, 4.2, Algorithm 1)
  cadjoint -- the continuous adjoint problem solved as a reversed forward
              problem, and its gradient (Sec. 3.3-3.6, eqs. AdjointProblem,
              FDwin22)
  mms      -- the manufactured-solution problem: exact solution, source and
              start-up history (Sec. 5, eqs. RTEdisp, RTEmansol)

Every function states the passage it follows.  "parity unpinned" marks the
readings the paper leaves open and nothing outside the oracle can confirm:
the exact FC blend-table values (the paper prints none) and the HG exponent
(3/2 as printed; no scattering numbers are printed).
"""
