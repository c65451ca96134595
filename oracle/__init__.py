"""CPU FP64 oracle for the nonlinear spectral multigrid (FAS) method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or execute anything in
this package.  The GPU library never calls it, links it or shares code with it.

It is a plain, slow, direct transcription of what the paper defines, written
for reading against the paper:

* ``fv``       -- TPFA half-transmissibilities and the mixed fine-level system
                  (Section 2.1, eqs. half-transmissibility and FV_matrix).
* ``levels``   -- the level operator A^l(x) assembled cell by cell from static
                  local matrices scaled by 1/kappa of the piecewise-constant
                  pressure (Section 3.2, Prop. 1; Appendix B), and its Picard
                  and Newton linearisations (Section 3.3, Props. 2 and 3).
* ``coarsen``  -- box aggregation, renumbering, local spectral problems,
                  PV traces, trace extensions, bubbles, P, Q and the static
                  coarse local matrices (Section 3.1, Appendix A).
* ``solvers``  -- backtracking (Alg. 1), the exponential-kappa step cap
                  (Section 4.1), Picard/Newton smoothing, the FAS V-cycle
                  (Alg. 2) and single-level Picard/Newton (Section 2.2), all
                  with exact sparse-direct linear solves.

Where the paper is silent or ambiguous, the reading taken is stated next to
the code that takes it.
"""
