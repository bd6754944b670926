"""FP64 CPU oracle for the clip-and-verify hot path (test infrastructure).

This package is the reference that the GPU path is checked against.  It is a
plain, slow, float64 NumPy restatement of what the paper (Clip-and-Verify:
linear constraint-driven domain clipping, arXiv 2512.11087) computes:

* ``box``       - concretization of a linear function over a box (Lemma A.2,
                  eq. 1 of the preliminaries);
* ``relaxed``   - relaxed clipping: single-constraint closed form (Thm 3.2),
                  parallel (Alg. 2) and sequential (Alg. 3) multi-constraint
                  forms;
* ``complete``  - complete clipping: the 1-D Lagrange dual of one constraint
                  (Thm 3.1), its continuous-knapsack twin (appendix on the
                  knapsack equivalence) and one pass of coordinate ascent over
                  several constraints (Alg. 1, eq. 4);
* ``crown``     - CROWN backward bound propagation (Lemma A.3 and the
                  plane recursion of appendix A.3) and the root pass that
                  caches per-neuron planes;
* ``pipeline``  - the batched per-subdomain pipeline (split constraints,
                  eqs. 9-10 -> relaxed clip -> re-concretize cached planes ->
                  CROWN -> concretize -> complete clip), the slope (alpha)
                  adjoint and Adam;
* ``exact``     - independent exact checkers for tiny problems: vertex
                  enumeration and a hand-written simplex in rational
                  arithmetic.

It is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP library and never imports it.

Where the paper is silent or garbled the oracle follows a stated reading;
each is named in the docstring of the function that takes it.
"""

from . import box, relaxed, complete, crown, pipeline, exact  # noqa: F401
