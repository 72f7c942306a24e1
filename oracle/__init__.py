"""FP64 CPU oracle for single-snapshot 2D harmonic recovery with BCCB Gram matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

Modules
-------
bccb_oracle     dictionary, Gram, eigenvalues, ISTA / FISTA / ADMM, objective, KKT
learned_oracle  unrolled learned FISTA forward and hand-derived backward

Parity status (every function is pinned by a CPU test against something other
than itself -- closed forms, brute force, textbook bounds or finite
differences -- except where a function's docstring says "parity unpinned").
"""
