"""FP64 CPU oracle of the heuristic VarLiNGAM hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never calls it, and it shares no code with the GPU library (the
seeded input generator in `synth` is the only module both sides use, and it computes none of
the method's arithmetic).

Contents (plain, slow, obviously correct NumPy in float64):
* `varlingam`  -- VAR fit, standardisation, pairwise residual (Eq. 1), entropy score (Eq. 2),
                  pairwise score matrix, approximate ordering (Alg. 1), B estimation, and the
                  original iterative DirectLiNGAM (Sec. 3 steps 1-5) as a comparator.
* `backward`   -- an independent torch-CPU float64 re-implementation of the score for
                  reference gradients.

Parity status per function is listed in the module docstrings ("pinned by" / "parity
unpinned").
"""
