"""FP64 CPU oracle for multi-bandwidth Gaussian summation (Lee & Gray, "Faster
Gaussian Summation: Theory and Experiment").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(`paper_1206_6857_amd`), and the library does not depend on it.

Modules
-------
exp64        own double-precision exp (Cody-Waite reduction + Taylor
             polynomial); used for every value that decides a pruning, so
             that decisions are reproducible bit for bit.
multiindex   graded multi-index sets for O(D^p) expansions (section 2).
hermite      Hermite functions h_n(t) = exp(-t^2) H_n(t) (section 1, note 2).
series       Hermite moments, H2H, H2L, L2L, direct Hermite evaluation,
             direct local accumulation, local evaluation (sections 1-3,
             Lemmas 1-3).
bounds       truncation-error bounds E_DH, E_DL, E_H2L (Lemmas 4-6) and the
             finite-difference error E_FD (section 5).
exhaustive   the plain definition G(x_q) = sum_r w_r exp(-|x_q-x_r|^2/2h^2)
             (section 1), FP64.
kdtree       kd-tree with cached statistics (section 6, Figure 5).
dualtree     the dual-tree algorithm with token error control (section 5,
             Theorem 2; section 6, Figures 6-8) run level by level, plus the
             depth-first form printed in the paper; it can also replay
             another run's choices after certifying each with its own bounds.
mlp          the pair-policy network (two ReLU layers), its masked squared
             loss, gradient and one Adam step, in FP64.
policy       features, cost-to-go and training records of the pair policy,
             computed from a decision trace.

Every function that has no independent pin says "parity unpinned" in its
docstring.  All functions here are pinned by tests under `tests/`.
"""
