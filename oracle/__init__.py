"""CPU oracle for symmetric (abelian) TensorMap permutes and contractions.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (``paper_2508_10076_amd``) and imports nothing from it.

Modules
-------
graded     sectors of the supported symmetries, graded spaces, and the storage
           layout of a TensorMap (block per coupled charge, one column-major
           matrix each).  Section "Grouping And Splitting Indices" of the
           abelian chapter (eq. abeliangrouping) and eq. linearindex.
dense      O1: plain dense definitions.  Bosonic permute = array transpose,
           contraction = tensordot (sections "Permutations", "Pairwise
           Contractions").  Fermionic networks: a graph evaluator that applies
           the SVect braiding sign R^{JJ}_I = -1 to every crossing and the
           pushed-twist pairing (section "Fermions and fusion categories").
blockwise  O2: plain per-channel implementation of Alg. "Abelian Tensor
           Permutation" and Alg. "Abelian tensor contraction", fp64, one numpy
           transpose per channel and one numpy matmul per coupled sector.
sampled    O1 evaluated entry by entry (for outputs too large to expand).
flops      useful block flops of a contraction (sum over sectors of 2 M N K).

All floating point is float64.  Every function cites the passage it follows.
"""
