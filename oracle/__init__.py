"""CPU reference (oracle) for the GeMSLR preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU library (no kernels,
headers, helpers or table generators); the only common ground is the seeded
input generator module, which holds none of the method's arithmetic.

Everything here is plain, slow and written to be checked against the paper
(Xu, Kalantzis, Li, Saad, "parGeMSLR", arXiv 2205.03224) by eye:

  partition.py  multilevel p-way vertex-separator reordering (Sec. 3, Alg. 3)
                with a geometric separator for grid graphs
  ilu.py        ILU(0) and the dual-threshold ILUT of Saad (Sec. 2.1)
  lowrank.py    Arnoldi / Krylov-Schur low-rank Schur-complement correction
                (Sec. 2.2-2.3, eqs. gemslr4 / gemslr6)
  gemslr.py     setup (Alg. 1) and apply M^{-1} (Alg. 2)
  fgmres.py     flexible GMRES accelerator (Sec. 4.1, Sec. 5)
  mlp.py        FP64 multilayer perceptron for the learned warm start
  rng.py        SplitMix64 counter-based generator for Arnoldi start vectors

Arithmetic is float64 / complex128 throughout.
"""

from . import rng, partition, ilu, lowrank, gemslr, fgmres, mlp  # noqa: F401
