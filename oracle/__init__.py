"""Independent FP64 CPU oracle for the H^2-ULV factorization and solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute anything in this package: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg use it.

The oracle follows Ma & Yokota, "An inherently parallel H^2-ULV factorization
for solving dense linear systems on GPUs" (arXiv 2502.02395), step by step and
in the paper's notation, with numpy/scipy LAPACK routines as single steps and
no blocking, fusion or reordering beyond what the paper states:

  kernels.py    kernel functions G(x, y) (Eq. 35, Eq. 36 and covariance kernels)
  tree.py       binary cluster tree, box geometry, near/far lists (Section 3.3,
                admissibility as defined in Section 6.2)
  construct.py  H^2 construction with pre-factorization (Algorithm 1,
                Sections 3.4-3.5): sampling, A_Close, interpolative decomposition
  h2matrix.py   the H^2 operator: nested bases, dense assembly, matvec
  ulv.py        ULV factorization (Algorithm 4 with an orthogonal QR completion
                of the shared basis, Eq. 32), the parallel substitution
                (Eq. 24-31), the naive block substitution (Algorithm 3) and
                iterative refinement / PCG
  flops.py      the canonical algorithmic flop count
  mlp.py        FP64 reference of the rank-predictor MLP (forward, backward,
                Adam) used to check the GPU training kernels
  ulv_lu.py     the LU variant of the factorization and substitution for
                non-symmetric kernel matrices (the paper states the method for
                symmetric positive definite matrices only; this variant keeps
                its structure with a pivot-free LU of the redundant blocks)

Each function's docstring cites the passage it follows and states the
reading it takes where the paper is silent or garbled.
"""
