"""CPU oracle for the two-site DMRG hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 (complex128) NumPy implementation of what the GPU path
computes, written from the paper's statement of the method:
  - the Bose-Hubbard Hamiltonian (Sec. 5, Eq. 2) and its exact diagonalisation,
  - its matrix product operator (Sec. 4.3, the MPS-MPO-MPS network figure),
  - U(1) block tensors (appendix A.1.1, symmetric nodes),
  - the two-site effective Hamiltonian applied to a vector (Sec. 4.2, the
    H_eff contractor; pairwise contraction as in appendix B.1.1),
  - an iterative lowest-eigenpair solver driven by that contractor (Sec. 4.2),
  - the truncated SVD with the paper's four truncation rules and error
    definition (appendix B.1.2, Eq. trunc_err),
  - the spin-1 Heisenberg chain of the paper's DMRG timing table (Sec. 3,
    Table tab:dmrgtimes): its Hamiltonian, exact diagonalisation and MPO,
  - the variational sweep (Sec. 4.3), here in two-site form.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this package.  It shares no code with the GPU library and never consumes
anything the GPU path produced; both sides read the seeded inputs of `synth`.

Pins: every function here is checked by `tests/test_oracle_*.py` against
closed forms, brute force, invariants or library special cases (see each
function's docstring).  Parity unpinned: the absolute energies of the U > 0,
chi-limited chains (cfg2..cfg5 sizes) have no closed form; they are pinned
only through the invariants and the exactly solvable limits run at the same L.
"""
from . import model, blocks, heff, lanczos, svd, dmrg, flops  # noqa: F401
