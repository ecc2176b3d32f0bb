"""CPU FP64 oracle for FCG-NO.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never routes through
it, and it shares no code with the HIP library; the two meet only through the
seeded generators in ``synth``.

Every function is written from the paper (Rudikov et al., "Neural operators
meet conjugate gradients: the FCG-NO method", ICML 2024) and cites the passage
it follows.  Plain definitions are written out; library primitives (FFT,
sparse direct solve, autograd) serve as single steps.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  stencil_apply / assemble     pinned: sine-mode eigenpairs, Dirichlet energy
  fcg                          pinned: FCG(I) == textbook CG, PCG(Jacobi),
                               one-step convergence with A^-1, A-orthogonality,
                               energy identity, finite termination, Table 1
  no_apply                     pinned: brute-force explicit-sum operator on tiny
                               grids, exact homogeneity, B(0) = 0
  sine-basis layer             pinned: analysis equals scipy's DST-I, the layer
                               with weights 1/lambda inverts constant-k A on the
                               kept sine modes and drops the others
  notay_loss / l2_loss         pinned: closed-form values on eigenvectors
  loss gradients (autograd)    pinned: central finite differences
  jacobi / sgs                 pinned: Table 1 iteration counts (statistical)
  sgs / rb_sgs                 pinned: the textbook SGS matrix (D+L) D^-1 (D+U) on
                               tiny grids, k-step error propagation, symmetry,
                               red-black colouring and point-sweep form
  adamw_step                   pinned: hand-computed first steps
  Theorem 1's gamma            not used; parity unpinned (not computed)
"""
from .fcgno_ref import *  # noqa: F401,F403
