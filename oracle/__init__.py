"""Plain FP64 CPU oracle for the plane-wave H*psi / block-Davidson path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path
(``paper_1709_10010_amd``) never does, and the two share no code.

Every function follows the mathematical definition it cites, with library
primitives (numpy FFT, matmul, LAPACK eigh) as single steps and no
blocking, fusion or reordering beyond that definition.

Modules
  gsphere      plane-wave sphere and kinetic energies
  grid         sphere <-> grid maps, grid FFTs, direct-sum DFT
  hamiltonian  H*psi (FFT path) and the dense H matrix
  davidson     block Davidson with the Teter-Payne-Allan preconditioner
  mlp          the learned preconditioner's network, loss and optimiser
  lanczos      Lanczos recursion on H and the continued fraction of its resolvent
  scf          density, Hartree and local exchange potentials, mixing, the SCF loop
  exx          the Fock exchange operator and its adaptively compressed form (ACE)

Parity status: every function is pinned by a test in
``tests/test_oracle_pins.py`` except the iteration counts and wall time of
``davidson`` ("parity unpinned": the paper prints no such numbers).
"""
from . import gsphere, grid, hamiltonian, davidson, mlp, lanczos, scf, exx  # noqa: F401
