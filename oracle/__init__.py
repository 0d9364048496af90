"""CPU FP64 oracle for the RbmSAT block-Gibbs hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path
(``paper_2311_02101_amd``); both sides receive the same seeded inputs and each
implements the counter-based generator from its published definition.

Modules:
  philox  -- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), NumPy uint64.
  rbmsat  -- free energy (eq. 1), negation transform (eq. 4), formula-RBM
             assembly and the block-Gibbs sweep (eqs. 2-3, 6-7), clause count,
             best tracking and variance EMA, in FP64.
"""
