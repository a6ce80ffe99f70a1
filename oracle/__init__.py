"""CPU oracle for the frame-potential hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library in ``paper_2205_09900_amd`` and neither imports
the other; both take seeded raw inputs from ``synth``.

Modules (each cites the passage of the paper it follows):
  philox        Philox4x32-10 counter generator (published definition)
  sampler       the ensembles: brickwork, local random, HEA (RY RZ + CZ), and
                the paper's HEA (RY(pi/4) wall, Pauli rotations, CNOT or CZ walls)
  dense         Tr(U^dagger V) from dense 2^n x 2^n unitaries (n <= 12)
  ancilla       the paper's single-amplitude construction (n <= 10)
  mpo           MPO-zip contraction for wide, shallow circuits (n up to 50)
  estimator     Monte Carlo F^(k), standard error, bootstrap, control variate
  statistics    Philox bootstrap, quantiles, fit region, layers to epsilon,
                sample-size rule
  haar_moments  F_Haar^(k) for U(d) by counting permutations
  weingarten    exact brickwork F^(k) by the permutation transfer
  closed_forms  special-case traces and frame potentials
  mlp           float64 reference forward/backward of the surrogate network
  qudit         brickwork of Haar U(q^2) gates on qudits: sampler, dense, MPO-zip

Parity status: every module is pinned by the tests in tests/test_oracle_*.py
against published values, closed forms, brute force or an independent
algorithm.
"""
