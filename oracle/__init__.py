"""Plain float64 CPU oracle for the Moment Tensor Potential hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the library; the two meet only in the seeded input generators of
``workloads``.

Modules:
  basis      brute-force enumeration of the basis functions
  neighbors  brute-force canonical periodic neighbour list
  mtp        energies, forces, virial, grade and parameter gradients
  maxvol     active-set update by MaxVol row swaps

Every function here is pinned by tests under tests/ (test_oracle_*.py)
against closed forms, invariants, library routines and brute force.
"""
