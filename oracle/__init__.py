"""CPU oracle for MPS perturbation theory — TEST INFRASTRUCTURE ONLY.

Plain, slow, double-precision implementations written from the paper
(Sharma & Chan, "A flexible multi-reference perturbation theory by minimizing
the Hylleraas functional with matrix product states", arXiv:1408.5092):

* ``fock``    — determinant (Fock) space second quantization: ladder
  operators with Jordan-Wigner signs, excitation operators E_pq, and the
  spin-free Hamiltonian written out from its definition.
* ``exact``   — the exact (uncontracted) second- and third-order energies:
  Hylleraas functional (Eq. hyll), first-order equation (Eq. pt2) solved
  directly in determinant space, E3 by the 2n+1 rule (Eq. 3rd); plus a
  factorised sum-over-states E2 for larger active spaces, and the
  reference state Psi0 (active-space ground state, optionally compressed to
  an MPS of bond dimension M0).
* ``mpo``     — matrix product operators (Eq. mpo) for the Dyall H0 and the
  perturbation V, built term by term.
* ``mps``     — the same-algorithm two-site sweep that minimises the
  Hylleraas functional over an MPS (Eq. mps1) with dense numpy tensors.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library; the only common module is the seeded input generator
``paper_1408_5092_amd.inputs``, which holds none of the method's arithmetic.
"""
