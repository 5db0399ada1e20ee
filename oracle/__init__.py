"""FP64 CPU oracle for the closed-shell CCSD-form residual, energy and Jacobi/DIIS solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never calls into it, and the
two share no code: only the seeded input recipes in ``gen/`` serve both.

Contents, each module citing the passage of the paper it follows:

* ``bruteforce``  -- the definition itself: the projections of e^{-T} H e^{T}|phi_0>
  onto the reference and onto singly and doubly excited determinants, evaluated in
  the full determinant space (paper Sec. II.A, Eqs. (eqn:energy), (eqn:amp); the
  cluster operator convention of Eq. (eqn: CC equation) and the T_N definition after it).
* ``so_ccsd``     -- spin-orbital CCSD residuals and energy (textbook factorisation),
  pinned to ``bruteforce`` on tiny inputs.
* ``cs_ccsd``     -- closed-shell spin-adapted residuals in T1-dressed form, pinned to
  ``so_ccsd`` through the spin-adaptation relations (Supporting Information S1).
* ``solver``      -- diagonal approximate-Jacobian update with DIIS (Sec. III.B) and the
  convergence test (Sec. III.A).
* ``ascc``        -- the transformed Hamiltonian Hbar = e^{S^dagger} H e^{-S^dagger} of a 1-CSF
  state (Eqs. (eqn:1CSF-S), (eqn: sim)) and the initial guess T^P(0) = S - S^2/2
  (Eq. (eqn:TP-guess)), pinned to determinant-space matrix exponentials and to the
  two-electron limit.
* ``triples``     -- the 1-CSF mixed triples T^M_3' (Sec. II.B.1, Eq. (eqn:H1TP)): the slice of
  triples with at least three primary spin orbitals, its spin-orbital working equations in
  T1-transformed form and their couplings into the closed-shell singles and doubles, and an
  ASCCSD solve; pinned to brute-force projections with T3 (``bruteforce`` extended to triples).
* ``plascc``      -- the partially linearised residual (Sec. II.C): the closed-shell residual
  without its terms with two powers of the mixed doubles T^M (Eq. (eqn: pnm split)), pinned to
  brute-force projections with T^M taken in the spin-orbital basis.
"""
