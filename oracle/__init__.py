"""FP64 CPU oracle for the Wilson-fermion HMC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes anything in this package: only ``tests/``, the ``smoke()`` check
in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously correct NumPy complex128 implementation
of what the hot path computes, on the full lattice (shifts by ``np.roll``),
with explicit 4x4 gamma matrices (no even/odd split, no spin projection), a
textbook unpreconditioned CG on D^dagger D, and forces written as the gradient
of the action.  It shares no code with the HIP path; the only common module is
``lgt_inputs`` (seeded random fields).

Modules and the parts of the paper they follow:

* ``su3``     su(N) projection (eq. 7 / S2.9), the left update exp (eq. 5, S2.1)
* ``lattice`` periodic shifts of site fields
* ``dirac``   Wilson-Dirac operator D(U) and D^dagger (the operator of S3.1;
              the paper names it but does not write it out)
* ``solver``  CG for A chi = phi with A = D^dagger D (S3.6, "Remarks on the
              role of the linear solver")
* ``action``  Wilson plaquette action, pseudofermion action S_f (S3.1), kinetic
              energy
* ``force``   matrix gradient G = dS/dU_R + i dS/dU_I (S2.12), force
              F = -1/2 P_su(3)[U G^dagger] (S2.9, S2.15 and the S4 listings),
              fermion force via delta S_f = -2 Re[eta^dagger (delta D) chi]
              (S3.12) and the building block I(U) = a^dagger D(U) b (S3.13)
* ``md``      leapfrog molecular dynamics (eqs. S2.1-S2.2; Sec. III B), Delta H
* ``stout``   stout smearing (Morningstar-Peardon) and its gradient through
              torch CPU autograd
"""
