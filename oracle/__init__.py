"""Plain, slow FP64 CPU oracle of the fourth-order entropy-stable lattice Boltzmann time loop.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (``paper_2403_13406_amd`` + ``libeslb.so``) never routes through it,
and the two share no code: this package imports nothing from the product and the
product imports nothing from here.  Only seeded input arrays are passed to both.

Source: Bellotti, Helluy, Navoret, "Fourth-order entropy-stable lattice Boltzmann
schemes for hyperbolic systems" (arXiv 2403.13406).  Every function cites the
section / equation / table it follows.

Modules
-------
lattice      D1Q2 / D2Q4 velocity sets, transport T(s) (eq. transportPhase),
             time step (Sec. 2.3), step count reading.
systems      target systems (Sec. 1.1), equilibria (Sec. 1.2.1-1.2.2),
             kinetic entropies (Examples of Sec. 1.2), population states and the
             per-population Bregman divergences used to solve for omega (Sec. 4).
relaxation   R_omega (eq. relaxationDiscretizationOmega) and the entropy-limited
             omega (eq. variableOmegaProblem, Sec. 5.1 factorisation).
scheme       basic brick psi (eq. basicBrickSplitting) and the composition Phi
             (eq. splittingToUse); standard LB comparator (Sec. 3.1); Schemes II/III
             (Sec. 6.1).
diagnostics  conserved sums, total microscopic entropy, macroscopic entropy (Sec. 4).
exact        exact solutions and L2 / Err-Estim norms (Sec. 3).
adjoint      plain adjoint of one relaxation stage and of the composed step.

Parity status: every function is pinned by a ``-m "not gpu"`` test against the
paper's printed values or an independent closed form / brute force, except
where a header says "parity unpinned".
"""
