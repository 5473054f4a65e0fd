"""CPU FP64 oracle for the DD-alpha-AMG twisted-mass clover Wilson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only tests/, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two
meet only through the seeded generators in lattice_inputs/.

Every function is written from the paper (arXiv:1710.06198) and from the
standard definitions it relies on, in plain complex128 torch-CPU code with
no blocking or fusion beyond what the definition states:

  dirac.py  the operator D(mu) = D + i mu Gamma5 (Sec. 1, Sec. 1.1) with
            the clover term, Gamma5-hermiticity, free-field closed forms
  mg.py     aggregation P (Sec. 1.1), Galerkin D_c = P^dag D P, SAP with MR
            block solves, GMRES/FGMRES, the error propagation of Eq. (1),
            the adaptive setup, two-step and shifted solves (Sec. 1.1)
  force.py  the pseudofermion force of S_f = phi^dag (D D^dag)^-1 phi
  mcrit.py  the bare mass m0 from the smallest-real-part eigenvalue
  evenodd.py  the even-odd Schur complement of D(mu)
  nd.py     the non-degenerate doublet D_ND(mubar, epsbar) of Eq. (2) and its
            unit-link momentum-space solve

All functions are pinned by tests/test_oracle_*.py against closed forms,
exact identities, brute force on tiny lattices and dense solves.
"""
