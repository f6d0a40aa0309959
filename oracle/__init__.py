"""Independent FP64 CPU oracle for the macro-element HDG local-problem path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
here, and this package imports nothing from the product except the seeded
input generators (which hold no discretisation arithmetic).

What it computes is the plain definition of the discrete problem: the weak
form of the hybridised method on C0 macro-element spaces (paper section 3.1,
eq. weak_form, with the interpolation spaces of section 3.2), assembled by
quadrature in physical coordinates, statically condensed (section 3.3.1,
eqs. global_problem / local_problem) and solved directly.  No blocking, fusion
or reordering beyond those equations.

Pins (see tests/test_oracle_*.py): exact monomial quadrature, closed-form dof
and face counts (complexity section, tables 1-2, and the dof tables of the
numerical-results section), exact reproduction of degree-p polynomial
solutions, a dense brute-force solve of the unhybridised system, L2
convergence of order p+1, the macro-element conservation and weak flux
continuity identities, finite differences for the adjoint.
"""
