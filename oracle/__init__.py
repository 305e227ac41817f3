"""CPU FP64 oracle for the stochastic Galerkin solver -- TEST INFRASTRUCTURE.

This package is a plain, slow, readable restatement of what the method of
arXiv 2310.14649 computes (stochastic Galerkin projection of the log-normal
Poisson problem, Sec. 2; two-grid restricted additive Schwarz preconditioned
flexible GMRES, Sec. 3).  It exists only to check the HIP implementation:
only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It imports nothing from the GPU package and shares
no code with it; both consume the arrays of the seeded input generator.

Modules
-------
pce      multi-indices, Hermite triple products, log-normal input PCE
fem      P1 stiffness matrices per input PCE term, load vector
sg       the coupled SG operator and its right-hand side
ras      overlap growth and the one-level restricted additive Schwarz map
coarse   Nicolaides coarse space and the Galerkin coarse operator
amg      smoothed-aggregation AMG hierarchy and its V-cycle
precond  the multiplicative two-level composition
krylov   flexible GMRES(m)
stats    mean / variance of a PCE field, Monte Carlo and collocation checks
cond     condition number of the SG operator against the deterministic one

Every function is in FP64 and cites the passage of the paper it restates.
Readings of passages that are silent, ambiguous or garbled are stated in
the docstrings where they are used.
"""
