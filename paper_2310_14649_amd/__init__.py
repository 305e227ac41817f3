"""MI355X-native intrusive stochastic Galerkin solver (arXiv 2310.14649).

The hot path lives in ``libsgsolve.so`` (HIP for gfx950, C ABI declared in
``include/sgsolve.h``); ``binding`` marshals arguments to it and
``inputs`` generates the seeded synthetic problem instances.
"""
__all__ = ["binding", "inputs"]
