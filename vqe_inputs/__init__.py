"""Seeded input generators shared by the oracle and the HIP path.

Integrals, the Jordan-Wigner Hamiltonian, the UCCSD rotation list and its
nearest-neighbour gate compilation.  Nothing here evaluates the MPS method.
"""
from .problem import Problem, make_problem  # noqa: F401
from .compile import GateList, compile_problem, rzz  # noqa: F401
from . import configs  # noqa: F401
