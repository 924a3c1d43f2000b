"""CPU oracle for the differentiable-MPS VQE hot path -- TEST INFRASTRUCTURE.

Three tiers, each checked against the one above it and against closed forms:
T1 ``sector`` (exact fixed-particle-number simulator, no Jordan-Wigner),
T2 ``statevector`` (dense 2^N vector over the JW Pauli sum) and
T3 ``mps`` (plain FP64 complex MPS with reverse-mode gradient), and
T3b ``alg1`` (the paper's Algorithm 1 with Hamiltonian splitting on T3's MPS).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything here.  The HIP library and its Python
binding share no code with this package and never import it.
"""
