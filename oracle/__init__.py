"""Oracle for the streaming subgraph matcher -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU path
computes, used to prove parity:

  * ``core``        ctypes wrapper of ``mnemonic_oracle.c``, a single-threaded
                    incremental matcher (problem definition of Section II-B,
                    batch phases of Algorithm 1, work units and the
                    duplicate-removal mask of Section VI).
  * ``brute``       brute force over every vertex map and every edge-instance
                    choice, for tiny graphs (pins ``core``).
  * ``closed_form`` homomorphic counts of labelled directed paths via sparse
                    matrix-vector products (pins counts at full size).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything here. The product library never does, and
this package imports nothing from it.
"""
