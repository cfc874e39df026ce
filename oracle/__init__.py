"""FP64 CPU oracle for the Stokes kernel sums -- test infrastructure only.

Imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``; never by the product package.
"""
