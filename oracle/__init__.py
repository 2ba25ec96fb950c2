"""FP64 CPU oracle for the Lennard-Jones Basin Hopping hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of bench.py.  The product path never imports it.
"""
