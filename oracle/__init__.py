"""FP64 CPU oracle of the particle-side CFD-DEM hot path.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of bench.py.  The HIP library and its binding never import it.
"""
