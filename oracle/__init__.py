"""CPU oracles for DBSCAN -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  ``dbscan_oracle`` is the numpy float64 reference;
``c_oracle`` wraps the plain C float64 reference (``dbscan_oracle.c``).
"""
