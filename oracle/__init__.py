"""Test infrastructure: plain, slow CPU oracles for the Jamiolkowski fidelity of a noisy circuit.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this package.  The
fidelity library never imports, links or calls anything here, and nothing here imports the
library (the two share only the seeded instance descriptions).
"""
