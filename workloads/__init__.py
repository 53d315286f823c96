"""Seeded synthetic inputs (conductivity fields, flow solve, particle release).

Shared by the oracle tests and the GPU path; holds none of the tracking
arithmetic.
"""
