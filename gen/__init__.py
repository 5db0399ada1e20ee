"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds random-number recipes only: no coupled-cluster arithmetic.
"""
