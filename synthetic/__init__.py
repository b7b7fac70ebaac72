"""Seeded synthetic inputs shared by the tests, ``bench.py`` and ``smoke()``.

This package holds parameter draws and workload recipes only: none of the
method's arithmetic (no transform, no step, no pulse formula, no mapping).
Both the library and the oracle consume what it produces.
"""
