"""Seeded synthetic inputs (meshes, right-hand sides, request streams).

This package is shared by the oracle and the GPU library's tests and
benchmarks; it holds none of the boundary-operator arithmetic.
"""
from . import meshes, rhs, cases  # noqa: F401
