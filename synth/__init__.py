"""Seeded synthetic inputs (meshes, droplet placements, request streams).

Shared by the CPU oracle's tests and the GPU library's tests and benchmark.
It contains no arithmetic of the lattice Boltzmann method.
"""
from . import cases, meshes  # noqa: F401
