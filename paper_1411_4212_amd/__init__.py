"""REWL (replica-exchange Wang-Landau) sampling of the classical Heisenberg
model on MI355X: HIP kernels behind the C ABI of include/rewl.h.

``paper_1411_4212_amd.rewl`` is the binding; ``paper_1411_4212_amd.workloads``
builds the seeded synthetic inputs.
"""
