"""MI355X-native SCF / MEX expansion force calculation (arXiv:1406.4254).

The compute path is the C-ABI library ``libetics.so`` (HIP kernels for gfx950),
reached through :mod:`paper_1406_4254_amd.etics`; :mod:`paper_1406_4254_amd.workloads`
draws the seeded synthetic inputs.  Nothing is imported eagerly, so the input
generators work on hosts without a GPU.
"""
__all__ = ["etics", "workloads"]
