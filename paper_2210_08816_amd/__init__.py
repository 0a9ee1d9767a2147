"""MI355X (gfx950) Krylov-vector library for the linear-stability analysis of
convection in a laterally heated cube: the projected Jacobian P J(X0) x, the
steady residual, Newton corrections and Chebyshev-Arnoldi leading
eigenvalues, behind the C ABI of include/kv.h.

`paper_2210_08816_amd.kv.Context` is the Python entry point; it loads the
in-tree libkv_hip.so (built by `python -m paper_2210_08816_amd.build`).
"""
from .kv import Context, KVError, load  # noqa: F401
