"""MI355X (gfx950) ABAC-preconditioned MINRES for the all-at-once wave equation.

The solver lives in the HIP library ``libabac.so`` (C ABI in ``include/abac.h``);
``paper_2306_03574_amd.abac`` is its Python binding.
"""
from .abac import Plan, Group, AbacError, load_library, workspace_bytes, EXPORTED  # noqa: F401
