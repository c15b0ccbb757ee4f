"""ASE-DF reconstruction, Lax-Friedrichs flux and SSP-RK3 update on MI355X.

Submodules:
  ase        -- Python binding of the C ABI in include/ase.h (libase.so)
  workloads  -- seeded synthetic problem generators (grids, exact averages)
  build      -- in-tree hipcc build of libase.so
"""
__all__ = ["ase", "workloads", "build"]
