"""Graphical Join hot path for AMD MI355X (gfx950).

Submodules:
  workloads -- seeded synthetic inputs (shared with the tests)
  gj        -- thin ctypes binding over the C-ABI library ``libgj.so``
"""
__all__ = ["workloads", "gj"]
