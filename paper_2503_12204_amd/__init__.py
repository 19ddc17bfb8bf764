"""MI355X (gfx950) hot path of D4orm: Monte Carlo score denoising of
multi-robot control deformations.

Submodules:
  workloads - problem records and seeded synthetic instances
  build     - compiles libd4.so with hipcc for gfx950
  _lib      - ctypes binding of libd4.so (imported on demand; raises if the
              library is missing)
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
