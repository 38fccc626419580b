"""MI355X (gfx950) solver for the first-order upwind Eikonal system, scheduled by cells.

``eik``       -- Python binding of the C ABI in include/eik.h (libeik.so, HIP kernels).
``workloads`` -- seeded synthetic problems (speed fields and exit nodes).
``build``     -- in-tree hipcc build of libeik.so.

Importing the package loads nothing native; ``eik.load()`` does, and raises when the library is
missing (there is no CPU fallback).
"""
__all__ = ["eik", "workloads", "build"]
