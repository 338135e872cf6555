"""MI355X (gfx950) hot path of quasi-dynamic traffic assignment.

The compute path is the HIP library libqdta.so (C ABI in include/qdta.h);
`qdta` is its ctypes binding.  Importing the package loads nothing.
"""
__all__ = ["qdta", "build"]
