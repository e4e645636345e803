"""FS-FEM (face-based smoothed FEM, T4) stiffness assembly and PCG solve for
MI355X (gfx950).  Every numerical step runs in the HIP kernels of
``csrc/`` behind the C ABI declared in ``include/sfem.h``; the Python side in
``sfem.py`` only marshals arguments.  ``meshgen`` generates seeded inputs.

Importing the package does not load the native library; ``sfem.lib()`` does,
and raises if it has not been built.
"""
__all__ = ["meshgen", "sfem"]
