"""STEV stiff-chemistry integrator for AMD Instinct MI355X (gfx950).

``stev``   ctypes binding of the HIP library libstev.so (the compute path)
``synth``  seeded synthetic mechanisms and cell fields (inputs only)
``build``  in-tree hipcc build of libstev.so
"""

__all__ = ["stev", "synth", "build"]
