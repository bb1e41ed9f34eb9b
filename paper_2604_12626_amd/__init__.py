"""MI355X-native tile-based 3D Gaussian Splatting sensor renderer (Habitat-GS hot path).

The compute path is the HIP library ``libgs.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/gs.h``.  ``binding`` marshals torch tensors to
that ABI; ``render`` adds the autograd function and the batched renderer.
Importing this package loads nothing; the first call into the binding loads
the library and raises if it is missing.
"""
__all__ = ["synth", "binding", "render"]
