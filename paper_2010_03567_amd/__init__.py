"""MI355X (gfx950) gravity hot path of arXiv:2010.03567: octree over
Morton-sorted integer coordinates, multipoles to octupole, one-sided walk with
the relative opening criterion, TreePM short-range kernel, symmetric FMM.

The compute lives in ``libg4hip.so`` (HIP kernels behind the C ABI of
``include/g4hip.h``); ``paper_2010_03567_amd.g4hip`` is its ctypes binding.
Importing the binding fails loudly when the library has not been built.
"""
__all__ = ["g4hip"]
