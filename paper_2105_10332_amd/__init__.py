"""MI355X-native two-dimensional swept-rule stencil solver (arXiv:2105.10332).

The solver itself is the HIP library ``libswept.so`` (C ABI in
include/swept.h); :mod:`.solver` binds it with PyTorch device memory.
Submodules load lazily so that the seeded input generators
(:mod:`.problems`) import without the GPU library.
"""
__all__ = ["problems", "solver", "build"]
