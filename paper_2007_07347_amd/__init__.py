"""MI355X (gfx950) implementation of the simplified discrete unified gas
kinetic scheme (sDUGKS, arXiv:2007.07347) for D2Q9 BGK flow on 2-D meshes.

The solver itself is libsdugks.so (C ABI in include/sdugks.h); `sdugks` is its
Python binding.
"""
