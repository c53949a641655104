"""MI355X (gfx950) implementation of the exhaustive mutual-information
epistasis scan of Fiuncho (arXiv 2201.03331), behind the C ABI of
include/fiuncho.h.  ``fiuncho`` is the ctypes binding, ``synth`` the seeded
input generator, ``build`` the in-tree hipcc build."""
