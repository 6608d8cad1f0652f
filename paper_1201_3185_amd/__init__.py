"""MI355X (gfx950) particle-mesh QUMOND solver after Angus et al., arXiv:1201.3185.

``paper_1201_3185_amd.qumond`` is the ctypes binding of the HIP library
(libqumond.so, built by ``paper_1201_3185_amd.build``); ``synth`` holds the
seeded synthetic disk generators.
"""
__all__ = ["qumond", "synth", "build"]
