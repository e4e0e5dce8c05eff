"""MI355X-native online Itakura-Saito NMF (arXiv:1106.4198).

The compute path is the HIP library built from ``csrc/`` (C ABI declared in
``include/isnmf.h``); ``binding`` wraps it with ctypes.  ``synth`` draws the
seeded synthetic spectrograms.  Import ``paper_1106_4198_amd.binding`` to use
the GPU path; it raises if the compiled library is missing.
"""
__all__ = ["binding", "synth", "build"]
