"""MI355X-native ray caster for float32 spectral cubes (RA x Dec x frequency).

Importing the package loads nothing native; `paper_1012_2909_amd.vr` binds the
HIP library and fails loudly when it is missing.
"""
__all__ = ["synth", "vr"]
