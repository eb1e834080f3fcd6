"""MI355X-native EOFA / optimal domain-wall solver.

Importing the package loads nothing native; ``paper_1710_09621_amd.eofa`` binds the
HIP library and ``paper_1710_09621_amd.inputs`` holds the seeded input generators.
"""
__all__ = ["inputs", "eofa"]
