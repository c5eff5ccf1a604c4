"""MI355X-native eMAGPIE: HIP kernels behind the libemagpie C ABI.

Importing this package loads nothing native; `paper_2511_01793_amd.emagpie`
loads the built library and fails loudly if it is missing.
"""
__all__ = ["synth"]
