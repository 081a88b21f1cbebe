"""MI355X-native homomorphic SZp: error-bounded compression, multi-stage
decompression and analytical operations on the intermediate stages, all as
hand-written HIP kernels behind a C ABI (libhsz.so).

The binding lives in ``paper_2603_25206_amd.hsz``; importing this package
alone loads nothing (so the seeded input generators in ``synth`` can be used
without a GPU).
"""
__all__ = ["hsz", "synth"]
