"""MI355X (gfx950) statevector emulator of Quantum Phase Estimation.

The compute path is libqpe.so (hand-written HIP kernels behind a C ABI, see
include/qpe.h); ``paper_2507_17175_amd.qpe`` is its ctypes binding.
"""
__version__ = "0.1.0"

__all__ = ["qpe"]
