"""MI355X-native (gfx950) state-vector and density-matrix simulation engine.

The numerical work runs in hand-written HIP kernels behind the C ABI of
include/nwq.h (libnwq.so, built by `python -m paper_2401_06861_amd.build`);
`paper_2401_06861_amd.nwq` is its ctypes binding.  PyTorch provides device
memory and streams only.
"""
__all__ = ["nwq"]
