"""MI355X-native hot path of the Eulerian diffuse-interface fracture method
of arXiv 2210.04037: a C-ABI library (libfv.so, HIP kernels for gfx950) and a
thin Python binding.  PyTorch only supplies device memory and streams."""

__all__ = ["abi", "solver"]
