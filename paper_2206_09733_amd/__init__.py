"""MI355X-native DGSEM residual and low-storage RK3 (HORSES3D, arXiv 2206.09733).

The HIP library is loaded on first use of `paper_2206_09733_amd.dgsem`; importing the package
itself touches neither the GPU nor the shared library.
"""
__all__ = ["dgsem", "synth"]
