"""MI355X-native masked 4D Gaussian rasterizer (4DGS-1K hot path).

Importing the package loads nothing; `paper_2503_16422_amd.render` loads the
HIP library libfdgs.so on first use and raises if it has not been built.
"""
__all__ = ["inputs", "render"]
