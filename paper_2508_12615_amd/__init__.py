"""MI355X-native wavelet rasterizer (WIPES, arXiv 2508.12615): forward and backward.

The compute path is the HIP library ``libwipes.so`` (hand-written gfx950
kernels behind a C ABI declared in ``include/wipes.h``).  Importing this
package does not load the library; ``paper_2508_12615_amd.binding`` does, and
fails loudly if it has not been built.
"""
__all__ = ["binding", "raster", "synth"]
