"""MI355X-native jump flooding (JFA) and dynamic jump flooding (dJFA).

Hot path of "GPU Voronoi Diagrams for Random Moving Seeds": flood passes,
seed moves and seed splats run as hand-written HIP kernels for gfx950 behind
the C ABI declared in ``include/vdflood.h`` (``libvdflood.so``).  The Python
binding in :mod:`paper_2209_00117_amd.vdflood` only marshals arguments; it
loads the library on first use and raises if it is missing.
"""
__all__ = ["inputs", "vdflood"]
