"""GlassNet per-pixel evaluation on MI355X (gfx950).

The compute path lives in a C-ABI shared library of hand-written HIP kernels
(`libglassnet.so`, built in-tree); `paper_2405_19056_amd.glassnet` is a thin
ctypes binding over it.  Importing this package loads nothing.
"""
