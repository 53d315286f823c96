"""MI355X (gfx950) semi-analytical particle tracker: HIP kernels behind a C ABI.

``pt`` is the Python binding of libpt.so (include/pt.h).  Build the library
with ``python -m paper_2302_13590_amd.build``.
"""
