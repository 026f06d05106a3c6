"""MI355X (gfx950) H^2-ULV dense solver: a C-ABI HIP library (include/h2.h,
csrc/) and its Python binding (h2.py).  Build with
``python -m paper_2502_02395_amd.build_lib``."""
