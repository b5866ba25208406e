"""mfgp: matrix-free Gaussian-process inference on AMD MI355X (gfx950).

The compute path is a C-ABI HIP library (``libmfgp.so``, declared in
``include/mfgp.h``).  ``paper_2605_17898_amd.mfgp`` is its thin Python binding;
importing this package does not load the library, so host-only tools (the
input generators) work without a GPU.
"""
