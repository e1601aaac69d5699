"""MI355X-native D3Q19 MRT-Smagorinsky LES hot path (HIP kernels behind a C-ABI).

Submodules
----------
``lbm``      thin ctypes binding of ``liblbm.so`` (names follow the C-ABI in
             ``include/lbm.h``); torch supplies device memory and streams.
``inputs``   seeded synthetic inputs (forcing-mode tables, request streams).
``params``   lattice parameters from physical ones (tau0 from Re, F0 from C_f).
``serving``  continuous-batching request loop over ``lbm_batch_step``.
``build``    compiles ``liblbm.so`` for gfx950 with hipcc.

Importing the package loads nothing; the first use of ``lbm`` loads the HIP
library and raises if it has not been built.
"""
