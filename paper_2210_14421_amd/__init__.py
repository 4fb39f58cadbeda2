"""MI355X (gfx950) library for the second-order Magnus step of all-electron
real-time TDDFT in an enriched finite-element basis (arXiv:2210.14421).

The HIP kernels and the C ABI live in ``csrc/`` and build into ``libefe.so``
(``python -m paper_2210_14421_amd.build``); ``paper_2210_14421_amd.efe`` is the
ctypes binding.  Importing this package loads nothing.
"""
