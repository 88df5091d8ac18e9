"""H2-compressed Fredkin-Koehler boundary double-layer operator on MI355X (gfx950).

``paper_1811_05731_amd.h2dlp`` is the binding of the C ABI in include/h2dlp.h
(libh2dlp.so, HIP kernels); ``paper_1811_05731_amd.serving`` batches matvec
requests over resident operators.  Importing this package loads nothing; the
binding module fails loudly when the library has not been built.
"""
