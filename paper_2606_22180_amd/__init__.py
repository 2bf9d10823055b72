"""FeLoG's single-GPU hot path on MI355X: random walks, skip-gram with negative
sampling and the FeeST feedback step, as HIP kernels behind a C ABI
(include/felog.h).  ``felog`` is the ctypes binding; ``build`` compiles the
library with hipcc for gfx950."""
