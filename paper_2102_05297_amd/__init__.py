"""Counter-guided autotuning search sweep on AMD Instinct MI355X (gfx950).

The product is the HIP library ``libcgs.so`` (C ABI in ``include/cgs.h``)
and its thin ctypes binding :mod:`paper_2102_05297_amd.cgs`.  Build the
library with ``python -m paper_2102_05297_amd.build``.
"""
