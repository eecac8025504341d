"""MI355X (gfx950) Contact-Field hot path of Lightning Grasp (arXiv 2511.07418).

The product is ``liblg.so`` (HIP kernels behind the C ABI of
``include/lg.h``); :mod:`paper_2511_07418_amd.lg` is its thin ctypes binding
and :mod:`paper_2511_07418_amd.pipeline` chains the four calls.  Build the
library with :func:`paper_2511_07418_amd.build.build`.
"""

__all__ = ["lg", "pipeline", "build"]
