"""MI355X (gfx950) hot path of quadratic B-spline cloth finite elements (arXiv 2506.18867).

The computation lives in ``libbsc.so`` (HIP kernels behind the C ABI of ``include/bsc.h``);
``paper_2506_18867_amd.bsc`` is its ctypes binding. Build with
``python -m paper_2506_18867_amd.build``."""
