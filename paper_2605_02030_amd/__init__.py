"""U-HNSW query path on AMD Instinct MI355X (gfx950).

The product is the C-ABI library ``libuhnsw.so`` (header ``include/uhnsw.h``);
``paper_2605_02030_amd.uhnsw`` is its ctypes binding. Build with
``python -m paper_2605_02030_amd.build``.
"""
