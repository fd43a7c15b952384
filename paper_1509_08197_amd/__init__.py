"""MI355X-native hot path of hierarchical-disparity-prediction (HDP) stereo.

The compute path lives in ``libhdp.so`` (hand-written HIP kernels for gfx950
behind a C ABI, declared in ``include/hdp.h``).  ``paper_1509_08197_amd.hdp``
is the thin Python binding; ``scenes`` draws seeded synthetic inputs.
"""
