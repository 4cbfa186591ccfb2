"""MI355X-native quasi-static plasma response (WAKE, arXiv:1411.3246).

The compute path lives in the HIP library built from ``csrc/``; the
``wake`` module binds its C ABI.  Import ``paper_1411_3246_amd.wake`` for the
library and ``paper_1411_3246_amd.inputs`` for seeded synthetic inputs.
"""
