"""MI355X-native full-neighbourhood move evaluation for VRP local search.

The device library (HIP kernels for gfx950 behind a C ABI, ``include/tga.h``)
is loaded by :mod:`paper_2506_17357_amd.tga`; seeded inputs come from
:mod:`paper_2506_17357_amd.workload`.  This file imports neither, so that
importing the input generators never loads the device library.
"""
