"""MI355X-native Vertex Block Descent (VBD) hot path.

The solver lives in a HIP/C++ shared library with a C ABI (include/vbd.h);
this package is its thin Python binding.  ``workloads`` holds the seeded
synthetic input generators.
"""
