"""MI355X-native VaFR hot path: log-polar (LP) shading by ray casting and the
inverse map to the display, as hand-written HIP kernels behind a C ABI.

Submodules are imported on demand so that ``inputs`` (seeded synthetic
workloads) can be used without loading the native library.
"""
