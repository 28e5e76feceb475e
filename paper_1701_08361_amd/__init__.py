"""MI355X-native NLINV hot path: HIP kernels behind a C-ABI (libnlinv.so) and a
thin ctypes binding.  Importing the package does not load the library; use
`paper_1701_08361_amd.nlinv` for the binding."""
