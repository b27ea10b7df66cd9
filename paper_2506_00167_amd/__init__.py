"""MI355X-native builder of the Cyrus+ O-DU puncturing codebook.

Submodules:
  workload  seeded synthetic inputs (no method arithmetic)
  cyrus     ctypes binding of libcyrus.so (HIP kernels behind a C ABI)
  build     compiles libcyrus.so for gfx950

Importing the package does not load the HIP library; ``cyrus.lib()`` does.
"""
