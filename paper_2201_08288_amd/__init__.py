"""MI355X-native level-by-level k-d tree build (HIP kernels behind a C ABI).

Importing the package loads nothing; ``paper_2201_08288_amd.kdtree`` loads the
HIP library ``libkdtree.so`` and fails loudly when it is missing.
"""
