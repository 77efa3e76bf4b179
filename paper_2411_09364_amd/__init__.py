"""MI355X-native LES substep library (HIP kernels behind a C ABI; see include/les.h).

Import the binding with `from paper_2411_09364_amd import les`; it loads the in-tree
liblesmi.so and raises ImportError when the library has not been built.
"""
