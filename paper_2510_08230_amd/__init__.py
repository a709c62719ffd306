"""MI355X-native sparse Krylov hot path: CSR SpMV and CG on gfx950.

The product is ``libspk.so`` (HIP kernels + the C ABI of include/spk.h);
``paper_2510_08230_amd.spk`` is its thin Python binding.
"""
