"""MI355X-native spacetime finite-element Dirac solver (arXiv:2103.14588).

Importing the package loads nothing native.  ``paper_2103_14588_amd.dirac_st``
binds the C-ABI library ``libdirac_st.so`` built from ``csrc/``; it raises if
the library is missing.  ``paper_2103_14588_amd.inputs`` holds the seeded
synthetic workloads.
"""
__all__ = ["inputs", "dirac_st"]
