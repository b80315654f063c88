"""MI355X-native dense Lindblad propagation (arXiv 2603.18052 hot path).

``paper_2603_18052_amd.lindblad`` binds the HIP library ``liblindblad.so``
(C-ABI declared in ``include/lindblad.h``); ``workloads`` builds the seeded
synthetic inputs.  Importing the package loads nothing: the binding loads
the library on first use and raises if it is missing.
"""
