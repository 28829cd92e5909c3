"""MI355X-native two-vector Four-Russians Nussinov folding.

The GPU path lives in ``libnf.so`` (built from ``csrc/``) behind the C ABI of
``include/nf.h``; ``paper_1307_7820_amd.nf`` is the thin Python binding.
Importing this package does not load the library; ``gen`` (seeded inputs) is
usable without a GPU.
"""

__all__ = ["gen", "nf"]
