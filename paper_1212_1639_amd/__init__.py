"""MI355X-native fully parallel particle filter / particle learning.

The compute path is the C-ABI library ``libpf_mi355x.so`` (hand-written HIP
for gfx950, declared in ``include/pf.h``); ``paper_1212_1639_amd.pf`` is its
thin ctypes binding.  Importing this package does not load the library, so
the seeded input generators in ``paper_1212_1639_amd.inputs`` can be used on
machines without a GPU.
"""
