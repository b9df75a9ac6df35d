"""MI355X-native two-body macro-ion particle-in-cell hot path.

The compute path lives in the HIP library libpic.so (C ABI declared in
include/pic.h); `paper_2208_08038_amd.pic` is its thin ctypes binding.
`paper_2208_08038_amd.inputs` describes the seeded synthetic workloads.
Importing the package loads nothing native; the binding loads the library
on first use and raises if it is missing.
"""
