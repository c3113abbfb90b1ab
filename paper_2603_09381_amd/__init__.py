"""MI355X-native proxy fast direct solver for 2-D multi-inclusion Helmholtz transmission.

The compute path is the C-ABI library ``libpmx.so`` (hand-written gfx950 HIP
kernels); ``paper_2603_09381_amd.pmx`` is its thin ctypes binding.  Importing this
package loads nothing; ``workloads`` holds the seeded input generators.
"""
