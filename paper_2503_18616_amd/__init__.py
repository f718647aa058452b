"""MI355X-native batched XPBD substep (FF-SRL, arXiv 2503.18616).

Submodules:
  workloads  seeded synthetic inputs (slab meshes, tool paths, compliances)
  xpbd       ctypes binding of the HIP C-ABI library (libxpbd.so)

Importing the package loads nothing; ``paper_2503_18616_amd.xpbd`` loads the
native library on first use and raises if it is missing.
"""
