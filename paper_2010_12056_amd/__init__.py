"""CP-ALS hot path (dimension-tree MTTKRP, multi-sweep dimension tree and
pairwise perturbation) on MI355X.  The compute lives in the HIP library
`libcpals.so`; `paper_2010_12056_amd.cpals` is its ctypes binding.  Importing
this package loads nothing; the library is loaded on first use of the binding.
"""
