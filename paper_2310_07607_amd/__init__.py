"""MI355X-native explicit SIPG-DG monodomain stepping under synchronous local
time stepping (arXiv:2310.07607).  The compute path is the HIP library
``libmdlts.so``; :mod:`paper_2310_07607_amd.mdlts` is its ctypes binding."""
