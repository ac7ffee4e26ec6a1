"""MI355X collective multigrid for PDE-constrained optimization under uncertainty.

Package layout:
  csrc/        HIP kernels (gfx950) and the C ABI of include/smg.h
  build.py     in-tree hipcc build of libsmg.so
  binding.py   ctypes binding (argument marshalling only)
  inputs.py    seeded synthetic problem instances

Importing the package loads nothing; ``binding.load()`` loads the library.
"""
