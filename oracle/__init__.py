"""FP64 CPU oracle for the kernel aggregated FMM -- TEST INFRASTRUCTURE.

Plain, slow, obviously correct implementations of what the evaluation pass
computes, written from the paper (Yan & Blackwell, Kernel Aggregated Fast
Multipole Method).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import anything here.  Nothing in the HIP
library imports, links or calls this package, and this package imports
nothing from the library.

Modules:
  direct   FP64 O(N_S N_T) direct sums of every kernel (C, OpenMP).
  ewald    FP64 Ewald sums for triply periodic Laplace charges + dipoles.
  kifmm    plain FP64 KIFMM with the paper's own kernel tables (NumPy).
  mlp      FP64 MLP forward/backward/Adam reference for the order predictor.
"""
