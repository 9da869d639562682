"""CPU reference ("oracle") for the semi-implicit anisotropic diffusion scheme.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
GPU library never loads it and shares no code with it.

Contents
  asd_oracle.c  plain C99, serial, FP64 implementation of the scheme
                (section 2 of Sharma & Hammett, arXiv:1008.0861)
  oracle.py     ctypes loader for the compiled C file
  torch_ref.py  FP64 torch-CPU re-statement of the same step, differentiated
                by autograd: the reverse-mode reference for the adjoint
  build.py      compiles asd_oracle.c with gcc (-O2 -ffp-contract=off)

Parity status (pins live in tests/test_oracle_*.py):
  limiters, Thomas / cyclic solves, sweeps, 2-D / 3-D steps, explicit step:
  pinned (closed forms, invariants, textbook reductions, brute force).
  torch_ref: pinned to the C oracle's forward and to central differences.
"""
