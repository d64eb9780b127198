"""CPU oracle for the butterfly-compressed multifrontal solver (TEST INFRASTRUCTURE).

A plain, slow, obviously correct FP64 implementation of what the GPU path
computes, written from the paper (Liu, Ghysels, Claus, Li, "Sparse
Approximate Multifrontal Factorization with Butterfly Compression for High
Frequency Wave Equations"):

  nd.py           geometric nested dissection, separator bisection (Sec. 5.1)
  symbolic.py     assembly tree, index sets I^s / I^u, extend-add maps (Sec. 2)
  multifrontal.py uncompressed multifrontal LU and solve (Alg. 1)
  gmres.py        restarted GMRES(30) with MGS, left preconditioning (Sec. 6)
  butterfly.py    interpolative decomposition, butterfly construction by
                  entry evaluation, extraction and application (Sec. 3)

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP path:
inputs come from the separate ``workloads`` generators.
"""
