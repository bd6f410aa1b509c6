"""Independent FP64 CPU oracle for the SIPDG monodomain PCG / agglomerated
multigrid method (arXiv 2602.16312).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, headers,
tables or helpers with the HIP library; the two meet only through the seeded
input arrays produced by ``workloads``.

Data structures are deliberately different from the GPU path: global scalar
CSR matrices (scipy.sparse) assembled entry by entry from the bilinear forms,
sparse triple products for the coarse operators, dense Cholesky for the
coarsest level.  All arithmetic is float64.

Parity status per function is stated in each module header; the functions
with no external pin are listed there as "parity unpinned".
"""
