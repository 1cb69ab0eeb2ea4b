"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU model of what the tiled QR path of the
thesis (Bouwmeester 2012, chapter "QR Factorization") computes:

* ``oracle.householder``: unblocked FP64 Householder QR, Q^T b, least squares
  and the backward-error measures (numpy, written from the textbook
  definition; the thesis states that the tiled algorithm produces exactly
  the R factor of the QR factorization and performs the same flops as the
  standard Householder algorithm).
* ``oracle.trees``: elimination lists, coarse-grain and tiled critical paths
  (plain C in ``tiledqr_lists.c``, loaded through ctypes).
* ``oracle.mlp``: the selector network's forward/backward pass in FP64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  It shares no code with
the product library (``paper_1303_3182_amd``) and imports nothing from it.
"""
