"""Plain FP64 CPU oracle for the TLR Cholesky / LDL^T hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package.  The
product (the HIP library and its Python binding) never imports, links or
calls it, and shares no code with it.

Contents (each function cites the passage of the paper it follows):

* ``dense``        -- covariance assembly, dense Cholesky (LAPACK through
                      numpy), dense unpivoted scalar LDL^T, triangular solves.
* ``tlr``          -- the TLR format (Section 1), compression of tiles by
                      truncated SVD, the left-looking TLR Cholesky and LDL^T
                      (Algorithms "Left Looking TLR Cholesky" and "Left
                      Looking TLR LDL^T", Eq. (1)-(3)) with the ARA step
                      replaced by exact SVD truncation of the assembled
                      Schur-complement tile, the TLR triangular solve
                      (Algorithm "TLR Triangular Solve"), the TLR matvec and
                      the SVD post-recompression of the low rank tiles
                      (Section 6.2).
* ``bookkeeping``  -- integer bookkeeping of the method: tile offsets, row
                      panel widths, the rank sort of "sortRanks" and the
                      active-set evolution of "updateSubset".
* ``philox``       -- Philox4x32-10 (Salmon et al., SC'11) and Box-Muller,
                      written from their published definitions, used only to
                      check the device generator bit for bit.
"""
