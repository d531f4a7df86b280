"""FP64 CPU oracle for the PSTD scattering method (test infrastructure only).

This package is the checker of the HIP path, not part of the product: only the
test suite, the smoke entry point and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library.  Every function is a plain,
slow transcription of the paper's definitions in double precision, citing the
section and equation it follows.

Modules
  fft            naive DFT, radix-2 and Bluestein FFTs (library-free)
  pstd           reduced units, stability bound, tables, the PSTD step and the
                 running surface DFT (Sections 2.1-2.5, 3.3)
  ntdf           near-to-distant-field projection over a virtual box
                 (Sections 3.1-3.2)
  partial_waves  phase shifts of the central square potential (Section 4)
"""
