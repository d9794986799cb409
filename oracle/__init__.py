"""CPU oracle for the approximate-DCT transform-coding method (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct restatement of what the paper
computes, in float64 and exact integers.  It exists only to check the GPU
library: only the test-suite, the smoke entry point and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the HIP library and never
imports it; the only module both sides use is `synth`, which draws input pixels
and does none of the method's arithmetic.

Modules
  matrices  exact DCT, the printed integer matrices, the orthogonalising scale
  codec     blockwise 2-D transform coding: forward, zig-zag, quantiser, inverse, PSNR
  sfg       the paper's fast algorithm (factorisation of T1) and its operation count
  search    the greedy angle-similarity search (closure and canonical forms, top-k scan)
  measures  error energy, MSE, coding gain, transform efficiency, circular statistics
  batch     SSE table over images x transforms x retention levels
  postfilter  float64 conv network forward/backward on bfloat16-rounded operands
  ssim      structural similarity of a reconstruction (Gaussian-window local statistics)
  jam       16- and 32-point matrices by the JAM construction; N x N transform coding
  nonortho  inverse decoder for non-orthogonal matrices (SDCT, BAS-2008b); coding gain vs correlation

Every function cites the passage of the paper it restates.  Readings taken where
the paper is silent or ambiguous are stated where they are used.
"""
