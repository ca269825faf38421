"""CPU oracle for the encrypted CCMM of 1:N iris matching (test infrastructure).

A slow, plain, obviously correct CPU implementation of what the GPU path
computes: CKKS-style secret-key encryption in the MSRLWE ("shared-a") format,
the RGSW-style encrypted matrix product (CCMM) of Section 2.3, the rescale of
Section 2.2.4, decryption and coefficient decoding, and the plaintext masked
Hamming truth of Section 2.1.

This package is test infrastructure.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code with the HIP library (it is written independently,
from the paper and from published definitions).

Modules:
  params  -- NTT-friendly primes, scaling factor, ring sizes
  prng    -- Philox4x64-10 and the samplers (uniform mod q, ternary, CDT Gaussian)
  ring    -- negacyclic products (schoolbook) and exact integer matrix products
  ckks    -- keygen, database / query encryption, CCMM, rescale, decryption
  iris    -- masked ternary encoding, shifts, popcount truth and decisions
  smallmod -- the int8 digit planes of the small-modulus (p^2) product of Section 6.3
  chain   -- the CCMM over the modulus chain of products n^2 (Section 6.3)
  bigmul  -- exact negacyclic products at ring degrees up to 2^16
  formatswitch -- the query's ring switch 2^16 -> N_Q, MSRLWE conversion and
             modulus switch (Appendix C.1)
"""
