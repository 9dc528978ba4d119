"""CPU oracle for the exact integer determinant and its modular pieces.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library.

Everything here is plain and slow on purpose: Python integers (exact), numpy
int64 where the bounds are checked, no blocking, no fusion.  Each function
names the passage of Dumas and Urbanska, "An introspective algorithm for the
integer determinant", that it follows, or the textbook definition it writes
out when the method reaches that definition exactly.

  det_bareiss          O1  det(A) by fraction-free (Bareiss) elimination
  det_bareiss_c        O1  the same definition in plain C (oracle/bareiss.c)
  det_mod_p            O2  det(A) mod p by Gaussian elimination over Z_p
  inverse_mod_p        --  A^{-1} mod p by Gauss-Jordan over Z_p
  dixon_digits         O3  p-adic digits of A^{-1} b (Section 2.2)
  solve_rational       O4  exact x = A^{-1} b over Q, its common denominator
  extended_bonus       O4  pi~ = s~^i / gcd(det(R N), s~^i) (Section 3.2)
  crt_symmetric        O5  Chinese remaindering into the symmetric range
  et_cra               O5  early-terminated CRA (Alg. 2.1, Lemma 2.1)
  rational_reconstruct O6  rational number reconstruction (extended Euclid)
  hadamard_bits        O7  exact Hadamard bound bits (Lemma 2.1)
"""
from .det_oracle import (  # noqa: F401
    det_bareiss,
    det_mod_p,
    inverse_mod_p,
    dixon_digits,
    dixon_length,
    solve_rational,
    extended_bonus,
    largest_invariant_factor,
    crt_symmetric,
    et_cra,
    et_k,
    rational_reconstruct,
    hadamard_bits,
    hadamard_sq,
    is_prime,
    det_introspective_oracle,
)
from .bareiss_c import det_bareiss_c, build_bareiss_c  # noqa: F401
