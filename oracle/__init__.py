"""CPU oracle for the encrypted CSR matrix-factorisation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or executes this package; only the test suite,
the smoke check and the CPU-baseline leg of the benchmark use it.

It is a plain, slow and deliberately unoptimised restatement of what the path
computes:

* ``params``    prime chains and roots for RNS-CKKS (textbook CKKS, Cheon-Kim-Kim-Song
                2017, the scheme the paper adopts in Sec. II-A.2 and Sec. IV-A).
* ``chacha``    the ChaCha20 block function of RFC 8439 (seeded randomness).
* ``sampling``  integer-only samplers (uniform residues, ternary, centred binomial).
* ``modarith``  exact modular multiplication on numpy uint64 arrays.
* ``ring``      negacyclic polynomial arithmetic in Z_q[X]/(X^N+1).
* ``rns``       CRT, fast basis conversion, rescale, ModDown.
* ``ckks``      keys, encryption, encoding, homomorphic add/mul (Eq. 6-9 of the
                paper), key switching, rotations, rescale.
* ``mf``        FP64 CSR matrix factorisation (Eq. 1-5, Alg. 1, Alg. 2).
* ``program``   the encrypted MF epoch over block-packed CSR rating ciphertexts
                (Alg. 1 evaluated as a synchronous epoch with the Alg. 2 accumulator).

Every floating-point quantity is float64; every residue is an exact integer.
"""
