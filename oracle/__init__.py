"""CPU oracle for the encrypted linear-layer product (TEST INFRASTRUCTURE ONLY).

A plain, slow, independent reference of what the model owner's homomorphic
linear-layer product computes: RNS-BFV key generation, encryption and
decryption (Sec. II.B, Sec. V), the batched polynomial encodings of App. A,
the forward product of Alg. 1 and the backward products (the gradient with
respect to the input by the Alg. 1 pattern, Sec. III.B.2; the weight-gradient
cross terms of Alg. 2), plus re-randomisation, noise flooding and masking of
every output ciphertext.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import,
call or link anything in this package.  It shares no code with the GPU path
and never imports it.  Heavy O(N^2) ring products run in a small plain-C
schoolbook helper (cref.c); everything else is Python integers and numpy.

Readings of points the paper leaves open (the primes, the NTT root, the
randomness, the flooding width, the backward encodings) are stated in the
module that implements each one.
"""
