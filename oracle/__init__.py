"""CPU FP64 oracle for the sketched Krylov f(A)b path -- TEST INFRASTRUCTURE.

This package is the slow, plain reference that the HIP path is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run it; the product
library never does, and it shares no code, tables or helpers with the HIP
sources (only the seeded input descriptions in ``workloads`` serve both).

Contents (each function cites the passage of Cortinovis, Kressner &
Nakatsukasa, "Speeding up Krylov subspace methods for computing f(A)b via
randomization", that it follows):

* ``rng``       SplitMix64 counter streams (published generator definition).
* ``sketch``    SRHT and sparse-sign embeddings Theta (Section 2.1.1).
* ``operators`` the synthetic operators as scipy CSR matrices.
* ``matfun``    f(K) e1 for small dense K: exp, (K + sigma I)^(+-1/2), polynomials.
* ``krylov``    Arnoldi (eq. (2)), the standard approximation f_m (eq. (4)),
                truncated orthogonalisation (Algorithm 2), the sketched
                compression and Algorithms 4/5, sFOM (eq. (9)).
* ``closed_form`` exact f(A)b for Dirichlet Laplacians (separable DST-I) and
                dense brute force, used only to pin the oracle itself.

Pins (tests/test_oracle_*.py, run with ``-m "not gpu"``): dense brute force
by eigendecomposition, diagonal closed forms, DST closed form at full size,
exactness at the minimal-polynomial degree, polynomial exactness
(Theorem 6 consequence), the Arnoldi relation and orthonormality, basis
invariance (Lemma 2), sFOM == sketch-and-solve (Remark 3), Lanczos
equivalence for symmetric A with k = 2 (Section 2.1.2), dense Sylvester
Hadamard and published SplitMix64 outputs for the sketches.
"""
