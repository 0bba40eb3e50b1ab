"""CPU oracle for the homomorphic convolution of Flash (arXiv 2401.16732).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the GPU library
(no kernels, headers, helpers, tables or constant generators).

It is deliberately plain and slow: every function states the passage of the
paper it follows, works in exact integers (Python ints or int64 numpy with
explicit reductions), and uses no NTT (batch encoding is interpolation at the
slot points, written out). The paper's convolution (Algorithm 1)
is a ring computation, so its result is unique given the ciphertext layout;
the oracle computes that result directly from the definitions.

Modules:
  params  - RNS prime search, Delta = floor(q/t), centred lifts (Notation table)
  ring    - schoolbook negacyclic product and DRot (eq. drot, Appendix A proof)
  bfv     - toy secret-key BFV encrypt / decrypt / noise (Table 2, eq. bfv_dec, Alg. 2)
  layout  - direct encoding (eq. de) of zero-padded, channel-packed inputs
  conv    - Algorithm 1, the weight polynomial, plain conv mod t, mask + extract,
            Freivalds combination
  calg1   - the same Algorithm 1 in plain C (int64 lazy accumulation)
  batch   - batch (slot) encoding by interpolation, PMult, and the server steps
            of the x^2 + x protocol

Parity pins: every function is checked by the `-m "not gpu"` tests against
closed forms, brute force or library routines (see tests/test_oracle_*.py).
"""
