"""FP64 CPU oracle for the fast damped Gauss-Newton (fLM) step for CP.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links it, and it
shares no code with that path: only the seeded input generators in `cpgen`
serve both.

Modules
-------
cp     -- the method as the paper states it: MTTKRP, Gram/Hadamard products,
          the fast update of Theorem 4.1 (fLMa and fLMb of Section 4.3), the
          complex variant of Section 5, the damping loop of Section 4.5.
brute  -- the plain damped Gauss-Newton step a <- a + (J^T J + mu I)^-1 J^T e
          of Section 3 with the Jacobian of Appendix B formed explicitly; the
          definition that pins the fast step on tiny tensors.

Pins (see tests/test_oracle_pins.py): every function here is checked against
something other than itself -- the explicit-Jacobian solve, the closed-form
inverse of K (Appendix E), the zero gradient at an exact rank-R tensor, exact
recovery of noiseless data, the cross-mode MTTKRP invariant, the Euler
identity J a = N vec(Y_hat), the decrease of the linearised residual
(the gain-ratio denominator), tau max diag(J^T J) (mu0), the model-preserving
normalisations, the closed form of each damping rule over a run of rejected
trials, and the generator's closed forms.  The damping
loop's trajectory (fit) has no printed worked example in the paper: parity
unpinned beyond those step-level pins and the recovery test.
"""
