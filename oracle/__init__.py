"""Slow, plain FP64 CPU oracle for MPO-times-MPS apply + variational compression.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls this package; only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the GPU path: the two meet only at the seeded inputs of `synth`.

Every function follows the paper's definitions (citations are to its sections
and equations) and uses NumPy / SciPy library primitives (einsum, QR, SVD) as
single steps, with no blocking or fusion beyond what the definitions state.

Modules:
  dense     -- MPS / MPO <-> dense vectors and matrices (Eq. general-MPS, Eq. MPO,
               Eq. binary).
  mps       -- scalar product, canonical form, truncation rule, exact MPO x MPS
               product, the two-site variational sweep (two independent routes),
               TT-SVD, error bookkeeping.
  mlp       -- the rank-predicting multilayer perceptron (forward, backward, Adam)
               in FP64, for gradient checks.
  rsvd      -- randomized range finder + small SVD (Halko, Martinsson, Tropp 2011).
"""
