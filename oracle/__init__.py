"""FP64 CPU oracle for the batched Bartlett grid search and its learned proposal.

Test infrastructure only. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package; the
product path never does. The oracle shares no code with the HIP library: it
reads the paper's definitions and nothing else.

Modules:
  bartlett  steering vectors, sample covariance, Bartlett spectrum, peak
            picking, parabolic refinement and the proposal moments.
  mlp       the proposal network: forward, MSE loss, backward and Adam.
"""
