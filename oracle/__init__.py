"""FP64 CPU oracle of the dipolar GPE split step.  Test infrastructure only:
imported by the test suite, the package smoke check and the benchmark's CPU
baseline, never by the GPU library."""
from .dgpe_oracle import *  # noqa: F401,F403
