"""FP64 CPU oracle of the PNA-style GCNN hot path.

Test infrastructure only: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with
the HIP library.
"""
from .pna import (CSR, Decisions, DecisionMismatch, ForwardRecord, STD_EPS, adamw,
                  backward, check_batch, csr_build, degree_scalers, forward,
                  layer_forward, pack, unpack)
