"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and
the benchmark. Random numbers and layout only: no part of the method."""
from .gen import (WORKLOADS, KD_COLS, VD_COLS, N_FEATURES, ALLOC, TO, FROM, TOFROM,  # noqa: F401
                  seeds, make_descriptors, param_count, he_init, glorot_init, sample_rows,
                  sample_kernels, noise, make_config, calibration_rows, agreement_kernels,
                  inputs_digest)
