"""FP64 CPU oracle for split-ETD3 (exprk3ds_real).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it.  The GPU library never calls
it, and it shares no code, tables or constants with the HIP sources: the
splitting coefficients, the phi-functions, the Tucker operator and the time
step are written here a second time, from the paper, in plain numpy.

Contents
  coeffs  - Table 1 (real, d = 2) and Table 3 (d > 2) closed forms, "+" set
  phi     - phi_0..phi_p of small matrices: exact spectral form (long double)
            for multiples of the Neumann pattern, augmented-matrix exponential
            otherwise
  tensor  - mu-mode product, Tucker operator, Kronecker-sum action (Section 2)
  etd     - reaction terms, phi bank, split phi action, eq. (exprk3) step
  adjoint - discrete adjoint of the step (vector-Jacobian product), loss
            gradients with respect to U0, reaction parameters and diffusion
            scale (import as oracle.adjoint)

Every function is pinned by tests/test_oracle_*.py against facts fixed by the
paper or by mathematics (closed forms, brute-force Kronecker products, exact
special cases, observed convergence orders); see those tests for the list.
"""
from .coeffs import split_coefficients, table1_real, table3_real
from .etd import (BANK_ENTRIES, G_FHN, G_NONE, G_SCHNAKENBERG, STAGE_SCALE, PhiBank, etd_step, integrate,
                  make_banks, reaction, split2_apply, Phi2Bank, etd2rkds_step, integrate_etd2rkds)
from .phi import phi, phi_all
from .tensor import kron_sum_action, mode_product, tucker

__all__ = [
    "split_coefficients", "table1_real", "table3_real", "BANK_ENTRIES", "G_FHN", "G_NONE", "G_SCHNAKENBERG",
    "STAGE_SCALE", "PhiBank", "etd_step", "integrate", "make_banks", "reaction", "split2_apply",
    "Phi2Bank", "etd2rkds_step", "integrate_etd2rkds",
    "phi", "phi_all", "kron_sum_action", "mode_product", "tucker",
]
