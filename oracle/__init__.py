"""FP64 CPU oracle of the SEM Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY: this package is the independent reference that the
GPU library is checked against.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does.
It shares no code with the HIP path.

Every function is plain double-precision arithmetic in the order the
mathematics is stated (textbook SEM on GLL points; the paper's Fig. 3 step
ordering, Sec. 3 problem definition and the error metrics of Sec. 4.2).
"""
from .oracle import (  # noqa: F401
    build_oracle, OracleMesh, OracleFluid, OracleProjection, OracleHSMG, gll, gl, lxd, interp_matrix, deriv_matrix, num_threads,
    bdf_ext_var,
)
from .metrics import (  # noqa: F401
    e_series, e_max, e_peak,
)
