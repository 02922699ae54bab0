"""Constants printed in the paper (Appendix B, Tables computedTrace and markovConsts).

The stable time step uses the computed trace constants C_T(N) of the GL
formulation (Section 3.4 chooses these over the analytic constants).  The
oracle's own generalised-eigenvalue computation of the same constants is
checked against these printed values in the tests.
"""
from __future__ import annotations

HEX, WEDGE, PYR, TET = 0, 1, 2, 3

# Appendix B, Table computedTrace: C_T(N), N = 1..9, full mass matrix.
COMPUTED_TRACE = {
    HEX: [9, 18, 30, 45, 63, 84, 108, 135, 165],
    WEDGE: [9.93, 18.56, 29.03, 42.99, 58.80, 78.01, 99.27, 123.76, 150.48],
    PYR: [11.68, 20.89, 32.84, 47.59, 65.17, 85.60, 108.90, 135.07, 164.11],
    TET: [12.22, 20.46, 29.18, 41.65, 54.45, 71.10, 88.32, 109.04, 130.67],
}

# Appendix B, Table computedTraceSEM: C_SEM(N), N = 1..9 (tets identical to the GL table).
COMPUTED_TRACE_SEM = {
    HEX: [3, 9, 18, 30, 45, 63, 84, 108, 135],
    WEDGE: [46.46, 51.70, 63.94, 83.32, 104.76, 132.20, 161.22, 195.95, 232.52],
    PYR: [31.58, 37.12, 47.59, 60.95, 77.14, 96.31, 118.52, 143.80, 172.13],
}

# Appendix B, Table markovConsts: C_M(N), N = 1..9.
MARKOV = {
    HEX: [3.00, 18.00, 55.73, 137.51, 293.97, 562.17, 985.92, 1616.24, 2511.47],
    WEDGE: [12.00, 54.27, 142.63, 308.34, 585.89, 1021.64, 1663.85, 2574.06, 3814.56],
    PYR: [12.92, 60.05, 175.51, 405.43, 809.95, 1460.93, 2442.26, 3849.94, 5792.11],
    TET: [20.00, 78.62, 195.58, 403.91, 744.85, 1265.54, 2021.09, 3073.26, 4491.62],
}

# Section 3.4, Table bounds: spectral radius of M^{-1}A and its bounds on the
# paper's (unavailable) hybrid mesh, N = 1..4; only the ordering is checkable.
BOUNDS_TABLE = {
    "rho(M^-1 A)": [10.89, 18.66, 28.18, 41.09],
    "rho(M^-1 A^s)": [11.26, 19.30, 29.05, 42.86],
    "computed C_T(N,K)": [12.22, 20.84, 32.76, 47.47],
    "computed C_T(N)": [17.24, 29.47, 46.32, 67.13],
    "analytic C_T(N)": [38.53, 74.73, 124.54, 186.81],
}


def trace_constant(etype: int, N: int) -> float:
    """Computed C_T(N) of the GL formulation, 1 <= N <= 9."""
    if not 1 <= N <= 9:
        raise ValueError("C_T(N) is tabulated for 1 <= N <= 9")
    return float(COMPUTED_TRACE[etype][N - 1])
