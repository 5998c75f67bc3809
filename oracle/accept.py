"""Well-posedness check of a (sigma, rho) draw through the oracle's own
lambda solve (eq:N14-N16): True when the mixing matrix exists and is SPD.
TEST INFRASTRUCTURE ONLY."""
import numpy as np

from . import OracleSim, OracleError


def oracle_accepts(sigma, rho):
    N = len(rho)
    try:
        OracleSim(N, 4, 4, sigma, rho, np.ones(N))
    except OracleError:
        return False
    return True
