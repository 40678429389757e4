"""Plain FP64 CPU oracle for the Gaussian log-likelihood path — TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library and is never on
the product path.

What it computes follows the paper directly:
  * Matérn covariance, eq. (1), Section IV-B;
  * Gaussian log-likelihood, eq. (2), Section IV-C;
  * Cholesky factor with positive diagonal, Section V-A;
  * simple-kriging prediction, Section VIII-D (implied by the PMSE experiment);
  * a Morton (Z-order) location ordering for the "appropriate ordering" of
    Section VI;
  * a Nelder-Mead maximiser of eq. (2) (the paper uses a derivative-free
    optimiser with 1e-3 tolerance, Section VIII-A);
  * the profile likelihood in (theta2, theta3), eq. (2) at its maximising variance
    (Section IV-C).
The method's mixed-precision factor approximates the exact result, so the
oracle is the exact FP64 definition; library primitives (LAPACK Cholesky and
triangular solve via numpy/scipy, scipy's modified Bessel K) serve as steps.
"""
from .matern import matern, matern_matrix, distances, cross_distances
from .morton import morton_keys, morton_order
from .likelihood import loglik, loglik_parts, cholesky_lower, simulate_field
from .kriging import krige
from .mle import nelder_mead, fit_mle
from .profile import profile_loglik, fit_mle_profile

__all__ = [
    "matern", "matern_matrix", "distances", "cross_distances",
    "morton_keys", "morton_order",
    "loglik", "loglik_parts", "cholesky_lower", "simulate_field",
    "krige", "nelder_mead", "fit_mle", "profile_loglik", "fit_mle_profile",
]
