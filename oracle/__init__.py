"""FP64 CPU oracle for parallel cross-validation of Gaussian-process models.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  The oracle shares no code with the HIP library; the
only module both sides consume is the seeded input generator, which holds none
of the method's arithmetic.

Every function follows the definitions of Gerber & Nychka, "Parallel
cross-validation: a scalable fitting method for Gaussian process models"
(arXiv:1912.13132), and cites the section / equation it writes out.
"""
from .pcv_oracle import (  # noqa: F401
    COV_EXP,
    COV_MATERN32,
    covariance,
    pairwise_distance,
    subset_cv,
    cv_loss,
    route_queries,
    predict,
    predict_problem,
    neg2_loglik_subset,
    gls_beta_subset,
)
from .mp_oracle import mp_subset_cv, mp_predict  # noqa: F401
from . import pcv_division as division  # noqa: F401
