"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package only *describes* workloads: theory programs as plain data, the
time grids, true parameter vectors, start vectors, and the random draws that
turn a vector of expected counts into Poisson counts.  It holds none of the
method's arithmetic: the expected counts (the histogram model of Eq. 1) are
computed by a caller-supplied function, so a test passes the oracle's model
and the GPU benchmark passes the library's own model evaluation.
"""

from .recipes import (  # noqa: F401
    TAU_MU,
    ref_p,
    ref_f,
    ref_lit,
    theory_exp_cos,
    theory_gauss_cos,
    theory_stg,
    theory_exp_gkt,
    theory_c2,
    theory_paper_eq4,
    config_c1,
    config_c2,
    config_c2_large,
    config_c3,
    config_c4,
    config_c5_ranges,
    config_paper_shape,
    config_multi_run,
    draw_counts,
    materialise,
    rng_for,
)
