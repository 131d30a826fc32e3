"""Plain, slow, FP64 CPU oracle for the muSR chi^2 / Poisson-likelihood path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything here; only the tests, the entry point's smoke check and the
benchmark's CPU-baseline leg do.  The oracle shares no code with the HIP
path: it reads the same plain-data theory programs and seeded inputs and
evaluates them with its own numpy / math code, following the paper's
definitions:

* Eq. 1   histogram model N(t) = N0 e^(-t/tau) [1 + A(t)] + Nbkg, t = n dt
* Eq. 2   chi^2 with d_err^2 = d (and 1 for empty bins, a stated reading)
* Eq. 3   Poisson log-likelihood ratio, minimised (a stated reading)
* Listing 2  predefined primitives se, ge, sg, stg (real 1/3 and 2/3)
* Listing 3  parameter / function / map indirection; tf = cos(2 pi nu t + phi)

Modules: ``model`` (cost and analytic gradient), ``scalar`` (pure-Python
cross-check for tiny inputs), ``fit`` (reference minimiser), ``errors``
(Gauss-Newton Hessian, covariance, likelihood profiles and their
one-standard-deviation crossings), ``expr`` (user-defined asymmetry
expressions, the run-time compiled theories' language, with symbolic
derivatives), ``seeder``
(reference network with BF16 rounding), ``philox`` (counter-based generator
from its published definition; the seeder's parameter draws and expected
rebinned counts live in ``seeder``).

Every function states the passage it follows.  Pins that tie each function to
something other than itself live in ``tests/test_oracle_*.py``.
"""
