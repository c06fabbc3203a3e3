"""Plain CPU FP64 oracle for the multi-resolution approximation (M-RA).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP path.

It follows Katzfuss, "A multi-resolution approximation for massive spatial
datasets" (JASA 2017, arXiv 1507.04789), in the paper's own notation:

  geometry.py    recursive partition and knots (Sec. 2.2, Sec. 2.5)
  covariance.py  C_0 = sigma^2 rho(||s - s'|| / kappa): Matern nu = 1.5
                 (eq. mat15) and exponential, with d/d log(kappa)
  mra.py         prior quantities W^l (eq. priorw), leaf quantities
                 (eq. helpquantities at m = M), the posterior recursion
                 (eq. posterior, mainquantities, helpquantities), the
                 log-likelihood d/u recursions (Sec. 3.3) and a forward-mode
                 (tangent) gradient of all of it
  predict.py     posterior predictive mean and variance (Sec. 3.4, Prop. 2),
                 the data gradient d loglik / d z = -Sigma^{-1} z from
                 the kriging residual at the observed locations, and the
                 generalised least-squares trend with its profile likelihood
  dense.py       brute-force n x n M-RA covariance from the closed form of
                 Sec. 2.4 ("Quality of the covariance approximation"), dense
                 likelihood, gradient and kriging; exact Gaussian process

Every function is pinned by tests that check it against something other
than itself (special cases, closed forms, brute force, finite differences).
"""
