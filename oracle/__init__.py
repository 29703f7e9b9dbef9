"""Plain, slow FP64 CPU oracle for phase-insensitive detector tomography.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and this package
never imports the product path; the two share no code.

What it computes (arXiv 2404.02844):

* ``poisson``   -- the coherent-probe matrix F (Eq. Fmatrix) from an accurate Poisson
                   pmf, its band above a threshold, and the tail-lumped variant.
* ``objective`` -- f(Pi) = ||F Pi - P||^2 + gamma * sum (Pi_{i,n} - Pi_{i+1,n})^2
                   (Eq. min_obj2 plus Eq. regul) and its gradient.
* ``simplex``   -- the Euclidean projection onto the probability simplex and its
                   row-wise M-fold version (Eq. Mp1_proj), sort-based and brute force.
* ``fista``     -- the largest Hessian eigenvalue by power iteration and the
                   accelerated projected-gradient iteration with function restart.
* ``certify``   -- the KKT residual of App. B (with the row multipliers), the
                   Frank-Wolfe gap, an active-set polish to the exact optimum on small
                   problems, and the POVM fidelity of Eq. fidelities.
* ``mlp``       -- FP64 forward/backward of the warm-start network and its input
                   resampling.
* ``newton``    -- the paper's two-stage two-metric projected truncated Newton method
                   (App. B, Algorithms 1-3).
* ``smoothing`` -- the long-range average of Eq. smoothing used before the paper's
                   stage-2-only second run.

Every reduction is FP64.  Functions cite the passage they follow.
"""
