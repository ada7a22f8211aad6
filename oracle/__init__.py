"""CPU oracle for the tree-cotree-gauged time-domain eddy-current solve.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code, tables or helpers with the HIP
library.

What it computes (plain definitions, FP64 throughout):

* ``spline``   -- open-knot B-splines, D-splines, Gauss-Legendre (Sec. 2.2).
* ``grid``     -- the global control grid of a multi-patch box, edge numbering
                  and edge classes (wirebasket / face / interior).
* ``assemble`` -- element-loop quadrature of the conductivity-weighted mass
                  matrix, the curl-curl stiffness, the curl-form or volume
                  source load (Sec. 2.2, matrices K_i, M_C, j_i) and the
                  initial-value load int sigma A(x,0) . w (Sec. 2.1).
* ``gauge``    -- Dirichlet set, the tree-cotree gauge of the insulating
                  region and the primal / dual / interior split with the
                  multiplier table (Sec. 3).
* ``solve``    -- implicit Euler (Sec. 2.2, implicit Euler system) on the
                  globally assembled gauged system with a sparse direct
                  factorisation; the FETI-DP field must equal this.
* ``errors``   -- L2 errors of B_h = curl A_h and of E_h = -dA_h/dt in the
                  conductor against a closed-form solution (Sec. 4).
"""
