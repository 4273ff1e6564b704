"""Plain CPU oracle of the inexact-subdomain Schwarz method (test infrastructure only).

This package is the correctness reference for the HIP library: a slow, direct,
complex128 implementation written from the paper (Bootland, Dwarka, Jolivet,
Dolean, Vuik, "Inexact subdomain solves using deflated GMRES for Helmholtz
problems", arXiv:2103.17081).  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP path; both receive the same seeded inputs.

Modules
-------
fem        P1 assembly of -Delta u - k^2 u = f on (0,1)^2 with u = 0 on the boundary
           (Sec. 2, eqs. 1-2), and of the local subdomain matrices: the Dirichlet
           restrictions R_j A R_j^T of eq. 3 and the impedance (Robin) variant.
partition  Cartesian overlapping subdomains, restriction index sets and the Boolean
           partition of unity D_j (Sec. 2, eq. 3; Sec. 3).
deflation  Deflation matrices Z_j (linear interpolation or the quadratic Bezier
           stencil of Sec. 2), the 2D Kronecker form (eq. 5), E_j, Q_j, P_j (eq. 4).
krylov     GMRES with modified Gram-Schmidt and Givens rotations; right-flexible
           FGMRES (Sec. 3).
schwarz    Restricted additive Schwarz preconditioner (eq. 3) with direct or
           deflated-GMRES subdomain solves, and the outer FGMRES driver.
coarse_space  Two-level variant (the step after the one-level method, Sec. 4): a global
           coarse space of piecewise-linear hats on a coarse grid of fine-grid lines,
           E_0 = Z_0^T A Z_0, and the deflation-type combination with eq. 3.
ilu        ILU(0) factorisation and ILU(0)-preconditioned GMRES local solves, the
           comparison of Sec. 3, Table 5.
cnn        float64 reference of the learned-initial-guess network (forward and
           backward), checked against finite differences.

Every floating-point quantity is complex128 (or float64).
"""
