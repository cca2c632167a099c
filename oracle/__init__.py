"""CPU oracle for the Sakurai-Sugiura complex-band-structure path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU path: the only
common module is ``workloads`` (seeded input arrays, no method arithmetic).

Everything here is plain, slow and complex128:
  * ``fd``      finite-difference weights from the exact Taylor system
  * ``ham``     the cell blocks H0, H+, H- = H+^T of the real-space Kohn-Sham
                Hamiltonian (paper Sec. 2, Eqs. 2-4), dense and sparse
  * ``qep``     the quadratic eigenvalue problem solved densely through a
                companion linearisation (QZ), the free-electron closed form,
                pairing / residual / H(k) checks (Eq. 5 selects the annulus),
                and k of a Bloch factor lambda = exp(i k a) (Sec. 2)
  * ``ss``      the Sakurai-Sugiura steps in the paper's order (Sec. 3.1,
                Algorithm 1; ring contour of Sec. 3.2) with dense solves,
                the Rayleigh-Ritz variant, a plain BiCG with its dual (and its
                residual history), and the iteration at which the
                load-balancing rule of Sec. 3.3 stops every solve
  * ``adjoint`` eigenvalue derivatives from left/right eigenvectors

Readings of the paper that the oracle fixes (each is listed in the design
notes as well):
  * P(z) = (H0 - E) + z H+ + z^-1 H-  (the negative of Eq. 4; same roots)
  * trapezoid weights w_j = z_j / N_int on each circle (the printed weight
    drops the radius; see ``ss.quadrature``)
  * SVD rank threshold relative to the largest singular value
"""
