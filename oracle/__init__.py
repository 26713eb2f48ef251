"""Plain FP64 CPU oracle for the BB energy minimiser of finite-difference micromagnetics.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct reference
against which the HIP library is checked.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path (the
HIP library and its Python binding) never does, and this package imports
nothing from the product.

Contents, following Abert et al., "Efficient Energyminimization in
Finite-Difference Micromagnetics" (arXiv:1405.2728):

* ``newell``    -- cell-averaged demagnetisation tensor of a cuboid grid
                   (Sec. 3: the demag field is an FFT-accelerated convolution on
                   a regular cuboid grid; the tensor itself follows Newell,
                   Williams and Dunlop, JGR 98 (1993)).
* ``fields``    -- demag / exchange / anisotropy / Zeeman fields, the effective
                   field of eq. (5) and the energy U(m) of Sec. 2.
* ``minimizer`` -- the midpoint (Cayley) projected-gradient step of eq. (7),
                   the Barzilai-Borwein step sizes of eq. (12) used alternately,
                   the torque stop rule and the warm-started hysteresis sweep of
                   Sec. 4.
* ``adjoint``   -- derivatives of U (for automatic differentiation), the
                   Riemannian Hessian on the product of unit spheres, conjugate
                   gradients for the adjoint field of a relaxed state and the
                   implicit parameter gradients (calculus on the energy of Sec. 2;
                   not in the paper).

Every function states the passage it follows.  Readings of passages that are
garbled or silent in the paper are listed in each module's docstring.
"""


