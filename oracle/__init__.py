"""CPU FP64 oracle for the Krylov-space Green's-function method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It is deliberately plain, slow and readable: NumPy/SciPy in
float64 / complex128, each function following the passage of the paper
(Balzer, Gdaniec & Potthoff, "Krylov-space approach to the equilibrium and
the nonequilibrium single-particle Green's function") that defines it.

Modules
    basis        occupation-number basis of a fixed (N_up, N_dn) sector
    hamiltonian  hopping / interaction operators, H.v, c and c^+
    lanczos      Lanczos recursion (Eq. recursion), tridiagonal T (Eq.
                 tmatrix), ground state (Sec. 2)
    propagate    short-iterative-Lanczos step (Eqs. newstate, udelta)
    greens       equilibrium G (Eq. psigreen) and the four-step
                 nonequilibrium G^<, G^>, Matsubara and mixed components
                 (Sec. 4)
    gradients    dense exact gradients (Frechet derivative of exp, ground-state
                 perturbation): the reference for the adjoint
    spectral     equilibrium spectra: conventional Lanczos G(omega) (Eq. gapprox),
                 time-dependent Lanczos G(t) on a fine grid, damped transform
    driven       driven H(t) = sum_j f_j(t) H_j by the fourth-order
                 commutator-free exponential integrator (Sec. 6 outlook)
    greens2      a four-time two-particle Green's function
                 <c+_a(t1) c+_b(t2) c_c(t3) c_d(t4)> by dense propagation of
                 two-time states (Sec. 6 outlook: higher-order functions)
    necpt        nonequilibrium cluster-perturbation theory: the CPT equation
                 (Eq. cpteq) on the discretised Keldysh contour, bath functions
                 (Eqs. gb1, gb2), free-fermion references for U = 0
    exact        dense references: Jordan-Wigner Fock-space operators,
                 full diagonalisation, matrix exponentials and the U=0
                 closed form used to pin the above
"""
from . import basis, hamiltonian, lanczos, propagate, greens, exact  # noqa: F401
