"""Plain FP64 CPU oracle for the synthetic iterative scheme (SIS) of
Wu, Zhang, Liu, Zhang & Reese, "A fast iterative scheme for the linearized
Boltzmann equation" (arXiv:1612.04488).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is written from the paper's equations in the paper's order, with
NumPy/SciPy primitives (FFT, sparse solve, eigenvalues) as single steps and no
blocking, fusion or reordering beyond what the equations state.  Where the
paper is silent (the fast spectral method is only cited) the reading taken is
stated in each function's docstring.

Modules
-------
velocity   discrete velocity grid, equilibrium, sources           (Sec. 2)
collision  fast-spectral linearized collision operator L = L+ - nu h
           (eq. LBE_collision, Sec. 2; FSM reading in the docstrings)
direct     slow non-FFT references for the collision operator (mode sum,
           sigma-representation quadrature) used only to pin `collision`
transport  1-D/2-D spatial grids, upwind sweeps, moments, flow rates
           (eqs. LBE_iteration, syn_LBE, first_order, diffusion_LBE)
solver     CIS / SIS outer iterations (Sec. 2.2, eq. guided)
modes      Fourier-mode convergence analysis (Sec. 2.3)
mixture    binary-mixture operator and SIS (Sec. 5)
"""
