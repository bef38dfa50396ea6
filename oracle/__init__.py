"""Plain FP64 CPU oracle for the helical-wave Hamiltonian (test infrastructure).

This package is test infrastructure only.  It may be imported by the tests,
by the smoke check of the package entry point and by the CPU-baseline leg of
the benchmark, and by nothing else: the GPU library never calls it and shares
no code with it.

It is written straight from the paper (Agarwal & Banerjee, "Solution of the
Schroedinger equation for quasi-one-dimensional materials using helical
waves", arXiv 2210.12252) in NumPy/SciPy double precision, favouring
transparency over speed:

* ``basis``      -- Bessel zeros, the cutoff-masked index set (Sec. 3.2,
                    eq. Energy_cutoff), the kinetic diagonal (eqs.
                    Laplacian_of_f_mnk and constants_abc, Alg. 5), the
                    Fourier x Gauss-Jacobi grid (Sec. 3.1) and the radial
                    functions xi_{n,k}(r) (App. B, eq. Basis_fun_derived).
* ``transforms`` -- the naive inverse transform (eq. Naive_Inverse_Transform)
                    and the quadrature forward transform (eq.
                    Fast_fwd_transform_cont), both as an explicit basis
                    matrix and as the separated sums of Sec. 3.4 evaluated
                    with explicit exponential matrices (no FFT).
* ``hamiltonian``-- the discrete operator H = kinetic diagonal + forward(V *
                    inverse(.)) (eqs. Simplify_2 and g_mnk, Alg. 5 at nu = 0)
                    as a dense matrix built two independent ways (the second
                    also one pair of angular modes at a time, for mid-size
                    bases), as a matrix-free apply, and its lowest eigenpairs
                    by LAPACK.
* ``precond``    -- the Teter-Payne-Allan diagonal preconditioner (Sec. 3.5).
* ``density``    -- the electron density sum_j occ_j |phi_j|^2 on the grid
                    (Sec. 4.2, the density equation, one (eta, nu) term).
* ``gradient``   -- derivatives of a field given by coefficients in helical
                    and Cartesian coordinates (App. C).
* ``mlp``        -- forward and backward pass of the small per-coefficient
                    network used as a learned preconditioner and its Adam
                    step (no paper source; it exists to check the GPU
                    kernels' gradients and updates).

Every function that is not pinned by a test against something other than
itself says "parity unpinned" in its docstring.
"""
