"""CPU FP64 oracle for the energy-stable hydrodynamic CDFT/PFC scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check the HIP library against
a plain, slow, obviously correct NumPy transcription of the paper
(Baskaran, Guan & Lowengrub, "Energy stable multigrid method for local and
non-local hydrodynamic models for freezing", arXiv 1503.07416).

It shares no code with the HIP path.  Every function cites the passage of the
paper it follows (section, equation label, appendix).  Modules:

``grid``      discrete operators, inner products and norms (App. E)
``models``    discrete PFC and CDFT free energies and their convex splittings
              (Sec. 5.2, 5.3; Lemmas CDFT_ineq / PFC_ineq)
``kernel``    the CDFT convolution kernel J, its split J = J_c - J_e, the
              h^2-weighted periodic convolution (Eq. discrete_convolution,
              Sec. 6) by direct sum and by DFT
``scheme``    the fully discrete scheme, Eqs. discrete_a-d, written in vector
              form with the App. E operators
``system``    the same scheme as the nonlinear system N(g) = S of App. G
              (with the printed typos corrected from Eqs. discrete_a-d)
``smoother``  damped point-block nonlinear Gauss-Seidel (App. G, damping of
              App. G "Damped Gauss-Seidel Iteration"), red-black ordered
``fas``       FAS multigrid V-cycle and the time stepper (Sec. 6, App. G)
``newton``    dense Newton on the system N(g) = S for tiny grids: the plain
              definition of the implicit step's solution
``linear``    closed forms of the linearised scheme (growth of small Fourier
              modes about a uniform state, viscous shear decay)
``gradflow``  the gradient-flow variant of the convex-splitting scheme
              (Thm. thm_grad, Eq. gradient_scheme): its rows, block smoother,
              FAS solver and stepper
``walls``     the PFC step in a channel (Sec. 6, sheared-nanocrystal run): no-slip
              moving walls and no-flux density in y, periodic in x
``three_d``   the PFC step in three dimensions (the extension Sec. 3 calls
              straightforward): 7-point operators, vector vorticity, 3x3
              velocity block

Pins (see tests/test_oracle_*.py): Fourier symbols and summation by parts of
the operators; two transcriptions of the scheme agree; FAS equals dense Newton;
discrete mass conservation and the discrete energy identity of App. F;
convex-splitting gap >= 0; energy non-increase for s in 1e-3..1e3; closed-form
linear growth and shear decay; uniform fixed points; symmetry equivariance;
FFT convolution equals the direct sum; the Cauchy errors the paper prints in
its convergence tables (tests/golden/); for the gradient-flow variant the
scheme written directly with dF_c, dF_e, dense Newton, the closed-form
amplification of a Fourier mode, mass, the dissipation identity and energy
decay for any s (tests/test_oracle_gradflow.py); for the channel dense Newton,
the Couette steady state and start-up, mirror symmetry, energy decay with
resting walls and the transfers on linear fields (tests/test_oracle_walls.py);
for 3D the reduction to the 2D oracle for z-independent states, axis-rotation
equivariance, dense Newton, closed-form linear growth, energy and mass for any
s, the transfers on linear fields (tests/test_oracle_three_d.py).
"""
