"""FP64 CPU oracle for the tensor-product nodal DG Vlasov-Poisson method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library (no kernels,
headers, tables or helpers); both sides receive the same seeded inputs from
``paper_2202_13532_amd.inputs``, which holds no arithmetic of the method.

Every routine is a plain, slow, obviously-correct NumPy transcription of the
paper's definitions, in float64:

* ``lgl``        -- LGL nodes/weights, Lagrange derivative matrix, the LGL
                    mass-matrix inverse, stiffness, Upsilon, Xi (Sec. 5.2).
* ``grid``       -- element geometry and node coordinates (Sec. 2, Sec. 5.3).
* ``rhs``        -- weak-form semi-discrete right-hand side with upwind faces
                    (eq. weak, eq. decoupled, eq. numerical_flux, App. A).
* ``poisson``    -- LGL->Fourier connection tensor by brute-force quadrature,
                    spectral Poisson solve for Phi and E (Sec. 5.3.2).
* ``rk``         -- Shu-Osher SSP-RK3 with Poisson at every stage (Sec. 6).
* ``diagnostics``-- mass, field energy and other moments.
* ``cfl``        -- RK3 + upwind DG stability limit from the Bloch symbol.
* ``mlp``        -- FP64 MLP forward/backward used to check the learned
                    correction's gradients.
* ``projection`` -- L2 projection between DG grids (fine -> coarse).
* ``harris``     -- Harris dispersion function of the loss-cone ring and its
                    roots (Sec. 4.1), for the paper's case studies.
* ``brute``      -- tiny-grid dense assembly of the weak form by quadrature in
                    all dimensions at once, used only to pin ``rhs``.

Parity status of each function is stated in its module header.
"""
