"""FP64 CPU oracle for the Sternheimer polarizability / Lanczos dielectric path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library never
calls it, and it shares no code, table or constant with the HIP library: both
sides consume only the seeded inputs of the ``synthetic`` package.

Contents (each function cites the passage of the paper it follows):

* ``pw``          - the discrete plane-wave problem: sphere, Gather/Scatter,
                    Hamiltonian, truncated Coulomb square root.
* ``sos``         - O1: chi0 as the explicit Adler-Wiser sum over all
                    conduction states of the dense Hamiltonian (Sec. II).
* ``sternheimer`` - the same chi0 through the Sternheimer equations of
                    Sec. III.A, solved densely (O1 cross-check) or matrix-free
                    with SciPy Krylov solvers (O2, for grids too big to
                    diagonalise).
* ``lanczos``     - Lanczos with full Gram-Schmidt reorthogonalisation on
                    eps - 1 (Sec. IV) and the projection of eps(z) - 1 on the
                    static basis (Sec. VI).
* ``lindhard``    - closed-form chi0 of the free-electron box (V = 0), used to
                    pin the oracle.
* ``sigma``       - the correlation self-energy pieces in the dielectric basis:
                    the integrand traces sigma_N, sigma_N0 and the Lorentzian
                    model term Sigma_A (Secs. II, III.B, IV) as sums over
                    states and as traces with H inverted by linear solves,
                    and the residue term Sigma_P from a real-frequency Lanczos
                    recursion per pole (Sec. VI).

Parity status: every function here is pinned by a test in tests/ against a
closed form, an invariant or brute force; none is "parity unpinned".
"""
