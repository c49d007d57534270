"""FP64 CPU oracle for the CTMRG environment of the rhombic-lattice network.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path; the one module both
sides read is the seeded input generator (which holds no CTMRG arithmetic).

Contents
--------
ctmrg         the method written out step by step in plain NumPy FP64
              (composite and double layer, environment init, enlarged
              corners, projectors from a full LAPACK SVD, absorption,
              sweeps, bond environment, norm per site, expectation values).
closed_forms  independent closed forms used to pin the oracle (Onsager,
              Houtappel's honeycomb Ising free energy, two-site gate algebra).
brute         exact contraction of small finite lattices by a row transfer
              matrix (no truncation), used to pin the move semantics.
gates         two-site gate and its rank-4 split, used to build test inputs.
fu            one full-update bond truncation: gate, environment of the
              gated composite, alternating least squares in its metric.
transfer      the column transfer matrix of the environment, dense, and its
              leading eigenvalues (correlation length).
gradients     directional derivatives of the oracle's objectives (ln kappa,
              <O>) by fourth-order central differences: the reference for
              the hand-written adjoint of the HIP path.
"""
