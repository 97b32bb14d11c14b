"""Plain FP64 CPU oracle for the p-multilevel preconditioned, statically condensed
HHO-dp Stokes solver of Botti & Di Pietro (arXiv 2009.13840).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke entry point and the benchmark's CPU-baseline leg do.  It shares
no code with the GPU library: the only common inputs are the seeded meshes and
fields of the ``synth`` package, which hold none of the method's arithmetic.

Modules, each written from the paper's definitions:

* ``geometry``   -- cell/face measures, centroids, diameters, outward normals (Sec. 2.1)
* ``quadrature`` -- Gauss rules on segments, triangles (collapsed), polygons, boxes
* ``bases``      -- hierarchical L2-orthonormal bases on cells and faces (Sec. 4.2)
* ``hho``        -- potential reconstruction, face residuals, HHO-dp local residuals
                    in matrix form (Sec. 2.2, 2.3.1, eq. def:HHOAB)
* ``hho_hp``     -- the HHO-hp scheme (cell velocity of degree k+1, hybrid
                    pressure; Sec. 2.3.2): local residuals, global system, v&p-cond
* ``condense``   -- v-cond and v&p-cond Schur complements (eqs. ST.1, ST.2)
* ``system``     -- global assembly, DOF/MNZ counts (Table tab:DOFsMNZsFormula),
                    level hierarchy by Galerkin projection (Sec. 3.1-3.2, 4.2)
* ``krylov``     -- GMRES smoother and flexible GMRES (Sec. 3.3)
* ``multilevel`` -- cell-patch Schwarz preconditioner and the V-cycle (Sec. 3.3)
* ``ilu``        -- zero-fill ILU, the paper's smoother preconditioner (Sec. 3.3, 5.2)
* ``solve``      -- end-to-end driver and error norms (Sec. 5.2)
* ``mlp``        -- reference network for the learned smoother (not in the paper)

Parity pins for every module live in ``tests/test_oracle_*.py``.
"""
