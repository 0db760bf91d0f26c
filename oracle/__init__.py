"""Plain FP64 CPU oracle for the Wilson-Dirac / domain-decomposition hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product library imports, links or
runs this package; only the test-suite, the smoke check and the CPU baseline
leg of the benchmark do. It is deliberately slow and literal: every operator
is written as the definition in the paper (numpy array operations, scipy
sparse/dense LU and plain CG/GMRES loops as library steps), with no blocking,
fusion or reordering beyond what the definition states.

Modules
-------
lattice    geometry: coordinates, blocks, colours, the Schur projector P.
dirac      the Wilson-Dirac operator D = 1 - kappa H (eq. Dw, Sec. 5),
           matrix-free and as a sparse matrix; gamma matrices.
schur      block operators (eq. domdec), Q, 1 - PQ (eq. detschur) and its
           inverse (eq. inverseschur), dim(P) (eq. dimproj).
solvers    dense / sparse LU and CG on the normal equations.
estimator  the stochastic estimator Delta = |M xi|^2 - |xi|^2 (eq. stacc,
           eq. Deltaistoch) for the full and the Schur-complement ratio.
network    FP64 forward and analytic backward of the gauge-covariant linear
           network used as a preconditioner (not from the paper).
"""
