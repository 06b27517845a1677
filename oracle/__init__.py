"""FP64 CPU oracle for the regularised spiral-MRI reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it;
the product library never calls it and shares no code with it (the only
common module is the seeded input generator ``synthetic``, which holds no
method arithmetic).

Everything here is numpy float64 / complex128, written from the paper's
equations:

* ``nudft``     forward model (Section 2, Eq. ModDirect) and its adjoint, the
                "DFT of the data" D (Eq. AnnMatGD).
* ``gram``      the trajectory-only matrix G (Eq. DG / Eq. AnnMatG), the lag
                kernel of the Gram operator and its circulant spectrum.
* ``toeplitz``  the Gram operator A^H A applied by zero-padded FFT
                (Section 3.4 rewriting) and as an explicit dense matrix.
* ``penalty``   first-order differences and the edge-preserving penalty
                (Section 3.3: Omega_1, Omega_0, Huber; hyperbolic variant).
* ``criterion`` the criterion J and its gradient (Appendix A, B).
* ``solver``    the pseudo-conjugate-gradient minimisation with a
                Polak-Ribiere correction (Section 3.3) and the dense closed
                form for the quadratic penalty.

Pins: every function is checked in tests/test_oracle_*.py against facts the
paper and the mathematics fix (adjoint identity, full Cartesian grid = 2D DFT,
dense Gram matrix, criterion rewriting identity, closed-form Dirichlet
spectrum, finite differences, dense closed-form solve, monotone criterion,
uniqueness, an independent quasi-Newton minimiser).  Nothing is "parity
unpinned".
"""
from . import nudft, gram, toeplitz, penalty, criterion, solver  # noqa: F401
from .nudft import forward, adjoint, adjoint_at, dense_matrix  # noqa: F401
from .gram import lag_kernel, lag_at, paper_G, khat, khat_at  # noqa: F401
from .toeplitz import apply_gram, dense_gram  # noqa: F401
from .solver import solve, solve_quadratic_dense  # noqa: F401
