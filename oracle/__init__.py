"""Plain, slow FP64 / complex128 CPU oracle for the exact-exchange hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's ``cpu_baseline`` leg may import anything from this package.  The
device library never calls it, and it shares no code, tables or helpers with
the device library.

What it computes (arXiv 2501.16572):

* ``fd``    -- central finite-difference weights of the second derivative and
               the 1D second-derivative operators per boundary condition
               (Sec. II: Bloch-periodic along extended directions, Dirichlet
               along vacuum directions).
* ``kron``  -- the solution operator f(L) of Eq. (fL), the 1D
               eigendecompositions of Eq. (FinalRepfL), the slice-wise
               Kronecker solve of Sec. II.A and the literal batch Kronecker
               solve of Sec. II.B with its four data reorganizations.
* ``dense`` -- brute force: the assembled 3D Laplacian and a direct solve of
               the discrete (screened) Poisson equation, Eqs. (Poisson) and
               (Poisson:SR).  This is the plain definition the Kronecker forms
               must reproduce.
* ``exx``   -- the exact-exchange application of Eq. (Vx:Poisson) and the
               exchange energy.

Readings taken where the paper is silent or garbled are listed in each
function's docstring.  Every function is pinned by tests under ``tests/``
against closed forms, brute force and invariants, not against itself.
"""

from . import fd, kron, dense, exx  # noqa: F401
