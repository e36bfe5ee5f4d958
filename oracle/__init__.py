"""CPU oracle for the sigma-mapped GLL spectral-element pressure-Poisson solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (``paper_2411_14977_amd``) never imports, links or executes it, and
this package never imports the product path.  Both sides may read the seeded
input generators in ``workloads/``, which hold none of the method's arithmetic.

Everything here is plain, slow and FP64 (NumPy / SciPy), written from the paper
(Melander, Laskowski, Sherwin, Engsig-Karup, "A p-multigrid accelerated nodal
spectral element method for free-surface incompressible Navier-Stokes model of
nonlinear water waves"):

* ``gll``      -- orthonormal Legendre recurrence, GLL nodes/weights, Vandermonde,
                  differentiation matrix, p-transfer matrix (Sec. 4.3 "Element
                  construction in 2D"; Sec. 5.2 "Transfer operators").
* ``mesh``     -- sigma-transformed element geometry (Sec. 2.2 eq. sigtrans and the
                  sigma-derivative formulas eq. 1_Scoef) and geometric factors.
* ``assemble`` -- element stiffness/mass, global assembly as a sum of local element
                  matrices (Sec. 4.2 eqs. fglobal, flocal, globallocal), right-hand
                  side, Dirichlet lifting, direct solve.
* ``pmg``      -- p-multigrid hierarchy (Sec. 5.1 eq. gridcoars, read as
                  ceil(P/2)), prolongation/restriction (Sec. 5.2), smoothers,
                  V-cycle (Sec. 5), outer flexible CG and defect correction
                  (Sec. 5.4).
* ``precision``-- rounding to FP32 / BF16 (the storage precisions of the inner V-cycle's
                  geometric factors and of the network's GEMM operands).
* ``mlp``      -- the element-local network used as a learned smoothing stage
                  (not in the paper; defined by its formulas only) and the
                  additive-Schwarz element solve it is checked against (Sec. 5.3).
"""
